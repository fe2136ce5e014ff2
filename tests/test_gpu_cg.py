"""GPU parity: GMRESR(relCG) -- the deflated CGNE of Sec. 4 with the spectral
preconditioner and the CG relaxation of Sec. 3, inside Alg. 3 -- and
GMRESR(eigCG) (Sec. 5) against the oracle and dense algebra on a small
lattice."""
import numpy as np
import pytest

import synth
from oracle import krylov
from oracle.lattice import WilsonKernel, norm
from oracle.zolotarev import Zolotarev
from gpu_util import require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu
MU = 0.05


@pytest.fixture(scope="module")
def lat():
    dims = (4, 4, 2, 4)
    U = synth.gauge_field(dims, 8, 0.45)
    k = WilsonKernel(dims, U, 1.4)
    w, Q = np.linalg.eigh(k.dense("K"))
    n = k.V * 12
    G5 = np.kron(np.eye(k.V), np.kron(np.diag([1.0, 1, -1, -1]), np.eye(3)))
    D = 0.5 * (1 + MU) * np.eye(n) + 0.5 * (1 - MU) * G5 @ (Q @ np.diag(np.sign(w)) @ Q.conj().T)
    H = G5 @ D
    h2, E = np.linalg.eigh(H @ H)
    z = Zolotarev(16, np.abs(w).min(), np.abs(w).max())
    sign = krylov.SignFunction(k, z)
    return dict(dims=dims, U=U, D=D, H=H, h2=h2, E=E, z=z, ov=krylov.Overlap(sign, MU), shape=(k.V, 4, 3))


def _ctx(ovl, lat):
    ctx = ovl.Context(lat["dims"])
    ctx.gauge_load(to_dev(lat["U"]))
    z = lat["z"]
    return ctx, ovl.zolo_from(z.nz, z.a, z.b, z.delta, z.omega, z.sigma)


def _params(ovl, mixed, defl):
    """mixed: False (FP64 sign calls), True (FP32 from 1e-6) or "half" (FP16
    storage from 3e-3 asked for, which the CG middle solve declines)."""
    return ovl.solver_defaults(rho=1.4, mu=MU, tol=1e-10, eta_tilde=1e-3, middle_cg=1, use_deflation=defl,
                               f32_threshold=(1e-6 if mixed else 10.0),
                               half_threshold=(3e-3 if mixed == "half" else 2.0), n_eig=16, m_eig=40)


def _space(lat, n, noise, seed):
    """n lowest eigenvectors of H^2 (perturbed by noise, re-orthonormalised),
    V^D = D V, and the Rayleigh-Ritz vectors and values of H^2 in their span
    (what the library builds its preconditioner from)."""
    Ev = lat["E"][:, :n].copy()
    if noise:
        rng = np.random.default_rng(seed)
        Ev = Ev + noise * (rng.normal(size=Ev.shape) + 1j * rng.normal(size=Ev.shape)) / np.sqrt(2 * Ev.shape[0])
        Ev, _ = np.linalg.qr(Ev)
    VD = lat["D"] @ Ev
    m, Y = np.linalg.eigh(VD.conj().T @ VD)
    S = Ev @ Y
    shape = lat["shape"]
    V = np.stack([Ev[:, i].reshape(shape) for i in range(n)])
    VDs = np.stack([VD[:, i].reshape(shape) for i in range(n)])
    pre = krylov.SpectralPreconditioner([S[:, i].reshape(shape) for i in range(n)], m)
    return V, VDs, pre


def _true_res(lat, b, x):
    return norm(b.reshape(-1) - lat["D"] @ x.reshape(-1)) / norm(b)


@pytest.mark.parametrize("mixed", [False, True, "half"])
def test_relcg_solve_vs_dense(lat, mixed):
    """No preconditioner: true residual <= 1e-10 with the dense D, the dense
    LU solution, and CG iteration counts close to the oracle's GMRESR(relCG)."""
    ovl = require_gpu()
    ctx, zg = _ctx(ovl, lat)
    b = synth.z2_source(lat["dims"], 90)
    x, st, code = ctx.solve(to_dev(b), zg, _params(ovl, mixed, 0))
    assert code == 0
    x = to_host(x)
    assert _true_res(lat, b, x) <= 1e-10
    xd = np.linalg.solve(lat["D"], b.reshape(-1))
    assert norm(x.reshape(-1) - xd) <= 2e-10 / MU * norm(xd)
    ref = krylov.gmresr_cg(lat["ov"], b, 1e-10, 1e-3)
    its, its_ref = st[0].sumr_iters, sum(ref.middle_iters)
    print("CG iterations gpu / oracle:", its, its_ref, "sign calls", list(st[0].sign_calls))
    assert 0.8 * its_ref <= its <= 1.25 * its_ref
    assert st[0].gmresr_steps >= 1 and sum(st[0].sign_calls) > 2 * its
    if mixed == "half":
        # the CG's own sign calls stay at FP32 or above (FP16 rounding swamps
        # H^2's low modes); only GMRESR's c = D u may use FP16 (one per step)
        assert st[0].sign_calls[2] <= st[0].gmresr_steps and st[0].sign_calls[1] > 0


@pytest.mark.parametrize("noise", [0.0, 0.1])
def test_relcg_spectral_preconditioner(lat, noise):
    """Spectral preconditioner from 16 eigenvectors of H^2 installed in the
    eigenspace (exact, or perturbed by 10 %): the solve still reaches 1e-10,
    takes fewer CG iterations than without it, and about as many as the
    oracle with the same preconditioner."""
    ovl = require_gpu()
    b = synth.z2_source(lat["dims"], 91)
    V, VD, pre = _space(lat, 16, noise, 3)
    ctx, zg = _ctx(ovl, lat)
    _, st0, code0 = ctx.solve(to_dev(b), zg, _params(ovl, False, 0))
    ctx.eigspace_set(16, 40, MU, to_dev(V), to_dev(VD))
    x, st, code = ctx.solve(to_dev(b), zg, _params(ovl, False, 1))
    assert code == 0 and code0 == 0
    assert _true_res(lat, b, to_host(x)) <= 1e-10
    ref = krylov.gmresr_cg(lat["ov"], b, 1e-10, 1e-3, precond=pre)
    its, its0, its_ref = st[0].sumr_iters, st0[0].sumr_iters, sum(ref.middle_iters)
    print("CG iterations preconditioned gpu / oracle, plain gpu:", its, its_ref, its0)
    assert its < its0
    assert 0.8 * its_ref <= its <= 1.25 * its_ref


def test_relcg_batch_of_two(lat):
    """Two right-hand sides in one call, each to 1e-10 with the dense D."""
    ovl = require_gpu()
    ctx, zg = _ctx(ovl, lat)
    B = np.stack([synth.z2_source(lat["dims"], 92), synth.point_source(lat["dims"], 3, 1, 2)])
    X, st, code = ctx.solve(to_dev(B), zg, _params(ovl, True, 0))
    assert code == 0
    X = to_host(X)
    for f in range(2):
        assert _true_res(lat, B[f], X[f]) <= 1e-10


def _eigcg_params(ovl, calc):
    return ovl.solver_defaults(rho=1.4, mu=MU, tol=1e-10, eta_tilde=1e-3, middle_cg=1, use_deflation=1,
                               eig_calc=calc, n_eig=8, m_eig=30, k_recalc=25, f32_threshold=10.0,
                               half_threshold=2.0)


def test_eigcg_matches_oracle(lat):
    """GMRESR(eigCG) (Sec. 5 collection on the relCG middle solve, Alg. 6,
    the Sec. 5.1 cap, each middle solve preconditioned with the eigenvectors
    held when it starts): two calculating solves on the GPU and in the oracle
    from the same sources give the same number of diagonalisations (within
    one), Ritz values and residual norms within 1e-3, held pairs with
    v^D = D v (dense D) to the sign accuracy used, and true residuals
    <= 1e-10; then a solve that only uses the vectors takes about the
    oracle's CG iterations and fewer than the undeflated solve."""
    from oracle import eig
    ovl = require_gpu()
    ctx, zg = _ctx(ovl, lat)
    E = eig.EigCG(8, 30, MU)
    for s in range(2):
        b = synth.z2_source(lat["dims"], 94 + s)
        x, st, code = ctx.solve(to_dev(b), zg, _eigcg_params(ovl, 1))
        assert code == 0
        assert _true_res(lat, b, to_host(x)) <= 1e-10
        ref = eig.gmresr_eigcg(lat["ov"], b, 1e-10, 1e-3, E, calc=True)
        info = ctx.eigspace_info()
        vals, res = E.ritz()
        print("solve", s, "CG its gpu / oracle", st[0].sumr_iters, sum(ref.middle_iters), "ndiag", info["ndiag"],
              E.ndiag, "ritz", np.round(np.sort(info["ritz"]), 5), np.round(np.sort(vals), 5))
        assert info["held"] == 8 and abs(info["ndiag"] - E.ndiag) <= 1
        assert np.abs(np.sort(info["ritz"]) - np.sort(vals)).max() < 1e-3
        assert np.abs(np.sort(info["resid"]) - np.sort(res)).max() < 1e-3
    v, vd = ctx.eigspace_get()
    v, vd = to_host(v), to_host(vd)
    for vi, di in zip(v, vd):
        assert abs(norm(vi) - 1.0) < 1e-10
        assert norm(lat["D"] @ vi.reshape(-1) - di.reshape(-1)) < 1e-3
    b = synth.z2_source(lat["dims"], 97)
    x, st, code = ctx.solve(to_dev(b), zg, _eigcg_params(ovl, 0))
    assert code == 0 and _true_res(lat, b, to_host(x)) <= 1e-10
    ref = eig.gmresr_eigcg(lat["ov"], b, 1e-10, 1e-3, E, calc=False)
    _, st0, _ = ctx.solve(to_dev(b), zg, _params(ovl, False, 0))
    its, its_ref, its0 = st[0].sumr_iters, sum(ref.middle_iters), st0[0].sumr_iters
    print("deflated CG iterations gpu / oracle, undeflated gpu:", its, its_ref, its0)
    assert 0.8 * its_ref <= its <= 1.25 * its_ref
    assert its < 0.8 * its0
