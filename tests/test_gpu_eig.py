"""GPU parity: Sec. 4 deflated start, Alg. 6 Rayleigh-Ritz, and eigSUMR
inside GMRESR(relSUMR) (Secs. 4-5) against the oracle and dense algebra."""
import numpy as np
import pytest

import synth
from oracle import eig, krylov
from oracle.lattice import WilsonKernel, g5, norm
from oracle.zolotarev import Zolotarev
from gpu_util import rel, require_gpu, to_dev, to_host

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
    h, Y = np.linalg.eigh(G5 @ D)
    z = Zolotarev(16, np.abs(w).min(), np.abs(w).max())
    return dict(dims=dims, U=U, k=k, D=D, G5=G5, h=h, Y=Y, z=z, shape=(k.V, 4, 3))


def _ctx(ovl, lat):
    ctx = ovl.Context(lat["dims"])
    ctx.gauge_load(to_dev(lat["U"]))
    z = lat["z"]
    return ctx, ovl.zolo_from(z.nz, z.a, z.b, z.delta, z.omega, z.sigma)


def _random_space(lat, k, seed):
    rng = np.random.default_rng(seed)
    V = rng.normal(size=(k,) + lat["shape"]) + 1j * rng.normal(size=(k,) + lat["shape"])
    VD = np.stack([(lat["D"] @ v.reshape(-1)).reshape(lat["shape"]) for v in V])
    return V, VD


def test_deflate_project_parity(lat):
    ovl = require_gpu()
    ctx, _ = _ctx(ovl, lat)
    V, VD = _random_space(lat, 7, 1)
    ctx.eigspace_set(7, 20, MU, to_dev(V), to_dev(VD))
    b = np.stack([synth.gaussian_source(lat["dims"], 5), synth.z2_source(lat["dims"], 6)])
    x0, dx0 = ctx.deflate_project(to_dev(b))
    x0, dx0 = to_host(x0), to_host(dx0)
    d = eig.Deflation(list(V), list(VD))
    for r in range(2):
        rx, rdx = d.project(b[r])
        assert rel(x0[r], rx) < 1e-11
        assert rel(dx0[r], rdx) < 1e-11


def test_rayleigh_ritz_parity(lat):
    ovl = require_gpu()
    ctx, _ = _ctx(ovl, lat)
    V, VD = _random_space(lat, 14, 2)
    ctx.eigspace_set(6, 20, MU, to_dev(V), to_dev(VD))
    ctx.eigspace_diagonalise()
    info = ctx.eigspace_info()
    assert info["held"] == 6
    v, vd = ctx.eigspace_get()
    v, vd = to_host(v), to_host(vd)
    M = np.stack([x.reshape(-1) for x in V], 1)
    MD = np.stack([x.reshape(-1) for x in VD], 1)
    rv, rvd, theta, C = eig.rayleigh_ritz(M, MD, 6, MU, 0.1)
    for i in range(6):
        ov = abs(np.vdot(rv[:, i], v[i].reshape(-1)))
        assert ov == pytest.approx(1.0, abs=1e-9)           # same vector up to a phase
        h_ref = np.vdot(rv[:, i], g5(rvd[:, i].reshape(lat["shape"])).reshape(-1)).real
        assert info["ritz"][i] == pytest.approx(h_ref, abs=1e-10)
        r_ref = norm(g5(rvd[:, i].reshape(lat["shape"])).reshape(-1) - h_ref * rv[:, i])
        assert info["resid"][i] == pytest.approx(r_ref, rel=1e-6, abs=1e-12)


def test_eigsumr_solves(lat):
    """Calculating solves collect Krylov vectors (Alg. 5) and diagonalise
    (Alg. 6); each returned Ritz vector is within its true residual of an
    eigenvalue of gamma_5 D; deflated solves reach 1e-10 with the oracle D."""
    ovl = require_gpu()
    ctx, zg = _ctx(ovl, lat)
    p = ovl.solver_defaults(rho=1.4, mu=MU, tol=1e-10, eta_tilde=1e-3, eig_calc=1, use_deflation=1,
                            n_eig=6, m_eig=30, f32_threshold=1e-6)
    D = lat["D"]
    for s in range(3):
        b = synth.z2_source(lat["dims"], 60 + s)
        x, st, code = ctx.solve(to_dev(b), zg, p)
        assert code == 0
        x = to_host(x)
        assert norm(b.reshape(-1) - D @ x.reshape(-1)) <= 1e-10 * norm(b)
    info = ctx.eigspace_info()
    assert info["held"] == 6 and info["ndiag"] >= 3
    ctx.eigspace_recompute(1.4, zg, 1e-12)
    v, _ = ctx.eigspace_get()
    for vi in to_host(v):
        vv = vi.reshape(-1)
        hv = np.vdot(vv, lat["G5"] @ D @ vv).real
        r = np.linalg.norm(lat["G5"] @ D @ vv - hv * vv)
        assert np.min(np.abs(lat["h"] - hv)) <= r + 1e-12
        assert r < 5e-2
    p2 = ovl.solver_defaults(rho=1.4, mu=MU, tol=1e-10, eta_tilde=1e-3, eig_calc=0, use_deflation=1,
                             n_eig=6, m_eig=30, f32_threshold=1e-6)
    b = synth.z2_source(lat["dims"], 70)
    x, st, code = ctx.solve(to_dev(b), zg, p2)
    assert code == 0
    assert norm(b.reshape(-1) - D @ to_host(x).reshape(-1)) <= 1e-10 * norm(b)


def test_eigsumr_trajectory_matches_oracle(lat):
    """Three calculating solves (Alg. 5 collection, Alg. 6 at every k = m and
    at the end of each middle solve) on the GPU and in the oracle, from the
    same sources: after each solve the same number of diagonalisations, and
    Ritz values and residual norms that agree (the relaxed sign calls round
    differently on the two sides, so the Krylov vectors drift apart slowly)."""
    ovl = require_gpu()
    ctx, zg = _ctx(ovl, lat)
    p = ovl.solver_defaults(rho=1.4, mu=MU, tol=1e-10, eta_tilde=1e-3, eig_calc=1, use_deflation=1,
                            n_eig=6, m_eig=30, f32_threshold=10.0)
    sign = krylov.SignFunction(lat["k"], lat["z"])
    ov = krylov.Overlap(sign, MU)
    E = eig.EigSUMR(6, 30, MU)
    for s in range(3):
        b = synth.z2_source(lat["dims"], 60 + s)
        _, _, code = ctx.solve(to_dev(b), zg, p)
        assert code == 0
        eig.gmresr_eigsumr(ov, b, 1e-10, 1e-3, E, calc=True)
        info = ctx.eigspace_info()
        vals, res = E.ritz()
        print("solve", s, "ndiag", info["ndiag"], E.ndiag, "ritz", np.round(info["ritz"], 5), np.round(vals, 5))
        assert info["ndiag"] == E.ndiag
        assert np.abs(np.sort(info["ritz"]) - np.sort(vals)).max() < 1e-3
        assert np.abs(np.sort(info["resid"]) - np.sort(res)).max() < 1e-3
    # after the third solve every Ritz value sits on an eigenvalue of gamma_5 D
    # (within its residual; not necessarily the six smallest)
    for th, r in zip(info["ritz"], info["resid"]):
        assert np.min(np.abs(lat["h"] - th)) <= min(1e-4, r)
