"""GPU parity for the batched solve: several right-hand sides of D[mu] x = b
(Sec. 1 eq. 1) solved together by GMRESR(relSUMR) (Algs. 1-3), every field
with its own recurrences, accuracies and convergence.  Each solution is
checked against a dense LU solve of the same overlap operator and by its true
residual with the oracle's FP64 D."""
import numpy as np
import pytest

import synth
from oracle import krylov
from oracle.lattice import WilsonKernel, norm
from oracle.zolotarev import Zolotarev
from gpu_util import require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu

DIMS = (4, 4, 4, 4)
RHO, MU = 1.4, 0.05


@pytest.fixture(scope="module")
def setup():
    U = synth.gauge_field(DIMS, 1, 0.3)
    k = WilsonKernel(DIMS, U, RHO)
    w, Q = np.linalg.eigh(k.dense("K"))
    z = Zolotarev(16, np.abs(w).min(), np.abs(w).max())
    n = k.V * 12
    G5 = np.kron(np.eye(k.V), np.kron(np.diag([1.0, 1, -1, -1]), np.eye(3)))
    S = Q @ np.diag(np.sign(w)) @ Q.conj().T
    Dd = 0.5 * (1 + MU) * np.eye(n) + 0.5 * (1 - MU) * G5 @ S
    D = krylov.Overlap(krylov.SignFunction(k, z), MU)
    return U, z, Dd, D


def _ctx(ovl, U, z):
    ctx = ovl.Context(DIMS)
    ctx.gauge_load(to_dev(U))
    return ctx, ovl.zolo_from(z.nz, z.a, z.b, z.delta, z.omega, z.sigma)


def _check(x, B, Dd, D, tol=1e-10):
    for f in range(B.shape[0]):
        b = B[f]
        bn = norm(b)
        if bn == 0.0:
            assert np.all(x[f] == 0)
            continue
        assert norm(b - D(x[f], 1e-15)) / bn <= tol, f"field {f}"
        xd = np.linalg.solve(Dd, b.reshape(-1))
        assert norm(x[f].reshape(-1) - xd) / norm(xd) <= 2 * tol / MU, f"field {f}"


@pytest.mark.parametrize("ladder", ["f64", "mixed"])
def test_batch_spin_colour(setup, ladder):
    """The twelve spin-colour point sources at the origin in one call."""
    ovl = require_gpu()
    U, z, Dd, D = setup
    ctx, zg = _ctx(ovl, U, z)
    B = np.stack([synth.point_source(DIMS, 0, s, c) for s in range(4) for c in range(3)])
    p = ovl.solver_defaults(rho=RHO, mu=MU, tol=1e-10, eta_tilde=1e-3,
                            f32_threshold=(1e-6 if ladder == "mixed" else 10.0))
    x, st, code = ctx.solve(to_dev(B), zg, p)
    assert code == 0
    _check(to_host(x), B, Dd, D)
    for s in st:
        assert s.gmresr_steps >= 1 and s.sumr_iters > 0 and s.mscg_iters > 0
        assert s.computed_relres <= 1e-10
    print("per-field SUMR iterations", [s.sumr_iters for s in st])


def test_batch_uneven(setup):
    """Fields of very different size and difficulty together: a zero field, a
    Gaussian field scaled by 1e6, a Z2 field and a point source; the zero field
    must come back zero and every other field converge on its own criterion."""
    ovl = require_gpu()
    U, z, Dd, D = setup
    ctx, zg = _ctx(ovl, U, z)
    B = np.stack([np.zeros((256, 4, 3), np.complex128),
                  1e6 * synth.gaussian_source(DIMS, 41),
                  synth.z2_source(DIMS, 42),
                  synth.point_source(DIMS, 17, 2, 1)])
    p = ovl.solver_defaults(rho=RHO, mu=MU, tol=1e-10, eta_tilde=1e-3, f32_threshold=1e-6,
                            half_threshold=3e-3)
    x, st, code = ctx.solve(to_dev(B), zg, p)
    assert code == 0
    _check(to_host(x), B, Dd, D)
    assert st[0].sumr_iters == 0 and st[0].mscg_iters == 0


def test_batch_matches_single(setup):
    """A field solved inside a batch and alone reach the same solution (to the
    solver tolerance; the sign precisions may differ between the two)."""
    ovl = require_gpu()
    U, z, Dd, D = setup
    ctx, zg = _ctx(ovl, U, z)
    B = np.stack([synth.gaussian_source(DIMS, 50 + i) for i in range(3)])
    p = ovl.solver_defaults(rho=RHO, mu=MU, tol=1e-11, eta_tilde=1e-3, f32_threshold=1e-6)
    xb, _, code = ctx.solve(to_dev(B), zg, p)
    assert code == 0
    xs, _, code = ctx.solve(to_dev(B[1:2]), zg, p)
    assert code == 0
    xb, xs = to_host(xb), to_host(xs)
    assert norm(xb[1] - xs[0]) / norm(xs[0]) <= 4e-11 / MU


def test_batch_limit(setup):
    """More right-hand sides than one call accepts is an argument error."""
    ovl = require_gpu()
    U, z, _, _ = setup
    ctx, zg = _ctx(ovl, U, z)
    B = np.zeros((17, 256, 4, 3), np.complex128)
    p = ovl.solver_defaults(rho=RHO, mu=MU)
    with pytest.raises(ovl.OvlError):
        ctx.solve(to_dev(B), zg, p)


def test_solve_many_uneven():
    """Independent lattice instances of different sizes solved at once (one
    context and stream each): every solution has a true residual <= 1e-10
    with the oracle's D, and equals the same instance solved alone."""
    ovl = require_gpu()
    import torch
    mu = 0.03
    z = Zolotarev(16, 0.2, 8.0 - RHO)
    specs = [((4, 4, 4, 4), 21, 0.25), ((4, 4, 4, 8), 22, 0.3), ((6, 4, 4, 8), 23, 0.2),
             ((4, 4, 4, 4), 24, 0.35), ((8, 4, 4, 4), 25, 0.3)]
    items, oracles = [], []
    for i, (dims, seed, eps) in enumerate(specs):
        U = synth.gauge_field(dims, seed, eps)
        ctx = ovl.Context(dims, stream=torch.cuda.Stream())
        ctx.gauge_load(to_dev(U))
        b = synth.z2_source(dims, 104 + i)
        zg = ovl.zolo_from(z.nz, z.a, z.b, z.delta, z.omega, z.sigma)
        items.append((ctx, zg, to_dev(b)))
        oracles.append((krylov.Overlap(krylov.SignFunction(WilsonKernel(dims, U, RHO), z), mu), b))
    p = ovl.solver_defaults(rho=RHO, mu=mu, tol=1e-10, eta_tilde=1e-3, f32_threshold=1e-6, half_threshold=3e-3)
    res = ovl.solve_many(items, p)
    torch.cuda.synchronize()
    for (ctx, zg, bd), (x, st, code), (D, b) in zip(items, res, oracles):
        assert code == 0
        xh = to_host(x)
        assert norm(b - D(xh, 1e-15)) / norm(b) <= 1e-10
        x1, _, code1 = ctx.solve(bd, zg, p)
        assert code1 == 0 and np.array_equal(to_host(x1), xh)
    for ctx, _, _ in items:
        ctx.close()


def test_solve_many_rejects_repeated_context(setup):
    ovl = require_gpu()
    U, z, _, _ = setup
    ctx, zg = _ctx(ovl, U, z)
    b = to_dev(synth.z2_source(DIMS, 9))
    with pytest.raises(ovl.OvlError):
        ovl.solve_many([(ctx, zg, b), (ctx, zg, b)], ovl.solver_defaults(rho=RHO, mu=MU))
