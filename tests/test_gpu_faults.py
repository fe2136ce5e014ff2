"""Failure handling of the solver, forced from the host so that every kernel
exits normally: SUMR restarts after loss of normalisation (Sec. 2; the
threshold of Sec. 6 lowered so that the relaxed sign function's drift trips
it), the outer iteration limit (best iterate returned), a non-finite
right-hand side, and a deflation space whose v^D carries errors (GMRESR,
Alg. 3, still converges: the deflated start only changes where the middle
solves begin, Sec. 4)."""
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
def c1():
    U = synth.gauge_field(DIMS, 1, 0.3)
    k = WilsonKernel(DIMS, U, RHO)
    w = np.linalg.eigvalsh(k.dense("K"))
    z = Zolotarev(16, np.abs(w).min(), np.abs(w).max())
    return U, z, krylov.Overlap(krylov.SignFunction(k, z), MU)


def _ctx(ovl, U, z):
    ctx = ovl.Context(DIMS)
    ctx.gauge_load(to_dev(U))
    return ctx, ovl.zolo_from(z.nz, z.a, z.b, z.delta, z.omega, z.sigma)


def test_forced_restarts_still_converge(c1):
    """With the normalisation test at 1e-4 instead of 0.1 the relaxed middle
    solves restart (their U errs by up to 1e-2); the solve still reaches the
    1e-10 true residual with the oracle's D."""
    ovl = require_gpu()
    U, z, ov = c1
    ctx, zg = _ctx(ovl, U, z)
    b = synth.z2_source(DIMS, 71)
    p = ovl.solver_defaults(rho=RHO, mu=MU, tol=1e-10, eta_tilde=1e-3, f32_threshold=1e-6, norm_restart=1e-4)
    x, st, code = ctx.solve(to_dev(b), zg, p)
    print("case forced restarts: status", code, "restarts", st[0].restarts, "SUMR", st[0].sumr_iters, flush=True)
    assert code == 0 and st[0].restarts > 0
    assert norm(b - ov(to_host(x), 1e-15)) <= 1e-10 * norm(b)
    ctx.close()


def test_outer_limit_returns_best_iterate(c1):
    """One GMRESR step with five SUMR iterations cannot reach 1e-10: the call
    returns OVL_ERR_NOT_CONVERGED with its iterate in x, which reduces the
    residual below ||b||."""
    ovl = require_gpu()
    U, z, ov = c1
    ctx, zg = _ctx(ovl, U, z)
    b = synth.z2_source(DIMS, 72)
    p = ovl.solver_defaults(rho=RHO, mu=MU, tol=1e-10, eta_tilde=1e-3, max_outer=1, max_middle=5)
    x, st, code = ctx.solve(to_dev(b), zg, p, allow=(-4,))
    xh = to_host(x)
    r = norm(b - ov(xh, 1e-14)) / norm(b)
    print("case outer limit: status", code, "relative residual", r, flush=True)
    assert code == -4
    assert np.all(np.isfinite(xh)) and r < 1.0
    assert st[0].gmresr_steps == 1 and st[0].sumr_iters <= 5
    ctx.close()


def test_non_finite_source_is_a_breakdown(c1):
    """A NaN in the right-hand side is reported as OVL_ERR_BREAKDOWN."""
    ovl = require_gpu()
    U, z, _ = c1
    ctx, zg = _ctx(ovl, U, z)
    b = synth.z2_source(DIMS, 73)
    b[5, 2, 1] = np.nan
    p = ovl.solver_defaults(rho=RHO, mu=MU, tol=1e-10)
    with pytest.raises(ovl.OvlError) as e:
        ctx.solve(to_dev(b), zg, p)
    assert e.value.code == -5
    ctx.close()


def test_corrupted_vD_still_converges(c1):
    """The eight lowest eigenvectors of gamma_5 D (dense, exact sign function) with images
    v^D = D v + noise of relative size 1e-2: the deflated GMRESR(relSUMR) solve
    still reaches 1e-10 with the oracle's D."""
    ovl = require_gpu()
    U, z, ov = c1
    ctx, zg = _ctx(ovl, U, z)
    n = 256 * 12
    w, Q = np.linalg.eigh(WilsonKernel(DIMS, U, RHO).dense("K"))
    G5 = np.kron(np.eye(256), np.kron(np.diag([1.0, 1, -1, -1]), np.eye(3)))
    D = 0.5 * (1 + MU) * np.eye(n) + 0.5 * (1 - MU) * G5 @ (Q @ np.diag(np.sign(w)) @ Q.conj().T)
    H = G5 @ D
    h, Y = np.linalg.eigh(0.5 * (H + H.conj().T))
    idx = np.argsort(np.abs(h))[:8]
    rng = np.random.default_rng(5)
    V = np.stack([Y[:, j].reshape(256, 4, 3) for j in idx])
    VD = np.stack([(D @ Y[:, j]).reshape(256, 4, 3) for j in idx])
    noise = rng.normal(size=VD.shape) + 1j * rng.normal(size=VD.shape)
    for i in range(8):
        noise[i] *= 1e-2 * norm(VD[i]) / norm(noise[i])
    ctx.eigspace_set(8, 16, MU, to_dev(V), to_dev(VD + noise))
    b = synth.z2_source(DIMS, 74)
    p = ovl.solver_defaults(rho=RHO, mu=MU, tol=1e-10, eta_tilde=1e-3, f32_threshold=1e-6, use_deflation=1,
                            n_eig=8, m_eig=16)
    x, st, code = ctx.solve(to_dev(b), zg, p)
    r = norm(b - ov(to_host(x), 1e-15)) / norm(b)
    print("case corrupted v^D: status", code, "GMRESR steps", st[0].gmresr_steps, "residual", r, flush=True)
    assert code == 0 and r <= 1e-10
    ctx.close()


def test_eigspace_save_load_roundtrip(c1, tmp_path):
    """An eigenspace built by a calculating solve, saved and loaded into a fresh
    context of the same lattice (same launch table), gives the same held
    vectors, Ritz values and residuals bit for bit, and the same deflated
    solve; a file for other extents is refused."""
    ovl = require_gpu()
    import torch
    U, z, ov = c1
    ctx, zg = _ctx(ovl, U, z)
    ctx.eigspace_set(6, 24, MU)
    p = ovl.solver_defaults(rho=RHO, mu=MU, tol=1e-10, eta_tilde=1e-3, f32_threshold=1e-6, use_deflation=1,
                            eig_calc=1, n_eig=6, m_eig=24)
    ctx.solve(to_dev(synth.z2_source(DIMS, 80)), zg, p)
    ctx.eigspace_recompute(RHO, zg, 1e-12)
    path = str(tmp_path / "eig.bin")
    ctx.eigspace_save(path)
    ctx2, _ = _ctx(ovl, U, z)
    ctx2.set_tuning(ctx.tuning())
    ctx2.eigspace_load(path)
    i1, i2 = ctx.eigspace_info(), ctx2.eigspace_info()
    assert i1 == i2
    v1, d1 = ctx.eigspace_get()
    v2, d2 = ctx2.eigspace_get()
    assert torch.equal(v1, v2) and torch.equal(d1, d2)
    pd = ovl.solver_defaults(rho=RHO, mu=MU, tol=1e-10, eta_tilde=1e-3, f32_threshold=1e-6, use_deflation=1,
                             n_eig=6, m_eig=24)
    b = to_dev(synth.z2_source(DIMS, 81))
    x1, s1, c1_ = ctx.solve(b, zg, pd)
    x2, s2, c2_ = ctx2.solve(b, zg, pd)
    print("case save/load: held", i1["held"], "SUMR", s1[0].sumr_iters, s2[0].sumr_iters, flush=True)
    assert c1_ == 0 and c2_ == 0 and torch.equal(x1, x2)
    other = ovl.Context((4, 4, 4, 8))
    other.gauge_generate(1, 0.3)
    with pytest.raises(ovl.OvlError) as e:
        other.eigspace_load(path)
    assert e.value.code == -1
    other.close()
    ctx.close()
    ctx2.close()
