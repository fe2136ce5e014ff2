"""GPU edge cases and full-size checks in the benchmark's launch
configurations: empty and oversized batches, the largest accepted batch, the
reduced-precision K at 16^3 x 32 on sampled sites against the oracle, and
sign(K)^2 = 1 at 16^3 x 32 in every storage precision (a property that holds
at any size, Sec. 1), and the eigensolver's argument checks."""
import numpy as np
import pytest

import synth
from oracle.lattice import WilsonKernel
from gpu_util import max_rel_elem, rel, require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu
MAX_NRHS = 16


def test_empty_and_oversized_batches_rejected():
    ovl = require_gpu()
    import torch
    dims = (4, 4, 4, 4)
    ctx = ovl.Context(dims)
    ctx.gauge_load(to_dev(synth.gauge_field(dims, 1, 0.3)))
    z = ovl.zolotarev_coeffs(8, 0.5, 6.6)
    empty = torch.zeros((0, 256, 4, 3), dtype=torch.complex128, device="cuda")
    big = torch.zeros((MAX_NRHS + 1, 256, 4, 3), dtype=torch.complex128, device="cuda")
    for psi in (empty, big):
        for call in (lambda: ctx.wilson_dslash(psi), lambda: ctx.kernel_K_apply(psi, 1.4),
                     lambda: ctx.sign(psi, 1.4, z, 1e-6), lambda: ctx.overlap(psi, 1.4, 0.05, z, 1e-6)):
            with pytest.raises(ovl.OvlError) as e:
                call()
            assert e.value.code == -1
    ctx.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "half"])
def test_largest_batch_matches_oracle(prec):
    """MAX_NRHS fields in one stencil launch on a ragged lattice, each against
    the oracle."""
    ovl = require_gpu()
    dims = (6, 4, 6, 5)
    p = {"f64": ovl.F64, "f32": ovl.F32, "half": ovl.HALF}[prec]
    U = synth.gauge_field(dims, 21, 0.4)
    ctx = ovl.Context(dims)
    ctx.gauge_load(to_dev(U))
    psi = np.stack([synth.gaussian_source(dims, 500 + f) for f in range(MAX_NRHS)])
    h = to_host(ctx.wilson_dslash(to_dev(psi), prec=p))
    ora = WilsonKernel(dims, U, 1.4)
    tol = {"f64": 1e-14, "f32": 2e-6, "half": 5e-3}[prec]
    for f in range(MAX_NRHS):
        assert max_rel_elem(h[f], ora.hop(psi[f])) < tol, f
    ctx.close()


@pytest.fixture(scope="module")
def c2():
    """The 16^3 x 32 workload: links eps 0.25 seed 2, ten exact kernel modes,
    N_Z = 20 on [|lambda_10|, lambda_max], Gaussian source seed 102."""
    ovl = require_gpu()
    dims = (16, 16, 16, 32)
    V = int(np.prod(dims))
    ctx = ovl.Context(dims)
    Ud = to_dev(np.zeros((V, 4, 3, 3)))
    ctx.gauge_generate(2, 0.25, out=Ud)
    ev, lmax = ctx.lowmodes_compute(1.4, 10, tol=1e-10)
    z = ovl.zolotarev_coeffs(20, max(abs(e) for e in ev), lmax)
    yield dict(ctx=ctx, Ud=Ud, z=z, dims=dims, V=V, ovl=ovl)
    ctx.close()


@pytest.mark.parametrize("prec", ["f32", "half"])
def test_K_16c32_sampled(c2, prec):
    """K in FP32 / FP16 storage at 16^3 x 32, autotuned as in the solve, on
    sampled sites against the oracle."""
    ovl, ctx = c2["ovl"], c2["ctx"]
    p = {"f32": ovl.F32, "half": ovl.HALF}[prec]
    psi = synth.gaussian_source(c2["dims"], 102)
    k = to_host(ctx.kernel_K_apply(to_dev(psi), 1.4, prec=p))
    rng = np.random.default_rng(1)
    V = c2["V"]
    sites = np.unique(np.concatenate([[0, V - 1, 15, 16 * 16 * 16 - 1, 16 * 16 * 16], rng.integers(0, V, 300)]))
    ref = WilsonKernel(c2["dims"], to_host(c2["Ud"]), 1.4).K_sites(psi, sites)
    err = max_rel_elem(k[sites], ref)
    print("case", prec, "max rel elem", err, "variants", ctx.tuning(), flush=True)
    assert err < {"f32": 2e-6, "half": 5e-3}[prec]


@pytest.mark.parametrize("prec,eta,tol", [("f32", 1e-6, 1e-5), ("half", 1e-2, 2e-2)])
def test_sign_squared_16c32(c2, prec, eta, tol):
    """sign(K)^2 psi = psi at 16^3 x 32 with the ten exact modes, in the
    reduced storage precisions the solver uses, to the accuracy asked for."""
    ovl, ctx = c2["ovl"], c2["ctx"]
    p = {"f32": ovl.F32, "half": ovl.HALF}[prec]
    psi = to_dev(synth.gaussian_source(c2["dims"], 103))
    s1, st = ctx.sign(psi, 1.4, c2["z"], eta, prec=p)
    s2, _ = ctx.sign(s1, 1.4, c2["z"], eta, prec=p)
    err = rel(to_host(s2), to_host(psi))
    print("case", prec, "sign^2 error", err, "mscg iterations", st.mscg_iters, flush=True)
    assert err < tol


def test_eigensolver_16c32_pairs_and_deflation(c2):
    """The standalone eigensolver at the benchmark's full size (n = 8, m = 40,
    two runs, Sec. 5.1 relaxation, mixed precision): every reported residual
    equals ||gamma_5 D v - h v|| recomputed with the FP64 operator at 1e-12,
    each v has unit norm, and the benchmark source solved from the deflated
    start reaches 1e-10 against the FP64 operator (properties that hold at
    any size)."""
    import torch
    ovl, ctx, z = c2["ovl"], c2["ctx"], c2["z"]
    p = ovl.solver_defaults(rho=1.4, mu=0.02, n_eig=8, m_eig=40, eig_eps=1e-4, f32_threshold=1e-6,
                            half_threshold=3e-3)
    code, hist, _ = ctx.eigensolve(ctx.source(ovl.SRC_Z2, seed=103), z, p, max_runs=2)
    print("case eigensolver 16^3x32 runs", hist, flush=True)
    assert code in (0, -4) and len(hist) >= 1
    info = ctx.eigspace_info()
    v, _ = ctx.eigspace_get()
    assert info["held"] == 8
    Dv, _ = ctx.overlap(v, 1.4, 0.02, z, 1e-12)
    g5Dv = Dv.clone()
    g5Dv[:, :, 2:, :] *= -1
    for i in range(8):
        h = float(torch.vdot(v[i].flatten(), g5Dv[i].flatten()).real)
        r = float(torch.linalg.vector_norm(g5Dv[i] - h * v[i]))
        assert abs(float(torch.linalg.vector_norm(v[i])) - 1.0) < 1e-10
        assert abs(h - info["ritz"][i]) < 1e-9 and abs(r - info["resid"][i]) < 1e-8, (i, h, r)
    ps = ovl.solver_defaults(rho=1.4, mu=0.02, tol=1e-10, eta_tilde=3e-3, use_deflation=1, n_eig=8, m_eig=40,
                             f32_threshold=1e-6, half_threshold=3e-3)
    b = ctx.source(ovl.SRC_GAUSS, seed=102)
    x, st, code = ctx.solve(b, z, ps)
    Dx, _ = ctx.overlap(x, 1.4, 0.02, z, 1e-13)
    res = float(torch.linalg.vector_norm(b - Dx) / torch.linalg.vector_norm(b))
    print("case deflated solve 16^3x32 SUMR iterations", st[0].sumr_iters, "true residual", res, flush=True)
    assert code == 0 and res <= 1e-10


def test_eigcg_16c32_solve_and_pairs(c2):
    """One calculating GMRESR(eigCG) solve at the benchmark's full size
    (n = 8, m = 30, mixed precision): the solution reaches 1e-10 against the
    FP64 operator, and every held pair has a unit v and v^D within 1e-3 of
    D v (FP64 operator at 1e-12): v^D comes from the CG's own relaxed H
    products, held to the Sec. 5.1 bound."""
    import torch
    ovl, ctx, z = c2["ovl"], c2["ctx"], c2["z"]
    p = ovl.solver_defaults(rho=1.4, mu=0.02, tol=1e-10, eta_tilde=1e-3, middle_cg=1, eig_calc=1, use_deflation=1,
                            n_eig=8, m_eig=30, f32_threshold=1e-6, half_threshold=3e-3)
    ctx.eigspace_set(8, 30, 0.02)   # start from an empty eigenspace
    b = ctx.source(ovl.SRC_POINT, site=0, spin=0, colour=0)
    x, st, code = ctx.solve(b, z, p)
    Dx, _ = ctx.overlap(x, 1.4, 0.02, z, 1e-13)
    res = float(torch.linalg.vector_norm(b - Dx) / torch.linalg.vector_norm(b))
    info = ctx.eigspace_info()
    print("case eigCG 16^3x32: CG iterations", st[0].sumr_iters, "diagonalisations", info["ndiag"],
          "true residual", res, flush=True)
    assert code == 0 and res <= 1e-10 and info["held"] == 8 and info["ndiag"] >= 1
    v, vd = ctx.eigspace_get()
    Dv, _ = ctx.overlap(v, 1.4, 0.02, z, 1e-12)
    for i in range(8):
        assert abs(float(torch.linalg.vector_norm(v[i])) - 1.0) < 1e-10
        assert float(torch.linalg.vector_norm(Dv[i] - vd[i])) < 1e-3


def test_eigensolver_arguments_rejected():
    """The standalone eigensolver refuses a zero start vector, more than 170
    eigenvectors (three sets must fit one 512-vector Rayleigh-Ritz), m <= n
    and a zero run limit, each with OVL_ERR_ARG and no work done."""
    ovl = require_gpu()
    import torch
    dims = (4, 4, 4, 4)
    ctx = ovl.Context(dims)
    ctx.gauge_load(to_dev(synth.gauge_field(dims, 1, 0.3)))
    z = ovl.zolotarev_coeffs(8, 0.5, 6.6)
    q0 = to_dev(synth.z2_source(dims, 1))
    zero = torch.zeros_like(q0)
    cases = [(zero, dict(n_eig=4, m_eig=10), 2), (q0, dict(n_eig=171, m_eig=200), 2),
             (q0, dict(n_eig=8, m_eig=8), 2), (q0, dict(n_eig=4, m_eig=10), 0)]
    for q, kw, runs in cases:
        p = ovl.solver_defaults(rho=1.4, mu=0.05, **kw)
        with pytest.raises(ovl.OvlError) as e:
            ctx.eigensolve(q, z, p, max_runs=runs)
        assert e.value.code == -1, (kw, runs)
    ctx.close()


def test_eigensolver_run_too_short_for_n():
    """A run that ends at the norm test before n_eig + 1 vectors are held (no
    diagonalisation yet) is reported as OVL_ERR_BREAKDOWN, not continued: on
    4^4 the Alg. 1 basis loses its normalisation well before 151 steps."""
    ovl = require_gpu()
    dims = (4, 4, 4, 4)
    ctx = ovl.Context(dims)
    ctx.gauge_load(to_dev(synth.gauge_field(dims, 1, 0.3)))
    z = ovl.zolotarev_coeffs(8, 0.5, 6.6)
    p = ovl.solver_defaults(rho=1.4, mu=0.05, n_eig=150, m_eig=200, f32_threshold=10.0, half_threshold=10.0)
    with pytest.raises(ovl.OvlError) as e:
        ctx.eigensolve(to_dev(synth.z2_source(dims, 1)), z, p, max_runs=2, eta_fixed=1e-6)
    assert e.value.code == -5
    ctx.close()
