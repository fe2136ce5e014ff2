"""Full-size parity: solves at the benchmark's sizes and launch configurations
checked with the oracle's FP64 overlap operator (Sec. 1, eq. 1; sign(K) with
the GPU's kernel low modes passed in as data and the same Zolotarev
coefficients, Sec. 3), and the FP64 overlap operator itself against the
oracle element by element on a multi-block lattice.

Every oracle input is generated on the host (the seeded generators); the
GPU's generated gauge fields and sources are compared with them bit for bit
at full size."""
import numpy as np
import pytest

import synth
from oracle import krylov
from oracle.lattice import WilsonKernel, norm
from oracle.zolotarev import Zolotarev
from gpu_util import max_rel_elem, rel, require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu
RHO = 1.4


def _generated(ovl, ctx, dims, seed, eps):
    """The GPU's generated field (left loaded in ctx) and the host's; they must
    agree bit for bit."""
    V = int(np.prod(dims))
    Ud = to_dev(np.zeros((V, 4, 3, 3)))
    ctx.gauge_generate(seed, eps, out=Ud)
    U = synth.gauge_field(dims, seed, eps)
    assert np.array_equal(to_host(Ud).view(np.uint64), U.view(np.uint64)), "generated links differ"
    return U


def _oracle_overlap(dims, U, mu, z, ctx=None, nlow=0, evals=None):
    """The oracle's D[mu], with the context's kernel low modes (as data) when
    nlow > 0, after checking that they are orthonormal eigenvectors of the
    oracle's K."""
    k = WilsonKernel(dims, U, RHO)
    low = None
    if nlow:
        vecs = to_host(ctx.lowmodes_get())
        for i in range(nlow):
            assert norm(k.K(vecs[i]) - evals[i] * vecs[i]) <= 1e-9, f"low mode {i}"
        G = vecs.reshape(nlow, -1).conj() @ vecs.reshape(nlow, -1).T
        assert np.abs(G - np.eye(nlow)).max() <= 1e-12
        low = krylov.LowModes(evals, vecs)
    return krylov.Overlap(krylov.SignFunction(k, z, low), mu)


def _zolo_pair(ovl, nz, a, b):
    z = Zolotarev(nz, a, b)
    return z, ovl.zolo_from(z.nz, z.a, z.b, z.delta, z.omega, z.sigma)


def test_headline_16c32_solve_with_oracle_operator():
    """The 16^3 x 32 benchmark solve (links eps 0.25 seed 2, ten exact kernel
    modes, N_Z = 20, mu = 0.02, Gaussian source seed 102, mixed ladder with
    middle solves to 3e-3): true residual <= 1e-10 with the oracle's D; and
    the GPU's FP64 D[mu] x against the oracle's at full size."""
    ovl = require_gpu()
    dims, mu = (16, 16, 16, 32), 0.02
    ctx = ovl.Context(dims)
    U = _generated(ovl, ctx, dims, 2, 0.25)
    ev, lmax = ctx.lowmodes_compute(RHO, 10, tol=1e-10)
    z, zg = _zolo_pair(ovl, 20, max(abs(e) for e in ev), lmax)
    b = synth.gaussian_source(dims, 102)
    bd = ctx.source(ovl.SRC_GAUSS, seed=102)
    assert np.array_equal(to_host(bd).view(np.uint64), b.view(np.uint64))
    p = ovl.solver_defaults(rho=RHO, mu=mu, tol=1e-10, eta_tilde=3e-3, f32_threshold=1e-6, half_threshold=3e-3,
                            max_middle=4000, max_mscg=20000)
    x, st, code = ctx.solve(bd, zg, p)
    print("case headline 16^3x32 status", code, "SUMR", st[0].sumr_iters, flush=True)
    assert code == 0
    xh = to_host(x)
    ov = _oracle_overlap(dims, U, mu, z, ctx, 10, ev)
    Dx = ov(xh, 1e-13)
    res = norm(b - Dx) / norm(b)
    print("case headline 16^3x32 oracle true residual", res, flush=True)
    assert res <= 1e-10
    Dg, _ = ctx.overlap(x, RHO, mu, zg, 1e-13)
    assert norm(to_host(Dg) - Dx) <= 1e-12 * norm(xh)
    ctx.close()


def test_uneven_instances_each_size_with_oracle_operator():
    """One instance of each size of the uneven batch (8^4, 8^3x16, 12^3x24,
    16^4; eps from the batch's generator, gauge seed 400 + i, Z2 source
    seed 104 + i, mu = 0.03, N_Z = 20, ten exact modes, mixed ladder), solved
    together through the batched entry point: each true residual <= 1e-10
    with the oracle's D."""
    ovl = require_gpu()
    import torch
    mu = 0.03
    eps = synth.instance_eps(24, 4)
    sizes = [(8, 8, 8, 8), (8, 8, 8, 16), (12, 12, 12, 24), (16, 16, 16, 16)]
    items, host = [], []
    for k, dims in enumerate(sizes):
        i = 6 * k
        ctx = ovl.Context(dims, stream=torch.cuda.Stream())
        U = _generated(ovl, ctx, dims, 400 + i, float(eps[i]))
        ev, lmax = ctx.lowmodes_compute(RHO, 10, tol=1e-10)
        z, zg = _zolo_pair(ovl, 20, max(abs(e) for e in ev), lmax)
        b = synth.z2_source(dims, 104 + i)
        items.append((ctx, zg, to_dev(b)))
        host.append((dims, U, z, ev, b))
    p = ovl.solver_defaults(rho=RHO, mu=mu, tol=1e-10, eta_tilde=1e-3, f32_threshold=1e-6, half_threshold=3e-3,
                            max_middle=4000, max_mscg=20000)
    res = ovl.solve_many(items, p)
    for (ctx, _, _), (dims, U, z, ev, b), (x, st, code) in zip(items, host, res):
        assert code == 0, dims
        ov = _oracle_overlap(dims, U, mu, z, ctx, 10, ev)
        r = norm(b - ov(to_host(x), 1e-13)) / norm(b)
        print("case instance", dims, "SUMR", st[0].sumr_iters, "oracle true residual", r, flush=True)
        assert r <= 1e-10
        ctx.close()


@pytest.mark.parametrize("nlow", [0, 6])
def test_overlap_apply_8c16_vs_oracle(nlow):
    """D[mu] psi in FP64 on 8^3 x 16 (32 blocks of 256 sites per field, two
    fields in one call) against the oracle element by element, with and
    without exactly treated kernel modes (N_Z = 20, both sides to 1e-13)."""
    ovl = require_gpu()
    dims, mu = (8, 8, 8, 16), 0.05
    ctx = ovl.Context(dims)
    U = _generated(ovl, ctx, dims, 5, 0.25)
    if nlow:
        ev, lmax = ctx.lowmodes_compute(RHO, nlow, tol=1e-11)
        a = max(abs(e) for e in ev)
    else:
        lo, _, _ = ctx.kernel_interval(RHO)
        ev, a, lmax = None, 0.95 * lo, 8.0 - RHO
    z, zg = _zolo_pair(ovl, 20, a, lmax)
    psi = np.stack([synth.gaussian_source(dims, 61), synth.z2_source(dims, 62)])
    out, _ = ctx.overlap(to_dev(psi), RHO, mu, zg, 1e-13)
    out = to_host(out)
    ov = _oracle_overlap(dims, U, mu, z, ctx, nlow, ev)
    for f in range(2):
        ref = ov(psi[f], 1e-13)
        err = max_rel_elem(out[f], ref)
        print("case overlap 8^3x16 nlow", nlow, "field", f, "max rel elem", err, flush=True)
        assert err <= 1e-12
        assert rel(out[f], ref) <= 1e-12
    ctx.close()


def test_kernel_interval_vs_dense_spectrum():
    """The Lanczos interval of |K| (set-up of the Zolotarev approximation when
    no modes are treated exactly) against the dense spectrum of the oracle's K
    on 4^4: the smallest Ritz value is within its residual bound of
    min |lambda|^2 and never below it; the largest never above max |lambda|."""
    ovl = require_gpu()
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 1, 0.3)
    ctx = ovl.Context(dims)
    ctx.gauge_load(to_dev(U))
    lo, err, hi = ctx.kernel_interval(RHO)
    w = np.abs(np.linalg.eigvalsh(WilsonKernel(dims, U, RHO).dense("K")))
    print("case interval", lo, err, hi, w.min(), w.max(), flush=True)
    assert lo * lo >= w.min() ** 2 * (1 - 1e-12)
    assert lo * lo - w.min() ** 2 <= max(err, 1e-9)
    assert abs(lo - w.min()) <= 1e-6
    assert hi <= w.max() * (1 + 1e-12) and hi >= 0.99 * w.max()
    ctx.close()


def test_c3_eigsumr_solve_with_oracle_operator():
    """The 24^3 x 48 precision form (links eps 0.25 seed 3, mu = 0.01,
    N_Z = 20 on the Lanczos interval, eigSUMR with n = 20, m = 60): one
    calculating mixed GMRESR(eigSUMR) solve (Algs. 3, 2, 5, 6) of the
    spin 0 colour 0 point source, then the deflated mixed solve (Sec. 4) of the
    spin 1 colour 0 point source; its true residual with the oracle's D is at
    most 1e-10."""
    ovl = require_gpu()
    dims, mu = (24, 24, 24, 48), 0.01
    ctx = ovl.Context(dims)
    U = _generated(ovl, ctx, dims, 3, 0.25)
    lo, _, _ = ctx.kernel_interval(RHO)
    z, zg = _zolo_pair(ovl, 20, 0.95 * lo, 8.0 - RHO)
    ctx.eigspace_set(20, 60, mu)

    def params(calc):
        return ovl.solver_defaults(rho=RHO, mu=mu, tol=1e-10, eta_tilde=1e-3, f32_threshold=1e-6,
                                   half_threshold=3e-3, max_middle=6000, max_mscg=20000, use_deflation=1,
                                   eig_calc=calc, n_eig=20, m_eig=60)
    b0 = ctx.source(ovl.SRC_POINT, site=0, spin=0, colour=0)
    _, st, code = ctx.solve(b0, zg, params(1))
    info = ctx.eigspace_info()
    print("case C3 calculating solve status", code, "SUMR", st[0].sumr_iters, "diagonalisations", info["ndiag"],
          flush=True)
    assert code == 0 and info["held"] == 20
    ctx.eigspace_recompute(RHO, zg, 1e-12)
    b = synth.point_source(dims, 0, 1, 0)
    x, st, code = ctx.solve(to_dev(b), zg, params(0))
    print("case C3 deflated solve status", code, "SUMR", st[0].sumr_iters, flush=True)
    assert code == 0
    xh = to_host(x)
    ctx.close()
    ov = _oracle_overlap(dims, U, mu, z)
    r = norm(b - ov(xh, 1e-13)) / norm(b)
    print("case C3 oracle true residual", r, flush=True)
    assert r <= 1e-10


def test_c3_half_sign_of_point_source():
    """sign(K) of a point source on 24^3 x 48 with FP16 storage at the relaxed
    accuracy 1e-2 (20 poles): before the multi-shift CG's vectors cover the
    lattice their outermost sites fall below FP32's normal range, where a
    site's FP16 scale cannot be inverted (such sites are stored as zero).  The
    call completes, and the result agrees with the FP64 sign at 1e-10 within
    the requested accuracy."""
    ovl = require_gpu()
    dims = (24, 24, 24, 48)
    ctx = ovl.Context(dims)
    ctx.gauge_generate(3, 0.25)
    lo, _, _ = ctx.kernel_interval(RHO)
    _, zg = _zolo_pair(ovl, 20, 0.95 * lo, 8.0 - RHO)
    b = ctx.source(ovl.SRC_POINT, site=0, spin=0, colour=0)
    s16, st16 = ctx.sign(b, RHO, zg, 1e-2, prec=ovl.HALF)
    s64, _ = ctx.sign(b, RHO, zg, 1e-10)
    h16, h64 = to_host(s16), to_host(s64)
    err = norm(h16 - h64) / norm(to_host(b))
    print("case C3 FP16 point-source sign: iterations", st16.mscg_iters, "difference", err, flush=True)
    assert np.all(np.isfinite(h16)) and err <= 1e-2
    ctx.close()
