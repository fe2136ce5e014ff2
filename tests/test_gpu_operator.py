"""GPU parity: Wilson hopping stencil and kernel K (paper Sec. 1, eq. 2) in
FP64 and FP32 against the oracle, element by element."""
import numpy as np
import pytest

import synth
from oracle.lattice import WilsonKernel
from gpu_util import max_rel_elem, rel, require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu

# several tiles plus a ragged tail (V not a multiple of 256), unequal extents
CASES = [(4, 4, 4, 4), (4, 6, 2, 8), (6, 4, 6, 5), (2, 2, 2, 2)]


@pytest.mark.parametrize("dims", CASES)
def test_hop_and_K_f64(dims):
    ovl = require_gpu()
    print("case", dims, flush=True)
    U = synth.gauge_field(dims, 11, 0.4)
    ora = WilsonKernel(dims, U, 1.4)
    psi = np.stack([synth.gaussian_source(dims, s) for s in (1, 2, 3)])
    ctx = ovl.Context(dims)
    ctx.gauge_load(to_dev(U))
    h = to_host(ctx.wilson_dslash(to_dev(psi)))
    k = to_host(ctx.kernel_K_apply(to_dev(psi), 1.4))
    for r in range(3):
        assert max_rel_elem(h[r], ora.hop(psi[r])) < 1e-14
        assert max_rel_elem(k[r], ora.K(psi[r])) < 1e-14


@pytest.mark.parametrize("dims", CASES[:2])
def test_hop_and_K_f32(dims):
    ovl = require_gpu()
    U = synth.gauge_field(dims, 12, 0.4)
    ora = WilsonKernel(dims, U, 1.4)
    psi = synth.gaussian_source(dims, 4)
    ctx = ovl.Context(dims)
    ctx.gauge_load(to_dev(U))
    h = to_host(ctx.wilson_dslash(to_dev(psi), prec=ovl.F32))
    k = to_host(ctx.kernel_K_apply(to_dev(psi), 1.4, prec=ovl.F32))
    # FP32 storage and arithmetic: a few units of 2^-24 per term, 8 terms
    assert max_rel_elem(h, ora.hop(psi)) < 2e-6
    assert max_rel_elem(k, ora.K(psi)) < 2e-6
    assert rel(k, ora.K(psi)) < 1e-6


def test_K_full_size_sampled():
    """16^3 x 32 (the FP64 solve workload), K on 256 sampled sites vs the oracle."""
    ovl = require_gpu()
    dims = (16, 16, 16, 32)
    V = 16 * 16 * 16 * 32
    ctx = ovl.Context(dims)
    Ud = to_dev(np.zeros((V, 4, 3, 3)))
    ctx.gauge_generate(2, 0.25, out=Ud)
    U = to_host(Ud)
    psi = synth.gaussian_source(dims, 102)
    k = to_host(ctx.kernel_K_apply(to_dev(psi), 1.4))
    ora = WilsonKernel(dims, U, 1.4)
    rng = np.random.default_rng(0)
    sites = np.concatenate([[0, V - 1, 15, 16 * 16 * 16 - 1], rng.integers(0, V, 252)])
    ref = ora.K_sites(psi, sites)
    assert max_rel_elem(k[sites], ref) < 1e-14


def test_gamma5_hermiticity_gpu():
    """(chi, K psi) = (K chi, psi) for the GPU operator (K Hermitian, Sec. 1)."""
    ovl = require_gpu()
    dims = (4, 4, 4, 6)
    ctx = ovl.Context(dims)
    ctx.gauge_load(to_dev(synth.gauge_field(dims, 3, 0.5)))
    a, b = synth.gaussian_source(dims, 5), synth.gaussian_source(dims, 6)
    Ka = to_host(ctx.kernel_K_apply(to_dev(a), 1.4))
    Kb = to_host(ctx.kernel_K_apply(to_dev(b), 1.4))
    lhs, rhs = np.vdot(a, Kb), np.vdot(Ka, b)
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


@pytest.mark.parametrize("dims", CASES[:2])
def test_hop_and_K_half(dims):
    """FP16 links and FP16 spinors (per-site scale), FP32 arithmetic: errors of
    a few units of 2^-11 relative to the field's largest component."""
    ovl = require_gpu()
    U = synth.gauge_field(dims, 13, 0.4)
    ora = WilsonKernel(dims, U, 1.4)
    psi = synth.gaussian_source(dims, 5)
    ctx = ovl.Context(dims)
    ctx.gauge_load(to_dev(U))
    h = to_host(ctx.wilson_dslash(to_dev(psi), prec=ovl.HALF))
    k = to_host(ctx.kernel_K_apply(to_dev(psi), 1.4, prec=ovl.HALF))
    assert max_rel_elem(h, ora.hop(psi)) < 5e-3
    assert rel(k, ora.K(psi)) < 2e-3


def test_half_storage_of_subnormal_sites():
    """FP16 storage of a field whose site magnitudes run from 1 down to 1e-44,
    as at the edge of the support of a Krylov vector grown from a point
    source: sites whose largest component is below the smallest normal float
    are stored as zero (their scale cannot be inverted), so every output is
    finite and the stencil and K agree with the oracle as for any other field."""
    ovl = require_gpu()
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 13, 0.4)
    ora = WilsonKernel(dims, U, 1.4)
    psi = synth.gaussian_source(dims, 6)
    psi = psi * np.logspace(0, -44, psi.shape[0])[:, None, None]
    ctx = ovl.Context(dims)
    ctx.gauge_load(to_dev(U))
    for nf in (1, 2):   # separate launch-table entries (and launch variants)
        x = np.stack([psi] * nf) if nf > 1 else psi
        h = to_host(ctx.wilson_dslash(to_dev(x), prec=ovl.HALF))
        k = to_host(ctx.kernel_K_apply(to_dev(x), 1.4, prec=ovl.HALF))
        h, k = (h[0], k[0]) if nf > 1 else (h, k)
        assert np.all(np.isfinite(h)) and np.all(np.isfinite(k))
        assert rel(h, ora.hop(psi)) < 5e-3
        assert rel(k, ora.K(psi)) < 2e-3
    ctx.close()


def test_two_row_links_and_fallback():
    """Links in SU(3) (Sec. 1, eq. 2) pass the test (deviation at rounding
    level) and the FP32 / FP16 stencils read two rows per link; the result
    matches the oracle as the full links do.  Links times the phase exp(0.3 i)
    (unitary, determinant not 1) fail it, the full links are used, and the
    stencils still match the oracle on those links."""
    ovl = require_gpu()
    dims = (4, 6, 2, 8)
    U = synth.gauge_field(dims, 15, 0.4)
    psi = synth.gaussian_source(dims, 7)
    for links, two_row in ((U, True), (U * np.exp(0.3j), False)):
        ora = WilsonKernel(dims, links, 1.4)
        ctx = ovl.Context(dims)
        ctx.gauge_load(to_dev(links))
        dev, tr = ctx.gauge_info()
        print("case two-row", two_row, "deviation", dev, flush=True)
        assert tr == two_row
        assert (dev < 1e-13) if two_row else (dev > 0.1)
        h32 = to_host(ctx.wilson_dslash(to_dev(psi), prec=ovl.F32))
        h16 = to_host(ctx.wilson_dslash(to_dev(psi), prec=ovl.HALF))
        ref = ora.hop(psi)
        assert max_rel_elem(h32, ref) < 2e-6
        assert max_rel_elem(h16, ref) < 5e-3
        if two_row:   # the same field through the full links
            ctx.set_option(ovl.OPT_TWO_ROW_LINKS, 0)
            assert not ctx.gauge_info()[1]
            f32 = to_host(ctx.wilson_dslash(to_dev(psi), prec=ovl.F32))
            assert max_rel_elem(f32, ref) < 2e-6 and rel(f32, h32) < 1e-6
            ctx.set_option(ovl.OPT_TWO_ROW_LINKS, 1)
            assert ctx.gauge_info()[1]
        ctx.close()


def _keys(prec, nf):
    # stencil launch table keys: (prec * 8 + epilogue) * 64 + field count
    return [(prec * 8 + e) * 64 + nf for e in range(4)]


@pytest.mark.parametrize("form", ["two_row", "full"])
@pytest.mark.parametrize("dims", [(8, 8, 8, 16), (4, 6, 2, 8)])
def test_every_launch_variant(dims, form):
    """Every stencil launch variant (traversal order, t-marching columns, lanes
    per site, LDS tiles with 1, 2, 4, 8 time slices per block with and without
    the tile's links in LDS, grouped XCD order of several fields' tiles, all
    fields of a tile in one lane with its links in registers), forced through
    the tuning table, for the plain stencil and K
    (two fields) and for the multi-shift CG's fused K^2 + sigma / dot launch
    (through sign(K)), in each storage precision, with the FP32 / FP16 links
    read as two rows (third rebuilt) and in full."""
    ovl = require_gpu()
    from oracle import krylov
    from oracle.zolotarev import Zolotarev
    print("case", dims, form, flush=True)
    U = synth.gauge_field(dims, 14, 0.3)
    ora = WilsonKernel(dims, U, 1.4)
    psi = np.stack([synth.gaussian_source(dims, 40), synth.z2_source(dims, 41)])
    z = Zolotarev(12, 0.3, 6.6)
    sref = krylov.SignFunction(ora, z)(psi[0], 1e-14)
    hop_ref = [ora.hop(p) for p in psi]
    k_ref = [ora.K(p) for p in psi]
    tol = {ovl.F64: 1e-14, ovl.F32: 2e-6, ovl.HALF: 5e-3}
    for prec in (ovl.F64, ovl.F32, ovl.HALF):
        variants = {ovl.F64: list(range(8)) + [12, 13, 14, 15], ovl.F32: list(range(20)),
                    ovl.HALF: list(range(22))}[prec]
        if dims == (4, 6, 2, 8):   # no split of x, y, z into 8 columns: 4, 5 and 21 unavailable
            variants = [v for v in variants if v not in (4, 5, 21)]
        for v in variants:
            ctx = ovl.Context(dims)
            ctx.gauge_load(to_dev(U))
            if form == "full":
                ctx.set_option(ovl.OPT_TWO_ROW_LINKS, 0)
            assert ctx.gauge_info()[1] == (form == "two_row")
            ctx.set_tuning({k: v for nf in (1, 2) for k in _keys(prec, nf)})
            h = to_host(ctx.wilson_dslash(to_dev(psi), prec=prec))
            k = to_host(ctx.kernel_K_apply(to_dev(psi), 1.4, prec=prec))
            for r in range(2):
                assert max_rel_elem(h[r], hop_ref[r]) < tol[prec], (prec, v)
                if prec == ovl.HALF:
                    assert rel(k[r], k_ref[r]) < 2e-3, (prec, v)
                else:
                    assert max_rel_elem(k[r], k_ref[r]) < tol[prec], (prec, v)
            zg = ovl.zolo_from(z.nz, z.a, z.b, z.delta, z.omega, z.sigma)
            eta = {ovl.F64: 1e-13, ovl.F32: 1e-6, ovl.HALF: 1e-2}[prec]
            s = to_host(ctx.sign(to_dev(psi[0]), 1.4, zg, eta, prec=prec)[0])
            assert rel(s, sref) < {ovl.F64: 1e-12, ovl.F32: 1e-5, ovl.HALF: 1e-2}[prec], (prec, v)
            assert ctx.tuning()[_keys(prec, 1)[2]] == v
            ctx.close()


def _sample_sites(dims, n, seed):
    V = int(np.prod(dims))
    L0, L1, L2 = dims[0], dims[1], dims[2]
    S3 = L0 * L1 * L2
    # lattice corners, the last site of the first x row, a time-slice boundary
    # and the faces of 8 x 8 x 4 tiles, then random sites
    fixed = [0, V - 1, L0 - 1, S3 - 1, S3, 7, 8, 7 * L0, 8 * L0, 3 * L0 * L1, 4 * L0 * L1]
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([fixed, rng.integers(0, V, n)]))


@pytest.mark.parametrize("prec", ["f32", "half"])
def test_dslash_32c64_sampled(prec):
    """The stand-alone 32^3 x 64 stencil as the benchmark launches it (links
    eps 0.25 seed 5, Gaussian source seed 7, autotuned launch variant): H psi
    on sampled sites against the oracle."""
    ovl = require_gpu()
    import torch
    dims = (32, 32, 32, 64)
    V = 32 * 32 * 32 * 64
    p = {"f32": ovl.F32, "half": ovl.HALF}[prec]
    ctx = ovl.Context(dims)
    Ud = torch.zeros((V, 4, 3, 3), dtype=torch.complex128, device="cuda")
    ctx.gauge_generate(5, 0.25, out=Ud)
    psi = ctx.source(ovl.SRC_GAUSS, seed=7)
    h = ctx.wilson_dslash(psi, p)
    print("case", dims, prec, "variant", ctx.tuning(), flush=True)
    sites = _sample_sites(dims, 400, 3)
    got = to_host(h)[sites]
    del h
    ref = WilsonKernel(dims, to_host(Ud), 1.4).hop_sites(to_host(psi), sites)
    assert max_rel_elem(got, ref) < {"f32": 2e-6, "half": 5e-3}[prec]
    ctx.close()


@pytest.mark.parametrize("prec", ["f32", "half"])
def test_dslash_24c48_12fields_sampled(prec):
    """Twelve fields in one stencil launch on 24^3 x 48 (the batched form of
    the eigSUMR workload, links eps 0.25 seed 3, autotuned launch variant):
    H psi_f on sampled sites of every field against the oracle."""
    ovl = require_gpu()
    import torch
    dims = (24, 24, 24, 48)
    V = 24 * 24 * 24 * 48
    p = {"f32": ovl.F32, "half": ovl.HALF}[prec]
    ctx = ovl.Context(dims)
    Ud = torch.zeros((V, 4, 3, 3), dtype=torch.complex128, device="cuda")
    ctx.gauge_generate(3, 0.25, out=Ud)
    B = torch.stack([ctx.source(ovl.SRC_GAUSS, seed=300 + f) for f in range(12)])
    h = ctx.wilson_dslash(B, p)
    print("case", dims, prec, "variant", ctx.tuning(), flush=True)
    sites = _sample_sites(dims, 120, 4)
    got = to_host(h)[:, sites]
    del h
    ora = WilsonKernel(dims, to_host(Ud), 1.4)
    Bh = to_host(B)
    for f in range(12):
        ref = ora.hop_sites(Bh[f], sites)
        assert max_rel_elem(got[f], ref) < {"f32": 2e-6, "half": 5e-3}[prec], f
    ctx.close()


@pytest.mark.parametrize("variant", [20, 21])
def test_dslash_24c48_12fields_multifield_variants(variant):
    """The multi-field FP16 stencils forced on twelve 24^3 x 48 fields (three
    groups of four: lexicographic tiles, and the XCD column order): H psi_f on
    sampled sites of every field against the oracle."""
    ovl = require_gpu()
    import torch
    dims = (24, 24, 24, 48)
    V = 24 * 24 * 24 * 48
    ctx = ovl.Context(dims)
    Ud = torch.zeros((V, 4, 3, 3), dtype=torch.complex128, device="cuda")
    ctx.gauge_generate(3, 0.25, out=Ud)
    ctx.set_tuning({_keys(ovl.HALF, 12)[0]: variant})
    B = torch.stack([ctx.source(ovl.SRC_GAUSS, seed=320 + f) for f in range(12)])
    print("case", dims, "half variant", variant, flush=True)
    h = ctx.wilson_dslash(B, ovl.HALF)
    assert ctx.tuning()[_keys(ovl.HALF, 12)[0]] == variant
    sites = _sample_sites(dims, 80, 5)
    got = to_host(h)[:, sites]
    del h
    ora = WilsonKernel(dims, to_host(Ud), 1.4)
    Bh = to_host(B)
    for f in range(12):
        ref = ora.hop_sites(Bh[f], sites)
        assert max_rel_elem(got[f], ref) < 5e-3, f
    ctx.close()
