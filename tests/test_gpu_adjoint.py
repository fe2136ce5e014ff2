"""GPU parity for the derivatives of S = Re(chi^H D[mu] psi): D^dagger chi and
the link gradient (derived from Sec. 1 eqs. 1, 2, 4 and Sec. 3 eq. 7) against
the oracle, whose formula is pinned by finite differences on the CPU."""
import numpy as np
import pytest

import synth
from oracle import adjoint
from oracle.lattice import norm
from oracle.zolotarev import Zolotarev
from gpu_util import require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu

RHO = 1.4


def _setup(ovl, dims, seed, eps, nz):
    U = synth.gauge_field(dims, seed, eps)
    z = Zolotarev(nz, 0.25, 8.0 - RHO)
    ctx = ovl.Context(dims)
    ctx.gauge_load(to_dev(U))
    zg = ovl.zolo_from(z.nz, z.a, z.b, z.delta, z.omega, z.sigma)
    return U, z, ctx, zg


@pytest.mark.parametrize("dims,nz", [((4, 4, 4, 4), 12), ((6, 4, 4, 8), 16)])
def test_adjoint_f64(dims, nz):
    ovl = require_gpu()
    mu = 0.05
    U, z, ctx, zg = _setup(ovl, dims, 9, 0.3, nz)
    psi = synth.gaussian_source(dims, 71)
    chi = synth.gaussian_source(dims, 72)
    dpsi, dU, st = ctx.overlap_adjoint(to_dev(psi), to_dev(chi), RHO, mu, zg, 1e-14)
    ref_psi = adjoint.psi_gradient(dims, U, RHO, z, mu, chi)
    ref_U = adjoint.link_gradient(dims, U, RHO, z, mu, psi, chi)
    assert norm(to_host(dpsi) - ref_psi) / norm(ref_psi) < 1e-11
    got = to_host(dU)
    assert norm(got - ref_U) / norm(ref_U) < 1e-11
    # element by element, relative to the largest entry
    assert np.abs(got - ref_U).max() <= 1e-11 * np.abs(ref_U).max()
    assert st.mscg_iters > 0


def test_adjoint_f64_8c16():
    """The 8^3 x 16 adjoint workload (links eps 0.25, seed 5, N_Z = 20, no
    exactly treated modes) in FP64 against the oracle."""
    ovl = require_gpu()
    dims, mu = (8, 8, 8, 16), 0.05
    U, z, ctx, zg = _setup(ovl, dims, 5, 0.25, 20)
    psi = synth.gaussian_source(dims, 105)
    chi = synth.gaussian_source(dims, 106)
    dpsi, dU, _ = ctx.overlap_adjoint(to_dev(psi), to_dev(chi), RHO, mu, zg, 1e-13)
    ref_U = adjoint.link_gradient(dims, U, RHO, z, mu, psi, chi, tol=1e-14)
    got = to_host(dU)
    assert norm(got - ref_U) / norm(ref_U) < 1e-10
    assert np.abs(got - ref_U).max() <= 1e-10 * np.abs(ref_U).max()
    ref_psi = adjoint.psi_gradient(dims, U, RHO, z, mu, chi, eta=1e-14)
    assert norm(to_host(dpsi) - ref_psi) / norm(ref_psi) < 1e-10


def test_adjoint_f32():
    """FP32 inversions and stencils, FP64 link accumulation: error of the
    single-precision solves (eta 1e-6) only."""
    ovl = require_gpu()
    dims, mu = (4, 4, 4, 8), 0.1
    U, z, ctx, zg = _setup(ovl, dims, 10, 0.3, 12)
    psi = synth.gaussian_source(dims, 73)
    chi = synth.z2_source(dims, 74)
    dpsi, dU, _ = ctx.overlap_adjoint(to_dev(psi), to_dev(chi), RHO, mu, zg, 1e-6, prec=ovl.F32)
    ref_U = adjoint.link_gradient(dims, U, RHO, z, mu, psi, chi)
    ref_psi = adjoint.psi_gradient(dims, U, RHO, z, mu, chi)
    assert norm(to_host(dU) - ref_U) / norm(ref_U) < 2e-5
    assert norm(to_host(dpsi) - ref_psi) / norm(ref_psi) < 2e-5


def test_adjoint_two_rhs_sum():
    """Two field pairs: D^dagger chi per field, link gradient summed."""
    ovl = require_gpu()
    dims, mu = (4, 4, 4, 4), 0.05
    U, z, ctx, zg = _setup(ovl, dims, 11, 0.3, 10)
    P = np.stack([synth.gaussian_source(dims, 80), synth.point_source(dims, 5, 1, 2)])
    C = np.stack([synth.gaussian_source(dims, 81), synth.gaussian_source(dims, 82)])
    dpsi, dU, _ = ctx.overlap_adjoint(to_dev(P), to_dev(C), RHO, mu, zg, 1e-14)
    ref = sum(adjoint.link_gradient(dims, U, RHO, z, mu, P[f], C[f]) for f in range(2))
    assert norm(to_host(dU) - ref) / norm(ref) < 1e-11
    for f in range(2):
        rp = adjoint.psi_gradient(dims, U, RHO, z, mu, C[f])
        assert norm(to_host(dpsi)[f] - rp) / norm(rp) < 1e-11


def test_autograd_function():
    """torch.autograd through the library: L = Re(chi^H D psi)."""
    ovl = require_gpu()
    import torch
    dims, mu = (4, 4, 4, 4), 0.05
    U, z, ctx, zg = _setup(ovl, dims, 12, 0.3, 10)
    psi = synth.gaussian_source(dims, 83)
    chi = synth.gaussian_source(dims, 84)
    Ut = to_dev(U).requires_grad_(True)
    pt = to_dev(psi).requires_grad_(True)
    y = ovl.OverlapFunction.apply(ctx, Ut, pt, RHO, mu, zg, 1e-14, ovl.F64)
    L = (to_dev(chi).conj() * y).sum().real
    L.backward()
    ref_U = adjoint.link_gradient(dims, U, RHO, z, mu, psi, chi)
    ref_psi = adjoint.psi_gradient(dims, U, RHO, z, mu, chi)
    assert norm(to_host(Ut.grad) - ref_U) / norm(ref_U) < 1e-11
    assert norm(to_host(pt.grad) - ref_psi) / norm(ref_psi) < 1e-11
    assert abs(float(L.detach()) - adjoint.action(dims, U, RHO, z, mu, psi, chi)) < 1e-10 * norm(psi) * norm(chi)
    del torch


def test_adjoint_rejects_low_modes():
    ovl = require_gpu()
    dims = (4, 4, 4, 4)
    U, z, ctx, zg = _setup(ovl, dims, 13, 0.3, 8)
    ctx.lowmodes_compute(RHO, 2, tol=1e-8)
    psi = to_dev(synth.gaussian_source(dims, 85))
    with pytest.raises(ovl.OvlError) as e:
        ctx.overlap_adjoint(psi, psi, RHO, 0.05, zg, 1e-10)
    assert e.value.code == -6
