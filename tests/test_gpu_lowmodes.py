"""GPU kernel low modes (set-up of the exactly treated part of sign(K),
Sec. 1 after eq. 4, Sec. 3) against dense eigendecomposition, and at the
16^3 x 32 workload through properties the oracle checks."""
import numpy as np
import pytest

import synth
from oracle import krylov
from oracle.lattice import WilsonKernel, norm
from oracle.zolotarev import Zolotarev
from gpu_util import rel, require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu


def test_lowmodes_vs_dense():
    ovl = require_gpu()
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 1, 0.3)
    k = WilsonKernel(dims, U, 1.4)
    w = np.linalg.eigvalsh(k.dense("K"))
    ref = w[np.argsort(np.abs(w))][:8]
    ctx = ovl.Context(dims)
    ctx.gauge_load(to_dev(U))
    ev, lmax = ctx.lowmodes_compute(1.4, 8, tol=1e-11)
    assert np.allclose(np.abs(ev), np.abs(ref), rtol=0, atol=1e-10)
    assert lmax >= np.abs(w).max()
    vecs = to_host(ctx.lowmodes_get())
    G = vecs.reshape(8, -1).conj() @ vecs.reshape(8, -1).T
    assert np.allclose(G, np.eye(8), atol=1e-12)
    for lam, v in zip(ev, vecs):
        assert norm(k.K(v) - lam * v) <= 2e-11


def test_lowmodes_full_size_properties():
    """16^3 x 32, 10 modes: oracle-checked eigen-residuals, orthonormality, and
    no mode below the Zolotarev interval left out: with the modes projected,
    sign(K)^2 psi = psi to the approximation error (a missed |lambda| < a would
    break it)."""
    ovl = require_gpu()
    dims = (16, 16, 16, 32)
    V = int(np.prod(dims))
    ctx = ovl.Context(dims)
    Ud = to_dev(np.zeros((V, 4, 3, 3)))
    ctx.gauge_generate(2, 0.25, out=Ud)
    ev, lmax = ctx.lowmodes_compute(1.4, 10, tol=1e-10)
    print("evals", ev, flush=True)
    vecs = to_host(ctx.lowmodes_get())
    k = WilsonKernel(dims, to_host(Ud), 1.4)
    for lam, v in zip(ev, vecs):
        assert norm(k.K(v) - lam * v) <= 1e-9
    G = vecs.reshape(10, -1).conj() @ vecs.reshape(10, -1).T
    assert np.allclose(G, np.eye(10), atol=1e-11)
    a = np.abs(ev).max()
    z = ovl.zolotarev_coeffs(20, a, lmax)
    psi = synth.gaussian_source(dims, 102)
    s1, _ = ctx.sign(to_dev(psi), 1.4, z, 1e-12)
    s2, _ = ctx.sign(s1, 1.4, z, 1e-12)
    assert rel(to_host(s2), psi) < 1e-10
