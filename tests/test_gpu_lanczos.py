"""GPU parity for the two-pass Lanczos sign function (the Lanczos approach
to sign(K) cited in Sec. 1 after eq. 4): against the dense spectral sign on
4^4, and on the multi-block 8^3 x 16 lattice against the oracle's Zolotarev
sign function evaluated to 1e-13 (whose approximation error there is below
1e-13), with and without exactly treated kernel modes."""
import numpy as np
import pytest

import synth
from oracle import krylov
from oracle.lattice import WilsonKernel, norm
from oracle.zolotarev import Zolotarev
from gpu_util import require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu
RHO = 1.4


@pytest.mark.parametrize("eta", [1e-6, 1e-10])
def test_lanczos_sign_vs_dense_4c4(eta):
    ovl = require_gpu()
    dims = (4, 4, 4, 4)
    U = synth.gauge_field(dims, 1, 0.3)
    w, Q = np.linalg.eigh(WilsonKernel(dims, U, RHO).dense("K"))
    ctx = ovl.Context(dims)
    ctx.gauge_load(to_dev(U))
    zg = ovl.zolotarev_coeffs(16, np.abs(w).min(), np.abs(w).max())
    psi = np.stack([synth.gaussian_source(dims, 3), synth.z2_source(dims, 4)])
    out, st = ctx.sign_lanczos(to_dev(psi), RHO, zg, eta)
    out = to_host(out)
    for f in range(2):
        ref = (Q @ (np.sign(w) * (Q.conj().T @ psi[f].reshape(-1)))).reshape(psi[f].shape)
        err = norm(out[f] - ref) / norm(psi[f])
        print("case 4^4 eta", eta, "field", f, "error", err, "steps", st.mscg_iters, flush=True)
        assert err <= eta
    ctx.close()


@pytest.mark.parametrize("nlow", [0, 6])
def test_lanczos_sign_8c16_vs_oracle(nlow):
    ovl = require_gpu()
    dims = (8, 8, 8, 16)
    U = synth.gauge_field(dims, 5, 0.25)
    ctx = ovl.Context(dims)
    ctx.gauge_load(to_dev(U))
    k = WilsonKernel(dims, U, RHO)
    low = None
    if nlow:
        ev, _ = ctx.lowmodes_compute(RHO, nlow, tol=1e-11)
        a = max(abs(e) for e in ev)
        low = krylov.LowModes(ev, to_host(ctx.lowmodes_get()))
    else:
        lo, _, _ = ctx.kernel_interval(RHO)
        a = 0.95 * lo
    z = Zolotarev(20, a, 8.0 - RHO)
    zg = ovl.zolo_from(z.nz, z.a, z.b, z.delta, z.omega, z.sigma)
    psi = synth.gaussian_source(dims, 11)
    out, st = ctx.sign_lanczos(to_dev(psi), RHO, zg, 1e-10)
    ref = krylov.SignFunction(k, z, low)(psi, 1e-13)
    err = norm(to_host(out) - ref) / norm(psi)
    print("case 8^3x16 nlow", nlow, "error", err, "Lanczos steps", st.mscg_iters, "Delta", z.delta, flush=True)
    assert err <= 1e-10 + 2 * z.delta
    ctx.close()
