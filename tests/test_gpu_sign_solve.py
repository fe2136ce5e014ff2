"""GPU parity: sign(K) by multi-shift CG with exact low modes (Sec. 1 eq. 4,
Sec. 3 eq. 7), the overlap operator (Sec. 1 eq. 1) and the GMRESR(relSUMR)
solve (Algs. 1-3) against the oracle on small lattices."""
import numpy as np
import pytest

import synth
from oracle import krylov
from oracle.lattice import WilsonKernel, norm
from oracle.zolotarev import Zolotarev
from gpu_util import rel, require_gpu, to_dev, to_host

pytestmark = pytest.mark.gpu


class Setup:
    def __init__(self, dims, seed, eps, nz, nlow=0, rho=1.4):
        self.dims = dims
        self.U = synth.gauge_field(dims, seed, eps)
        self.k = WilsonKernel(dims, self.U, rho)
        w, Q = np.linalg.eigh(self.k.dense("K"))
        self.w, self.Q = w, Q
        order = np.argsort(np.abs(w))
        self.low = None
        a = np.abs(w).min()
        if nlow:
            idx = order[:nlow]
            self.low = krylov.LowModes(w[idx], Q[:, idx].T.reshape(nlow, self.k.V, 4, 3))
            a = np.abs(w[order[nlow - 1]])
        self.z = Zolotarev(nz, a, np.abs(w).max())
        self.sign = krylov.SignFunction(self.k, self.z, self.low)


@pytest.fixture(scope="module")
def c1():
    # the plain-method configuration: 4^4, eps 0.3, seed 1, rho 1.4, N_Z = 16
    return Setup((4, 4, 4, 4), 1, 0.3, 16)


def _ctx(ovl, s):
    ctx = ovl.Context(s.dims)
    ctx.gauge_load(to_dev(s.U))
    if s.low is not None:
        ctx.lowmodes_set(list(s.low.evals), to_dev(s.low.evecs))
    zg = ovl.zolo_from(s.z.nz, s.z.a, s.z.b, s.z.delta, s.z.omega, s.z.sigma)
    return ctx, zg


def test_sign_f64(c1):
    ovl = require_gpu()
    ctx, zg = _ctx(ovl, c1)
    psi = np.stack([synth.gaussian_source(c1.dims, 21), synth.z2_source(c1.dims, 22)])
    out, st = ctx.sign(to_dev(psi), 1.4, zg, 1e-13)
    got = to_host(out)
    for r in range(2):
        ref = c1.sign(psi[r], 1e-13)
        assert rel(got[r], ref) < 1e-12
    assert st.mscg_iters > 0


def test_sign_lowmodes_f64():
    ovl = require_gpu()
    s = Setup((4, 4, 2, 6), 5, 0.5, 12, nlow=6)
    ctx, zg = _ctx(ovl, s)
    psi = synth.gaussian_source(s.dims, 23)
    got = to_host(ctx.sign(to_dev(psi), 1.4, zg, 1e-13)[0])
    assert rel(got, s.sign(psi, 1e-13)) < 1e-12


def test_sign_f32_error(c1):
    ovl = require_gpu()
    ctx, zg = _ctx(ovl, c1)
    psi = synth.gaussian_source(c1.dims, 24)
    got = to_host(ctx.sign(to_dev(psi), 1.4, zg, 1e-5, prec=ovl.F32)[0])
    ref = c1.sign(psi, 1e-14)
    # asked-for accuracy 1e-5 plus FP32 rounding of the accumulated result
    assert rel(got, ref) < 1e-5


def test_overlap_f64(c1):
    ovl = require_gpu()
    ctx, zg = _ctx(ovl, c1)
    psi = synth.gaussian_source(c1.dims, 25)
    got = to_host(ctx.overlap(to_dev(psi), 1.4, 0.05, zg, 1e-13)[0])
    ref = krylov.Overlap(c1.sign, 0.05)(psi, 1e-13)
    assert rel(got, ref) < 1e-12


def test_zero_source(c1):
    ovl = require_gpu()
    ctx, zg = _ctx(ovl, c1)
    psi = np.zeros((c1.k.V, 4, 3), complex)
    got = to_host(ctx.sign(to_dev(psi), 1.4, zg, 1e-10)[0])
    assert np.all(got == 0)


@pytest.mark.parametrize("ladder", ["f64", "mixed"])
def test_solve_c1(c1, ladder):
    """GMRESR(relSUMR) on the 4^4 plain-method case: true residual <= 1e-10
    with the oracle's FP64 D, and agreement with a dense LU solve."""
    ovl = require_gpu()
    ctx, zg = _ctx(ovl, c1)
    mu = 0.05
    b = synth.point_source(c1.dims)
    p = ovl.solver_defaults(rho=1.4, mu=mu, tol=1e-10, eta_tilde=1e-3,
                            f32_threshold=(1e-6 if ladder == "mixed" else 10.0))
    x, st, code = ctx.solve(to_dev(b), zg, p)
    assert code == 0
    x = to_host(x)
    D = krylov.Overlap(c1.sign, mu)
    assert norm(b - D(x, 1e-15)) / norm(b) <= 1e-10
    n = c1.k.V * 12
    G5 = np.kron(np.eye(c1.k.V), np.kron(np.diag([1.0, 1, -1, -1]), np.eye(3)))
    S = c1.Q @ np.diag(np.sign(c1.w)) @ c1.Q.conj().T
    Dd = 0.5 * (1 + mu) * np.eye(n) + 0.5 * (1 - mu) * G5 @ S
    xd = np.linalg.solve(Dd, b.reshape(-1))
    assert rel(x, xd) <= 2e-10 / mu
    s = st[0]
    assert s.gmresr_steps >= 1 and s.sumr_iters > 0
    if ladder == "mixed":
        assert s.sign_calls[1] > 0          # single-precision sign calls used
    print("stats", s.as_dict())


def test_sign_half_error(c1):
    ovl = require_gpu()
    ctx, zg = _ctx(ovl, c1)
    psi = synth.gaussian_source(c1.dims, 26)
    got = to_host(ctx.sign(to_dev(psi), 1.4, zg, 1e-2, prec=ovl.HALF)[0])
    ref = c1.sign(psi, 1e-14)
    assert rel(got, ref) < 1e-2


def test_solve_c1_half_ladder(c1):
    """Sign calls with accuracy >= 3e-3 in FP16 storage, >= 1e-6 in FP32, the
    rest in FP64: still a true residual <= 1e-10."""
    ovl = require_gpu()
    ctx, zg = _ctx(ovl, c1)
    b = synth.z2_source(c1.dims, 31)
    p = ovl.solver_defaults(rho=1.4, mu=0.05, tol=1e-10, eta_tilde=1e-3, f32_threshold=1e-6,
                            half_threshold=3e-3)
    x, st, code = ctx.solve(to_dev(b), zg, p)
    assert code == 0
    D = krylov.Overlap(c1.sign, 0.05)
    assert norm(b - D(to_host(x), 1e-15)) / norm(b) <= 1e-10
    assert st[0].sign_calls[2] > 0
    print("half ladder stats", st[0].as_dict())


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_graph_replay_identical(c1, prec):
    """The multi-shift CG replays graphs of four iterations after the first
    chunk; with graphs off every kernel is launched on its own.  Same kernels,
    same order, fixed-order reductions: bitwise the same result and count."""
    ovl = require_gpu()
    eta = {0: 1e-12, 1: 1e-6, 2: 1e-2}[prec]
    psi = to_dev(synth.gaussian_source(c1.dims, 27))
    out = []
    for graphs in (True, False, True):
        ctx, zg = _ctx(ovl, c1)
        ctx.set_option(ovl.OPT_AUTOTUNE, 0)   # one launch variant: the same tile sums everywhere
        ctx.set_option(ovl.OPT_GRAPHS, graphs)
        s, st = ctx.sign(psi, 1.4, zg, eta, prec=prec)
        s2, st2 = ctx.sign(psi, 1.4, zg, eta, prec=prec)   # a second call replays the cached graph
        out.append((to_host(s), st.mscg_iters, to_host(s2)))
        ctx.close()
    for s, n, s2 in out[1:]:
        assert n == out[0][1]
        assert np.array_equal(s, out[0][0]) and np.array_equal(s2, out[0][0])


def test_solve_graphs_off_matches(c1):
    """A whole mixed-precision solve with and without graphs: same iterate."""
    ovl = require_gpu()
    b = to_dev(synth.gaussian_source(c1.dims, 28))
    p = ovl.solver_defaults(rho=1.4, mu=0.05, tol=1e-10, eta_tilde=1e-3, f32_threshold=1e-6,
                            half_threshold=3e-3)
    xs = []
    for graphs in (True, False):
        ctx, zg = _ctx(ovl, c1)
        ctx.set_option(ovl.OPT_AUTOTUNE, 0)
        ctx.set_option(ovl.OPT_GRAPHS, graphs)
        x, st, code = ctx.solve(b, zg, p)
        assert code == 0
        xs.append((to_host(x), st[0].mscg_iters))
        ctx.close()
    assert xs[0][1] == xs[1][1] and np.array_equal(xs[0][0], xs[1][0])


def test_solve_adaptive_poles(c1):
    """With the adaptive option every sign call inside the solver takes the
    fewest Zolotarev poles whose error Delta(n) on the same interval is at
    most a quarter of the accuracy asked for (Sec. 3: the sign error is
    bounded by the larger of Delta and the inversion error).  The solve
    still reaches a true residual <= 1e-10 with the oracle's FP64 D, with
    fewer multi-shift iterations than with all 16 poles in every call."""
    ovl = require_gpu()
    b = synth.z2_source(c1.dims, 32)
    p = ovl.solver_defaults(rho=1.4, mu=0.05, tol=1e-10, eta_tilde=1e-3, f32_threshold=1e-6,
                            half_threshold=3e-3)
    D = krylov.Overlap(c1.sign, 0.05)
    iters = {}
    for adaptive in (False, True):
        ctx, zg = _ctx(ovl, c1)
        ctx.set_option(ovl.OPT_ADAPTIVE_NZ, adaptive)
        x, st, code = ctx.solve(to_dev(b), zg, p)
        assert code == 0
        assert norm(b - D(to_host(x), 1e-15)) / norm(b) <= 1e-10
        iters[adaptive] = st[0].mscg_iters
        ctx.close()
    print("multi-shift iterations, fixed / adaptive poles:", iters)
    assert iters[True] < iters[False]


def test_solve_outer_accuracy_printed(c1):
    """The GMRESR outer products at the accuracy Alg. 3 prints: each step may
    move the true residual from the computed one by ||A u - c|| |alpha| / ||c||
    < eps ||b|| ||u|| / ||c|| <= eps ||b|| / mu (the eigenvalues of D(mu) are at
    least mu in modulus), so after k steps it is within eps ||b|| (1 + k / mu);
    with the default eps ||b|| / 4 it stays <= 1e-10.  The printed bound asks
    for no more FP64 work than the default."""
    ovl = require_gpu()
    ctx, zg = _ctx(ovl, c1)
    mu, tol = 0.05, 1e-10
    b = synth.point_source(c1.dims)
    p = ovl.solver_defaults(rho=1.4, mu=mu, tol=tol, eta_tilde=1e-3, f32_threshold=1e-6)
    D = krylov.Overlap(c1.sign, mu)
    res, f64_calls = {}, {}
    for mode in (0, 1):
        ctx.set_option(ovl.OPT_OUTER_PRINTED, mode)
        x, st, code = ctx.solve(to_dev(b), zg, p)
        assert code == 0
        s = st[0]
        assert s.computed_relres <= tol
        res[mode] = norm(b - D(to_host(x), 1e-15)) / norm(b)
        f64_calls[mode] = s.dslash_calls[0]
        k = s.gmresr_steps
    assert res[0] <= tol
    assert res[1] <= tol * (1.0 + k / mu)
    assert f64_calls[1] <= f64_calls[0]
    print("true residuals", res, "FP64 stencil calls", f64_calls)
