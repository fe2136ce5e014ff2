"""Pins for the oracle's multi-shift CG, sign function, overlap operator,
SUMR and GMRESR (paper Secs. 1-3, Algs. 1-3) against dense linear algebra
and exact identities."""
import numpy as np
import pytest

import synth
from oracle import krylov
from oracle.lattice import WilsonKernel, g5, norm
from oracle.zolotarev import Zolotarev


class Dense:
    def __init__(self, dims, seed, eps, rho=1.4):
        self.dims = dims
        self.k = WilsonKernel(dims, synth.gauge_field(dims, seed, eps), rho)
        Kd = self.k.dense("K")
        self.w, self.Q = np.linalg.eigh(Kd)
        n = Kd.shape[0]
        self.G5 = np.kron(np.eye(self.k.V), np.kron(np.diag([1.0, 1, -1, -1]), np.eye(3)))
        self.n = n

    def fn(self, f, psi):
        v = psi.reshape(-1)
        return (self.Q @ (f(self.w) * (self.Q.conj().T @ v))).reshape(psi.shape)

    def sign_dense(self):
        return self.Q @ np.diag(np.sign(self.w)) @ self.Q.conj().T


@pytest.fixture(scope="module")
def small():
    return Dense((2, 2, 2, 2), 1, 0.5)


@pytest.fixture(scope="module")
def mid():
    return Dense((4, 4, 2, 2), 2, 0.4)


def test_mscg_shift_residuals(mid):
    z = Zolotarev(12, np.abs(mid.w).min(), np.abs(mid.w).max())
    b = synth.gaussian_source(mid.dims, 3)
    tol = np.full(z.nz, 1e-11)
    res = krylov.multishift_cg(mid.k.K2s, z.sigma, b, tol)
    for s, x in zip(z.sigma, res.x):
        r = norm(b - mid.k.K2s(x, s)) / norm(b)
        assert r <= 5e-11
        xd = mid.fn(lambda w: 1.0 / (w * w + s), b)
        assert norm(x - xd) / norm(xd) < 1e-9
    # larger shifts converge in fewer iterations
    order = np.argsort(z.sigma)
    assert np.all(np.diff(res.shift_iters[order]) <= 0)


@pytest.mark.parametrize("fixture", ["small", "mid"])
def test_rational_sign_vs_dense(fixture, request):
    """eps(K) psi from the multi-shift CG equals Q eps(Lambda) Q^dagger psi:
    the rational function is applied exactly up to the inversion error."""
    d = request.getfixturevalue(fixture)
    z = Zolotarev(16, np.abs(d.w).min(), np.abs(d.w).max())
    sgn = krylov.SignFunction(d.k, z)
    psi = synth.gaussian_source(d.dims, 4)
    out = sgn(psi, 1e-13)
    assert norm(out - d.fn(z, psi)) / norm(psi) < 1e-12
    assert norm(out - d.fn(np.sign, psi)) / norm(psi) < 1e-12 + 2 * z.delta


def test_lowmode_projection_vs_dense(mid):
    """Exact treatment of the n lowest |lambda| modes: the Zolotarev interval
    starts at |lambda_{n+1}|... here a = the n-th smallest |lambda| (Sec. 3),
    and sign(K) matches the spectral definition (Sec. 1, eq. 4)."""
    nlow = 6
    order = np.argsort(np.abs(mid.w))
    low = order[:nlow]
    evecs = mid.Q[:, low].T.reshape(nlow, mid.k.V, 4, 3)
    lm = krylov.LowModes(mid.w[low], evecs)
    a = np.abs(mid.w[order[nlow - 1]])
    z = Zolotarev(16, a, np.abs(mid.w).max())
    sgn = krylov.SignFunction(mid.k, z, lm)
    psi = synth.gaussian_source(mid.dims, 5)
    out = sgn(psi, 1e-13)
    assert norm(out - mid.fn(np.sign, psi)) / norm(psi) < 1e-12 + 2 * z.delta


def test_sign_squared_and_ginsparg_wilson(mid):
    """sign(K)^2 = 1 and D[0] gamma_5 (1 - 2 D[0]) + gamma_5 D[0] = 0 (Sec. 1, eq. 3)
    to within the approximation error."""
    z = Zolotarev(16, np.abs(mid.w).min(), np.abs(mid.w).max())
    sgn = krylov.SignFunction(mid.k, z)
    psi = synth.gaussian_source(mid.dims, 6)
    tol = 1e-12 + 4 * z.delta
    assert norm(sgn(sgn(psi, 1e-13), 1e-13) - psi) / norm(psi) < tol
    D0 = krylov.Overlap(sgn, 0.0)
    t = D0(g5(psi), 1e-13)
    gw = t - 2.0 * D0(g5(D0(psi, 1e-13)), 1e-13) + g5(D0(psi, 1e-13))
    assert norm(gw) / norm(psi) < tol


def test_overlap_spectrum_on_circle(small):
    """gamma_5 sign(K) is unitary, so the eigenvalues of D[mu] lie on the circle
    of centre (1 + mu)/2 and radius (1 - mu)/2; gamma_5 D is Hermitian (Sec. 1)."""
    mu = 0.05
    z = Zolotarev(16, np.abs(small.w).min(), np.abs(small.w).max())
    ov = krylov.Overlap(krylov.SignFunction(small.k, z), mu)
    n = small.n
    D = np.empty((n, n), complex)
    e = np.zeros((small.k.V, 4, 3), complex)
    for j in range(n):
        e.reshape(-1)[j] = 1.0
        D[:, j] = ov(e, 1e-14).reshape(-1)
        e.reshape(-1)[j] = 0.0
    ev = np.linalg.eigvals(D)
    assert np.allclose(np.abs(ev - 0.5 * (1 + mu)), 0.5 * (1 - mu), atol=1e-11)
    H = small.G5 @ D
    assert np.allclose(H, H.conj().T, atol=1e-11)


def test_sumr_equals_gmres(mid):
    """Alg. 2 (zeta = 1) is a short-recurrence form of GMRES: iterate j equals the
    GMRES iterate of the same Krylov dimension; its residual estimate
    rho |tau_hat| equals the true residual; the basis q_j (Alg. 1) is orthonormal."""
    S = mid.sign_dense()
    Uu = mid.G5 @ S
    mu = 0.05
    rho = (1 - mu) / (1 + mu)
    A = np.eye(mid.n) + rho * Uu
    b = synth.gaussian_source(mid.dims, 7)
    qs = []
    full = krylov.sumr(lambda v, eta: (Uu @ v.reshape(-1)).reshape(v.shape), rho, b, 1e-300,
                       maxiter=25, on_step=lambda q, u: qs.append(q.reshape(-1).copy()))
    Q = np.array(qs).T
    assert np.allclose(Q.conj().T @ Q, np.eye(Q.shape[1]), atol=1e-12)
    for m in (1, 3, 10, 25):
        r = krylov.sumr(lambda v, eta: (Uu @ v.reshape(-1)).reshape(v.shape), rho, b, 1e-300,
                        maxiter=m)
        xg = krylov.gmres_dense(A, b.reshape(-1), m)
        assert norm(r.x.reshape(-1) - xg) / norm(xg) < 1e-12
        true = norm(b.reshape(-1) - A @ r.x.reshape(-1))
        assert r.history[-1] == pytest.approx(true, rel=1e-10)
    assert full.iters == 25


def test_gmresr_vs_dense_solve(mid):
    """GMRESR(relSUMR) (Alg. 3 around Alg. 2) reaches ||b - D x|| <= 1e-10 ||b||
    and agrees with a dense LU solve to the freedom that residual leaves."""
    mu = 0.05
    z = Zolotarev(16, np.abs(mid.w).min(), np.abs(mid.w).max())
    ov = krylov.Overlap(krylov.SignFunction(mid.k, z), mu)
    Dd = 0.5 * (1 + mu) * np.eye(mid.n) + 0.5 * (1 - mu) * mid.G5 @ mid.sign_dense()
    for b in (synth.point_source(mid.dims), synth.z2_source(mid.dims, 8)):
        res = krylov.gmresr_sumr(ov, b, 1e-10, 1e-3)
        xd = np.linalg.solve(Dd, b.reshape(-1))
        true = norm(b.reshape(-1) - Dd @ res.x.reshape(-1)) / norm(b)
        assert true <= 1e-10
        assert norm(res.x.reshape(-1) - xd) / norm(xd) <= 2e-10 / mu
        assert 1 <= res.steps <= 10


# --- the sign accuracy -> multi-shift stopping rule (Sec. 3, eq. 7 and the
# text after it: the sign error is the larger of Delta and the inversion
# error of x^2 + sigma_l) --------------------------------------------------------

SHIFT_ETAS = (1e-2, 1e-4, 1e-6)


def _per_shift_worst(d, z, psi, eta, tol):
    """max_l  omega_l ||K (x_l - x_l*)|| N_Z / (eta ||psi||), x_l* from the dense
    eigendecomposition: the share of each pole in the inversion error of
    eps(K) psi = K sum_l omega_l x_l, in units of its budget eta ||psi|| / N_Z."""
    res = krylov.multishift_cg(d.k.K2s, z.sigma, psi, tol)
    pv = d.Q.conj().T @ psi.reshape(-1)
    worst = 0.0
    for l in range(z.nz):
        xs = (d.Q @ (pv / (d.w * d.w + z.sigma[l]))).reshape(psi.shape)
        e = z.omega[l] * norm(d.k.K(res.x[l] - xs))
        worst = max(worst, e * z.nz / (eta * norm(psi)))
    return worst


@pytest.mark.parametrize("fixture", ["small", "mid"])
@pytest.mark.parametrize("nz", [12, 20])
def test_sign_accuracy_bounds_inversion_error(fixture, nz, request):
    """A sign call at accuracy eta keeps the error of the rational function
    within eta ||psi|| (against the dense Q eps(Lambda) Q^dagger psi), and each
    pole's share within eta ||psi|| / N_Z, for eta from the relaxed 1e-2 down
    to 1e-6, on 2^4 and 4x4x2x2."""
    d = request.getfixturevalue(fixture)
    z = Zolotarev(nz, np.abs(d.w).min(), np.abs(d.w).max())
    psi = synth.gaussian_source(d.dims, 4)
    exact = d.fn(z, psi)
    for eta in SHIFT_ETAS:
        out = krylov.SignFunction(d.k, z)(psi, eta)
        assert norm(out - exact) <= eta * norm(psi)
        assert _per_shift_worst(d, z, psi, eta, krylov.shift_tolerances(z, eta)) <= 1.0


PLANTED_SHIFT_RULES = {
    "budget not split over the poles": lambda z, eta: eta * 2.0 * np.sqrt(z.sigma) / z.omega,
    "sigma for sqrt(sigma)": lambda z, eta: eta * 2.0 * z.sigma / (z.nz * z.omega),
    "four times looser": lambda z, eta: eta * 8.0 * np.sqrt(z.sigma) / (z.nz * z.omega),
}


@pytest.mark.parametrize("name", sorted(PLANTED_SHIFT_RULES))
def test_sign_accuracy_pin_rejects_planted_rules(name, small, mid):
    """The per-pole budget check above fails for plausible mistakes in the
    stopping rule, on at least one lattice and accuracy."""
    rule = PLANTED_SHIFT_RULES[name]
    worst = 0.0
    for d in (small, mid):
        for nz in (12, 20):
            z = Zolotarev(nz, np.abs(d.w).min(), np.abs(d.w).max())
            psi = synth.gaussian_source(d.dims, 4)
            for eta in SHIFT_ETAS:
                worst = max(worst, _per_shift_worst(d, z, psi, eta, rule(z, eta)))
    assert worst > 1.2, f"planted rule '{name}' not detected ({worst:.2f})"
