"""Pins for the oracle's deflated CGNE with the spectral preconditioner and
GMRESR(relCG) (paper Sec. 4 and its CGNE algorithm, Sec. 3 relaxation, Alg. 3)
against dense linear algebra."""
import numpy as np
import pytest

import synth
from oracle import krylov
from oracle.lattice import WilsonKernel, norm
from oracle.zolotarev import Zolotarev

MU = 0.05


class DenseH:
    """Dense H = gamma_5 D[mu] with the exact sign function, and the oracle's
    sign function (Zolotarev + multi-shift CG) on the same lattice."""

    def __init__(self, dims, seed, eps, nz=16):
        self.dims = dims
        self.k = WilsonKernel(dims, synth.gauge_field(dims, seed, eps), 1.4)
        w, Q = np.linalg.eigh(self.k.dense("K"))
        n = w.size
        self.shape = (self.k.V, 4, 3)
        G5 = np.kron(np.eye(self.k.V), np.kron(np.diag([1.0, 1, -1, -1]), np.eye(3)))
        S = Q @ np.diag(np.sign(w)) @ Q.conj().T
        self.D = 0.5 * (1 + MU) * np.eye(n) + 0.5 * (1 - MU) * G5 @ S
        self.H = G5 @ self.D
        self.h2, self.E = np.linalg.eigh(self.H @ self.H)   # ascending eigenvalues of H^2
        self.z = Zolotarev(nz, np.abs(w).min(), np.abs(w).max())
        self.sign = krylov.SignFunction(self.k, self.z)

    def apply_H(self, v, eta=None):
        return (self.H @ v.reshape(-1)).reshape(v.shape)

    def low(self, n, noise=0.0, seed=0):
        """The n lowest eigenvectors of H^2 (orthonormalised after an optional
        random perturbation of relative size noise) and their Ritz values."""
        E = self.E[:, :n].copy()
        if noise:
            rng = np.random.default_rng(seed)
            E = E + noise * (rng.normal(size=E.shape) + 1j * rng.normal(size=E.shape)) / np.sqrt(2 * E.shape[0])
            E, _ = np.linalg.qr(E)
        H2 = self.H @ self.H
        ritz = [float(np.vdot(E[:, i], H2 @ E[:, i]).real) for i in range(n)]
        return [E[:, i].reshape(self.shape) for i in range(n)], ritz


@pytest.fixture(scope="module")
def tiny():
    return DenseH((2, 2, 2, 2), 3, 0.5)


@pytest.fixture(scope="module")
def mid():
    return DenseH((4, 4, 2, 2), 2, 0.4)


def _op_matrix(f, n, shape):
    cols = []
    for j in range(n):
        e = np.zeros(n, complex)
        e[j] = 1.0
        cols.append(f(e.reshape(shape)).reshape(-1))
    return np.array(cols).T


def test_preconditioner_moves_low_modes_to_c2(tiny):
    """Exact eigenvectors: the n smallest eigenvalues of Hhat^-1 H^2 Hhat^-1
    become c^2 = 3/4, every other eigenvalue of H^2 stays."""
    n = 6
    psis, ritz = tiny.low(n)
    P = krylov.SpectralPreconditioner(psis, ritz)
    N = tiny.H.shape[0]
    Pm = _op_matrix(P, N, tiny.shape)
    M = Pm @ tiny.H @ tiny.H @ Pm
    got = np.sort(np.linalg.eigvalsh(0.5 * (M + M.conj().T)))
    want = np.sort(np.concatenate([np.full(n, 0.75), tiny.h2[n:]]))
    assert np.abs(got - want).max() < 1e-12
    assert np.allclose(Pm, Pm.conj().T, atol=1e-14)   # Hermitian, so CG applies


def test_cgne_returns_inverse_of_H(tiny):
    """The closing x = H Hhat^-1 x_j makes CGNE return H^-1 b, with and
    without the preconditioner; deflating the lowest modes cuts iterations."""
    b = synth.gaussian_source(tiny.dims, 5)
    ref = np.linalg.solve(tiny.H, b.reshape(-1)).reshape(b.shape)
    r0 = krylov.cgne(tiny.apply_H, b, 1e-12)
    psis, ritz = tiny.low(12)
    r1 = krylov.cgne(tiny.apply_H, b, 1e-12, precond=krylov.SpectralPreconditioner(psis, ritz))
    for r in (r0, r1):
        assert norm(tiny.apply_H(r.x) - b) <= 1e-10 * norm(b)
        assert norm(r.x - ref) <= 1e-9 * norm(ref)
    assert r1.iters < r0.iters


def test_cgne_deflation_gain_grows_with_n(mid):
    """Deflating more of the lowest eigenvectors of H^2 exactly never costs
    CG iterations, and 16 of them at least halve the count on this lattice
    (its condition number drops about 11-fold)."""
    b = synth.z2_source(mid.dims, 7)
    its = []
    for n in (0, 4, 8, 16):
        pre = None
        if n:
            psis, ritz = mid.low(n)
            pre = krylov.SpectralPreconditioner(psis, ritz)
        r = krylov.cgne(mid.apply_H, b, 1e-10, precond=pre)
        assert norm(mid.apply_H(r.x) - b) <= 1e-9 * norm(b)
        its.append(r.iters)
    assert all(a >= b_ for a, b_ in zip(its, its[1:])), its
    assert its[0] >= 2 * its[-1], its


@pytest.mark.parametrize("noise", [0.0, 0.1])
def test_gmresr_cg_vs_dense_solve(mid, noise):
    """GMRESR(relCG) with the oracle's relaxed sign function: true residual
    <= 1e-10 against the dense D, the dense LU solution, and -- even with
    eigenvectors perturbed by 10 % (relative residuals ||r_i|| / m_i from
    0.16 up to several) -- about half the CG iterations of the solve without
    the preconditioner (Sec. 4: the spectral preconditioner needs only rough
    eigenvectors)."""
    b = synth.point_source(mid.dims)
    ov = krylov.Overlap(mid.sign, MU)
    psis, ritz = mid.low(16, noise=noise, seed=1)
    res0 = krylov.gmresr_cg(ov, b, 1e-10, 1e-3)
    res1 = krylov.gmresr_cg(ov, b, 1e-10, 1e-3, precond=krylov.SpectralPreconditioner(psis, ritz))
    xd = np.linalg.solve(mid.D, b.reshape(-1))
    for res in (res0, res1):
        assert norm(b.reshape(-1) - mid.D @ res.x.reshape(-1)) <= 1e-10 * norm(b)
        assert norm(res.x.reshape(-1) - xd) <= 2e-10 / MU * norm(xd)
    assert 2 * sum(res1.middle_iters) <= sum(res0.middle_iters) + 10
