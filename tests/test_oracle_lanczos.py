"""Pins for the oracle's two-pass Lanczos sign function (the Lanczos approach
to sign(K) cited in Sec. 1 after eq. 4) against the dense spectral
definition sign(K) = Q sign(Lambda) Q^dagger (Sec. 1, eq. 4)."""
import numpy as np
import pytest

import synth
from oracle import krylov, lanczos
from oracle.lattice import WilsonKernel, norm


class Dense:
    def __init__(self, dims, seed, eps):
        self.dims = dims
        self.k = WilsonKernel(dims, synth.gauge_field(dims, seed, eps), 1.4)
        self.w, self.Q = np.linalg.eigh(self.k.dense("K"))

    def sign(self, psi):
        return (self.Q @ (np.sign(self.w) * (self.Q.conj().T @ psi.reshape(-1)))).reshape(psi.shape)


@pytest.fixture(scope="module", params=[((2, 2, 2, 2), 1, 0.5), ((4, 4, 2, 2), 2, 0.4)])
def dense(request):
    return Dense(*request.param)


@pytest.mark.parametrize("eta", [1e-4, 1e-8, 1e-12])
def test_lanczos_sign_vs_dense(dense, eta):
    """The result is within eta ||psi|| of the exact sign function (no
    rational approximation error), with and without exactly treated modes."""
    psi = synth.gaussian_source(dense.dims, 5)
    lmax = np.abs(dense.w).max()
    r = lanczos.lanczos_sign(dense.k, psi, eta, lmax)
    assert r.converged
    assert norm(r.out - dense.sign(psi)) <= eta * norm(psi)
    order = np.argsort(np.abs(dense.w))[:4]
    low = krylov.LowModes(dense.w[order], dense.Q[:, order].T.reshape(4, *dense.k.shape))
    r2 = lanczos.lanczos_sign(dense.k, psi, eta, lmax, low)
    assert norm(r2.out - dense.sign(psi)) <= eta * norm(psi)
    assert r2.iters <= r.iters


def test_lanczos_sign_squared_is_one(dense):
    psi = synth.z2_source(dense.dims, 6)
    lmax = np.abs(dense.w).max()
    s1 = lanczos.lanczos_sign(dense.k, psi, 1e-12, lmax).out
    s2 = lanczos.lanczos_sign(dense.k, s1, 1e-12, lmax).out
    assert norm(s2 - psi) <= 1e-10 * norm(psi)


def test_lanczos_sign_rejects_planted(dense, monkeypatch):
    """T^{-1} e_1 in place of T^{-1/2} e_1 (the sign function of K^2 instead
    of K's) fails the dense comparison."""
    psi = synth.gaussian_source(dense.dims, 5)
    lmax = np.abs(dense.w).max()

    def inv_e1(alpha, beta):
        k = len(alpha)
        T = np.diag(np.asarray(alpha)) + (np.diag(beta[: k - 1], 1) + np.diag(beta[: k - 1], -1) if k > 1 else 0)
        e = np.zeros(k)
        e[0] = 1.0
        return np.linalg.solve(T, e)
    monkeypatch.setattr(lanczos, "_inv_sqrt_e1", inv_e1)
    r = lanczos.lanczos_sign(dense.k, psi, 1e-8, lmax)
    assert norm(r.out - dense.sign(psi)) > 1e-2 * norm(psi)
