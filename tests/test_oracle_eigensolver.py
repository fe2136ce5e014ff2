"""Pins for the oracle's standalone eigSUMR eigensolver (Sec. 6, eigenvector
calculation: Alg. 1 basis, Alg. 5 collection, Alg. 6, restarts) and its
three-set re-diagonalisation (Sec. 5), against dense linear algebra with the
exact overlap operator."""
import numpy as np
import pytest

import synth
from oracle import eig
from oracle.lattice import norm
from test_oracle_cg import MU, DenseH

DELTA = 0.1


class ExactOverlap:
    """D[mu] = (1 + mu)/2 + (1 - mu)/2 U with the exact dense unitary U."""

    def __init__(self, D, mu):
        self.D, self.mu = D, mu
        self.Um = (2.0 * D - (1.0 + mu) * np.eye(D.shape[0])) / (1.0 - mu)
        self.etas = []

    def __call__(self, v, eta):
        return (self.D @ v.reshape(-1)).reshape(v.shape)

    def U(self, v, eta):
        self.etas.append(eta)
        return (self.Um @ v.reshape(-1)).reshape(v.shape)


@pytest.fixture(scope="module")
def mid():
    return DenseH((4, 4, 2, 2), 2, 0.4)


def _lowest(mid, n):
    """The n eigenvalues h of gamma_5 D whose eigenvectors are lowest in
    D^+ D + 2 mu delta gamma_5 D (there h^2 + 2 mu delta h), ascending."""
    h = np.linalg.eigvalsh(mid.H)
    return np.sort(h[np.argsort(h ** 2 + 2 * MU * DELTA * h)][:n])


def test_unitary_is_exact(mid):
    ov = ExactOverlap(mid.D, MU)
    assert np.abs(ov.Um.conj().T @ ov.Um - np.eye(ov.Um.shape[0])).max() < 1e-13


def test_eigensolver_converges_to_the_dense_eigenpairs(mid):
    """With the exact U the eigensolver reaches residuals <= 1e-3 for six
    eigenvectors; their Ritz values are the dense eigenvalues selected by
    D^+ D + 2 mu delta gamma_5 D to 1e-5, and each vector's residual is the
    true ||gamma_5 D v - h v||."""
    ov = ExactOverlap(mid.D, MU)
    E = eig.EigSUMR(6, 30, MU, delta=DELTA, eps=1e-3)
    starts = []
    collect = E.collect

    def spy(q, u):   # every collected q with the eigenvectors held at the time
        starts.append((q.copy(), [v.copy() for v in E.V[:E.n]]))
        collect(q, u)

    E.collect = spy
    runs = eig.eigsumr_eigensolver(ov, synth.z2_source(mid.dims, 5), E, restarts=20)
    # each later run starts from a unit vector orthogonal to the eigenvectors
    for r in runs[:-1]:
        q, vs = starts[r.applies]
        assert abs(norm(q) - 1.0) < 1e-12
        assert max(abs(np.vdot(v.reshape(-1), q.reshape(-1))) for v in vs) < 1e-12
    assert runs[-1].resid.max() <= 1e-3 and len(runs) < 20
    assert np.abs(np.sort(runs[-1].ritz) - _lowest(mid, 6)).max() < 1e-5
    for v, h, r in zip(E.V, *E.ritz()):
        vv = v.reshape(-1)
        assert abs(norm(vv) - 1.0) < 1e-10
        assert abs(np.linalg.norm(mid.H @ vv - h * vv) - r) < 1e-10
    # residuals fall from run to run (the three-set step never loses ground)
    mr = [r.resid.max() for r in runs]
    assert all(b <= a * 1.05 for a, b in zip(mr, mr[1:])), mr


def test_three_identical_sets_reduce_to_one(mid):
    """Three copies of the same exact eigenvector set (differently mixed) span
    only n directions: the canonical orthonormalisation drops the rest and
    returns the exact eigenpairs (Cholesky of V^H V would fail here)."""
    n = 6
    h, Y = np.linalg.eigh(mid.H)
    idx = np.argsort(h ** 2 + 2 * MU * DELTA * h)[:n]
    rng = np.random.default_rng(3)
    sets = []
    for _ in range(3):
        Q, _ = np.linalg.qr(rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)))
        P = Y[:, idx] @ Q
        sets.append(([P[:, i].reshape(mid.shape) for i in range(n)],
                     [(mid.D @ P[:, i]).reshape(mid.shape) for i in range(n)]))
    with pytest.raises(np.linalg.LinAlgError):
        V = np.stack([v.reshape(-1) for vs, _ in sets for v in vs], axis=1)
        np.linalg.cholesky(V.conj().T @ V)
    v, vD, theta = eig.rediagonalise_sets(sets, n, MU, DELTA)
    th = np.sort(theta)
    want = np.sort(h[idx] ** 2 + 2 * MU * DELTA * h[idx])
    assert np.abs(th - want).max() < 1e-12
    for i in range(n):
        vi = v[:, i]
        hv = np.vdot(vi, mid.H @ vi).real
        assert np.linalg.norm(mid.H @ vi - hv * vi) < 1e-10


def test_union_never_raises_the_ritz_values(mid):
    """Rayleigh-Ritz over the union of three sets gives each of the n lowest
    values at most what any one set gives alone (Cauchy interlacing), so the
    three-set step can only improve the estimates."""
    n = 4
    rng = np.random.default_rng(8)
    h, Y = np.linalg.eigh(mid.H)
    idx = np.argsort(h ** 2 + 2 * MU * DELTA * h)[:n]
    sets = []
    for k in range(3):
        P = Y[:, idx] + 0.3 * (rng.normal(size=(Y.shape[0], n)) + 1j * rng.normal(size=(Y.shape[0], n))) / np.sqrt(
            Y.shape[0])
        P, _ = np.linalg.qr(P)
        sets.append(([P[:, i].reshape(mid.shape) for i in range(n)],
                     [(mid.D @ P[:, i]).reshape(mid.shape) for i in range(n)]))
    _, _, th_all = eig.rediagonalise_sets(sets, n, MU, DELTA)
    for s in sets:
        _, _, th_one = eig.rediagonalise_sets([s], n, MU, DELTA)
        assert np.all(np.sort(th_all) <= np.sort(th_one) + 1e-14)
