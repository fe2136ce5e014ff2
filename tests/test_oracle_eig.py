"""Pins for the oracle's deflation (Sec. 4) and eigSUMR (Sec. 5, Algs. 5-6)
against dense linear algebra and exact identities."""
import numpy as np
import pytest

import synth
from oracle import eig, krylov
from oracle.lattice import WilsonKernel, g5, norm
from oracle.zolotarev import Zolotarev

MU = 0.05


@pytest.fixture(scope="module")
def tiny():
    dims = (2, 2, 2, 2)
    k = WilsonKernel(dims, synth.gauge_field(dims, 3, 0.6), 1.4)
    w, Q = np.linalg.eigh(k.dense("K"))
    n = k.V * 12
    G5 = np.kron(np.eye(k.V), np.kron(np.diag([1.0, 1, -1, -1]), np.eye(3)))
    D = 0.5 * (1 + MU) * np.eye(n) + 0.5 * (1 - MU) * G5 @ (Q @ np.diag(np.sign(w)) @ Q.conj().T)
    h, Y = np.linalg.eigh(G5 @ D)
    z = Zolotarev(16, np.abs(w).min(), np.abs(w).max())
    ov = krylov.Overlap(krylov.SignFunction(k, z), MU)
    return dict(dims=dims, k=k, D=D, G5=G5, h=h, Y=Y, ov=ov, shape=(k.V, 4, 3))


def test_rayleigh_ritz_on_invariant_subspace(tiny):
    """Alg. 6 on a non-orthogonal basis of an exact invariant subspace returns
    the exact eigenpairs of gamma_5 D, with theta = h^2 + 2 mu delta h."""
    rng = np.random.default_rng(1)
    idx = np.argsort(np.abs(tiny["h"]))[:6]
    Psi = tiny["Y"][:, idx]
    A = rng.normal(size=(6, 6)) + 1j * rng.normal(size=(6, 6))
    V = Psi @ A
    VD = tiny["D"] @ V
    v, vD, theta, C = eig.rayleigh_ritz(V, VD, 6, MU, 0.1)
    hs = tiny["h"][idx]
    assert np.allclose(np.sort(theta), np.sort(hs ** 2 + 2 * MU * 0.1 * hs), atol=1e-12)
    for i in range(6):
        hv = np.vdot(v[:, i], tiny["G5"] @ vD[:, i]).real
        assert np.linalg.norm(tiny["G5"] @ vD[:, i] - hv * v[:, i]) < 1e-11
        assert np.min(np.abs(hs - hv)) < 1e-12
    assert np.allclose(v.conj().T @ v, np.eye(6), atol=1e-12)


def test_deflation_exact_eigenvectors(tiny):
    """Sec. 4 with exact eigenvectors projects them out of the residual:
    r0 = b - D x0 is orthogonal to every gamma_5 psi_j."""
    idx = np.argsort(np.abs(tiny["h"]))[:8]
    vecs = [tiny["Y"][:, j].reshape(tiny["shape"]) for j in idx]
    dvecs = [(tiny["D"] @ tiny["Y"][:, j]).reshape(tiny["shape"]) for j in idx]
    d = eig.Deflation(vecs, dvecs)
    b = synth.gaussian_source(tiny["dims"], 3)
    x0, Dx0 = d.project(b)
    assert np.allclose(Dx0.reshape(-1), tiny["D"] @ x0.reshape(-1), atol=1e-12)
    r0 = b.reshape(-1) - tiny["D"] @ x0.reshape(-1)
    for v in vecs:
        assert abs(np.vdot(g5(v).reshape(-1), r0)) < 1e-12
    assert norm(r0) < norm(b)


def test_eigsumr_ritz_pairs_are_eigenpairs(tiny):
    """After calculating solves (Algs. 3, 2, 5, 6) each Ritz value lies within
    its true residual of an eigenvalue of gamma_5 D (Hermitian residual bound),
    and the solves reach the 1e-10 residual."""
    E = eig.EigSUMR(6, 24, MU)
    for s in range(2):
        b = synth.z2_source(tiny["dims"], 40 + s)
        res = eig.gmresr_eigsumr(tiny["ov"], b, 1e-10, 1e-3, E, calc=True)
        assert norm(b.reshape(-1) - tiny["D"] @ res.x.reshape(-1)) <= 1e-10 * norm(b)
    assert E.ndiag >= 2
    for v in E.V:
        vv = v.reshape(-1)
        hv = np.vdot(vv, tiny["G5"] @ tiny["D"] @ vv).real
        r = np.linalg.norm(tiny["G5"] @ tiny["D"] @ vv - hv * vv)
        assert np.min(np.abs(tiny["h"] - hv)) <= r + 1e-12
        assert r < 1e-2
    # deflated solve still converges to the right answer
    E.recompute(tiny["ov"])
    b = synth.z2_source(tiny["dims"], 50)
    res = eig.gmresr_eigsumr(tiny["ov"], b, 1e-10, 1e-3, E, calc=False)
    assert norm(b.reshape(-1) - tiny["D"] @ res.x.reshape(-1)) <= 1e-10 * norm(b)


def test_sign_accuracy_bound_shape():
    """Eq. (bound): chi = 1 for the first two diagonalisations, sqrt(n) after;
    the bound shrinks as (m - n) k grows."""
    E = eig.EigSUMR(4, 12, MU, eps=1e-4, krecalc=25)
    e0 = E.sign_accuracy()
    assert e0 == pytest.approx(2 * 1e-4 / (np.sqrt(8 * 25) * (1 - MU)))
    E2 = eig.EigSUMR(4, 44, MU, eps=1e-4, krecalc=25)
    assert E2.sign_accuracy() < e0
    E.ndiag = 2
    assert E.sign_accuracy() == pytest.approx(2 * e0)
