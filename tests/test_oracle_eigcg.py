"""Pins for the oracle's eigCG (Sec. 5 collection on the relCG middle solve,
Alg. 6 diagonalisation, the Sec. 5.1 cap on the sign accuracy) and the
spectral preconditioner it feeds (Sec. 4), against dense linear algebra with
the exact overlap operator."""
import numpy as np
import pytest

import synth
from oracle import eig, krylov
from oracle.lattice import norm
from test_oracle_cg import MU, DenseH


class ExactOverlap:
    """D[mu] as a dense matrix (the sign accuracy argument is recorded and
    otherwise ignored)."""

    def __init__(self, D, mu):
        self.D, self.mu, self.etas = D, mu, []

    def __call__(self, v, eta):
        self.etas.append(eta)
        return (self.D @ v.reshape(-1)).reshape(v.shape)


@pytest.fixture(scope="module")
def mid():
    return DenseH((4, 4, 2, 2), 2, 0.4)


@pytest.fixture(scope="module")
def run(mid):
    """Two calculating GMRESR(eigCG) solves (n = 8, m = 30) with the exact D."""
    ov = ExactOverlap(mid.D, MU)
    E = eig.EigCG(8, 30, MU)
    out = []
    for s in range(2):
        b = synth.z2_source(mid.dims, 20 + s)
        out.append((b, eig.gmresr_eigcg(ov, b, 1e-10, 1e-3, E, calc=True)))
    return ov, E, out


def test_collected_pairs_are_unit_vectors_and_their_images(mid, run):
    """Every held pair satisfies v^D = D v and ||v|| = 1 (the collection takes
    D w = gamma_5 H w and D H w = gamma_5 H H w from the CG's own products)."""
    _, E, out = run
    assert len(E.V) == E.n and E.ndiag >= 4
    for v, vd in zip(E.V, E.VD):
        assert abs(norm(v) - 1.0) < 1e-12
        assert norm(mid.D @ v.reshape(-1) - vd.reshape(-1)) < 1e-12
    for b, res in out:
        assert norm(b.reshape(-1) - mid.D @ res.x.reshape(-1)) <= 1e-10 * norm(b)


def test_collection_before_the_first_diagonalisation(mid):
    """Five CG iterations hold ten vectors (two per iteration, fewer than m):
    each of unit norm, with v^D = D v, and the pair of one iteration is
    (w, H w) for the iteration's direction w."""
    E = eig.EigCG(8, 30, MU)
    b = synth.z2_source(mid.dims, 31)
    krylov.cgne(lambda v, e: mid.apply_H(v), b, 1e-12, maxiter=5, on_iter=E.collect_cg)
    assert len(E.V) == 10 and E.ndiag == 0
    for i, (v, vd) in enumerate(zip(E.V, E.VD)):
        assert abs(norm(v) - 1.0) < 1e-12
        assert norm(mid.D @ v.reshape(-1) - vd.reshape(-1)) < 1e-12
    for i in range(0, 10, 2):
        hw = mid.apply_H(E.V[i])
        assert norm(hw / norm(hw) - E.V[i + 1]) < 1e-12


def test_ritz_values_reach_the_lowest_eigenvalues_of_H(mid, run):
    """After two solves the eight Ritz values of gamma_5 D equal its eight
    eigenvalues of smallest modulus (dense eigh) to 1e-5, with residual norms
    below 1e-2 (eigCG is a rough eigensolver, Sec. 6)."""
    _, E, _ = run
    h = np.linalg.eigvalsh(mid.H)
    want = np.sort(h[np.argsort(np.abs(h))][: E.n])
    vals, res = E.ritz()
    assert np.abs(np.sort(vals) - want).max() < 1e-5
    assert res.max() < 1e-2


def test_deflated_solve_reaches_the_exact_eigenvector_gain(mid, run):
    """A solve preconditioned with the collected vectors takes no more CG
    iterations than one preconditioned with the exact eight lowest
    eigenvectors of H^2 (plus a small slack), and at most 60 % of the
    undeflated count (Sec. 6: the CG deflation reaches its theoretical gain
    even with rough eigenvectors)."""
    ov, E, _ = run
    b = synth.z2_source(mid.dims, 7)
    plain = krylov.gmresr_cg(ov, b, 1e-10, 1e-3)
    psis, ritz = mid.low(8)
    exact = krylov.gmresr_cg(ov, b, 1e-10, 1e-3, precond=krylov.SpectralPreconditioner(psis, ritz))
    defl = eig.gmresr_eigcg(ov, b, 1e-10, 1e-3, E, calc=False)
    its = [sum(r.middle_iters) for r in (plain, exact, defl)]
    assert norm(b.reshape(-1) - mid.D @ defl.x.reshape(-1)) <= 1e-10 * norm(b)
    assert its[2] <= its[1] + 4 and its[2] <= 0.6 * its[0], its


def test_spectral_preconditioner_from_held_vectors(mid):
    """From exact eigenvectors of H^2 mixed by a random unitary (and their D
    images), the Rayleigh-Ritz construction recovers Sec. 4's preconditioner
    built from the eigenvectors themselves, as an operator."""
    n = 6
    psis, ritz = mid.low(n)
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)))
    P = np.stack([p.reshape(-1) for p in psis], axis=1) @ Q
    V = [P[:, i].reshape(mid.shape) for i in range(n)]
    VD = [(mid.D @ P[:, i]).reshape(mid.shape) for i in range(n)]
    a = eig.spectral_preconditioner(V, VD)
    b = krylov.SpectralPreconditioner(psis, ritz)
    x = synth.gaussian_source(mid.dims, 9)
    assert norm(a(x) - b(x)) < 1e-10 * norm(x)


def test_calculating_solves_respect_the_eigenvector_bound(mid):
    """While collecting, no CG sign call is looser than the Sec. 5.1 bound in
    force at the time, and the bound is tighter than the CG relaxation
    alone would ask for."""
    E = eig.EigCG(8, 30, MU)
    seen = []

    def cap():
        seen.append(E.sign_accuracy())
        return seen[-1]

    b = synth.z2_source(mid.dims, 30)
    eta_cg = []

    def H(v, eta):
        eta_cg.append(eta)
        return mid.apply_H(v)

    krylov.cgne(H, b, 1e-3, eps_A=1e-3, eta_cap=cap, on_iter=E.collect_cg)
    assert len(seen) > 0 and len(eta_cg) == 2 * len(seen) + 1
    for i, c in enumerate(seen):
        assert eta_cg[2 * i] <= c and eta_cg[2 * i + 1] <= c
    assert min(seen) < 1e-3
