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


# --- eq. (bound) of Sec. 5.1 as a sign accuracy -------------------------------


def _held_state(tiny, E, ts, ndiag, uv_hist):
    """Put n held pairs (v_i, D v_i) into E, each v_i an exact eigenvector of
    gamma_5 D mixed with a second one by t_i, so that its residual is known
    only through the dense operator; returns the true residuals."""
    h, Y, D, G5 = tiny["h"], tiny["Y"], tiny["D"], tiny["G5"]
    order = np.argsort(np.abs(h))
    vs, vds, res = [], [], []
    for i, t in enumerate(ts):
        v = (Y[:, order[i]] + t * Y[:, order[10 + i]]) / np.sqrt(1.0 + t * t)
        hv = G5 @ (D @ v)
        res.append(np.linalg.norm(hv - v * np.vdot(v, hv).real))
        vs.append(v.reshape(tiny["shape"]))
        vds.append((D @ v).reshape(tiny["shape"]))
    E.V, E.VD, E.shape = vs, vds, tiny["shape"]
    E.theta = np.zeros(len(ts))
    E.ndiag = ndiag
    E.uv_hist = list(uv_hist)
    return np.array(res)


def _target(eps, r0):
    """Eq. (targetdelta): the largest v^D error that keeps the residual gap below eps^2."""
    return np.sqrt(eps * eps + r0 * r0) - r0


def _unrelaxed_limit_ok(tiny, accuracy):
    """With one new vector per cycle, k = 1 and rotation entries of modulus one
    nothing in eq. (bound) is relaxed, so for the first two diagonalisations it
    is eq. (targetdelta) at the residual of the best converged eigenvector, and
    the sign accuracy is 2 ||delta^D|| / (1 - mu) (v^D = ((1+mu) v + (1-mu) U v)/2).
    The relaxation factors scale it by 1/sqrt((m - n) k) and by the inverse
    mean of max|UV| over the recent diagonalisations."""
    eps, n = 1e-3, 4
    ok = True
    E = eig.EigSUMR(n, n + 1, MU, eps=eps, krecalc=1)
    ok &= accuracy(E) == pytest.approx(2 * eps / (1 - MU), rel=1e-12)      # nothing held: r0 = 0
    for ndiag in (1, 2):
        E = eig.EigSUMR(n, n + 1, MU, eps=eps, krecalc=1)
        res = _held_state(tiny, E, [0.2, 0.05, 0.1, 0.3], ndiag - 1, [1.0])
        ok &= accuracy(E) == pytest.approx(2 * _target(eps, res.min()) / (1 - MU), rel=1e-10)
        E = eig.EigSUMR(n, n + 4, MU, eps=eps, krecalc=9)
        res = _held_state(tiny, E, [0.2, 0.05, 0.1, 0.3], ndiag - 1, [0.5, 2.0])
        ok &= accuracy(E) == pytest.approx(2 * _target(eps, res.min()) / (1 - MU) / 6.0 / 1.25, rel=1e-10)
    return bool(ok)


def test_sign_accuracy_unrelaxed_limit_is_targetdelta(tiny):
    assert _unrelaxed_limit_ok(tiny, lambda E: E.sign_accuracy())


def _planted(chi_always=False, worst_residual=False, no_gamma5=False):
    def acc(E):
        if len(E.V) < E.n or E.theta is None:
            r0 = 0.0
        else:
            rs = []
            for v, vD in zip(E.V[:E.n], E.VD[:E.n]):
                g = vD if no_gamma5 else g5(vD)
                rs.append(norm(g - np.vdot(v.reshape(-1), g.reshape(-1)).real * v))
            r0 = max(rs) if worst_residual else min(rs)
        chi = np.sqrt(E.n) if (chi_always or E.ndiag >= 2) else 1.0
        uv = np.mean(E.uv_hist) if E.uv_hist else 1.0
        dd = chi * _target(E.eps, r0) / (np.sqrt((E.m - E.n) * E.krecalc) * uv)
        return 2.0 * dd / (1.0 - E.mu)
    return acc


@pytest.mark.parametrize("mistake", ["chi_always", "worst_residual", "no_gamma5"])
def test_sign_accuracy_limit_rejects_planted(tiny, mistake):
    """The limit check fails for sqrt(n) applied from the start, for the worst
    instead of the best converged residual, and for a residual without gamma_5."""
    assert not _unrelaxed_limit_ok(tiny, _planted(**{mistake: True}))


def _rotation_blocks(tiny, E, solves=2, block=None):
    """Run calculating solves; at every diagonalisation measure the rotation
    C (new eigenvectors = old basis x C) by least squares and return pairs
    (recorded max|UV|, measured max over new eigenvectors i < n and new Krylov
    vectors j >= n')."""
    out = []
    orig = E.diagonalise

    def diag():
        if len(E.V) <= E.n:
            return orig()
        nprev = E.n if E.ndiag > 0 else 0
        B = eig._mat(E.V)
        nd = E.ndiag
        orig()
        if E.ndiag > nd:
            C = np.linalg.lstsq(B, eig._mat(E.V[:E.n]), rcond=None)[0]
            out.append((E.uv_hist[-1], np.abs(C[nprev:, :]).max()))
    E.diagonalise = diag
    for s in range(solves):
        eig.gmresr_eigsumr(tiny["ov"], synth.z2_source(tiny["dims"], 60 + s), 1e-10, 1e-3, E, calc=True)
    return out


def test_uv_block_is_new_krylov_vectors(tiny):
    """max|UV| of eq. (bound) is taken over the rotation entries that carry the
    new Krylov vectors (j >= n') into the new eigenvectors (i < n)."""
    pairs = _rotation_blocks(tiny, eig.EigSUMR(6, 24, MU))
    assert len(pairs) >= 3
    for rec, meas in pairs:
        assert rec == pytest.approx(meas, rel=1e-6)


class _OldBlock(eig.EigSUMR):
    """Planted mistake: max|UV| over the held (old) rows instead of the new ones."""
    def diagonalise(self):
        if len(self.V) <= self.n:
            return
        nprev = self.n if self.ndiag > 0 else 0
        v, vD, theta, C = eig.rayleigh_ritz(eig._mat(self.V), eig._mat(self.VD), self.n, self.mu, self.delta)
        self.V = [v[:, i].reshape(self.shape) for i in range(self.n)]
        self.VD = [vD[:, i].reshape(self.shape) for i in range(self.n)]
        self.theta = theta
        self.ndiag += 1
        self.uv_hist = (self.uv_hist + [float(np.abs(C[: max(nprev, 1), :]).max())])[-10:]


def test_uv_block_rejects_planted(tiny):
    pairs = _rotation_blocks(tiny, _OldBlock(6, 24, MU))
    assert any(abs(rec - meas) > 1e-3 * meas for rec, meas in pairs)


class _Injected:
    """D[mu] whose sign function errs by exactly eta ||psi|| in a random
    direction: the worst error a sign call at accuracy eta may make."""
    def __init__(self, tiny, seed):
        self.mu, self.t = MU, tiny
        self.S = tiny["G5"] @ (2.0 * tiny["D"] - (1 + MU) * np.eye(tiny["D"].shape[0])) / (1 - MU)
        self.rng = np.random.default_rng(seed)

    def U(self, psi, eta):
        e = self.rng.normal(size=psi.size) + 1j * self.rng.normal(size=psi.size)
        e *= eta * norm(psi) / np.linalg.norm(e)
        return g5((self.S @ psi.reshape(-1) + e).reshape(psi.shape))

    def __call__(self, psi, eta):
        return 0.5 * (1 + self.mu) * psi + 0.5 * (1 - self.mu) * self.U(psi, eta)


def _new_vector_error(tiny, E, seed=7, solves=2):
    """For the first two diagonalisations: sqrt(k) times the largest error the
    new Krylov vectors of the cycle carry into a held v^D, over the target of
    eq. (targetdelta) at the residual the bound used (k cycles of such errors
    adding up as a random walk, the relaxation argument of Sec. 5.1)."""
    D = tiny["D"]
    ratios = []
    orig = E.diagonalise

    def diag():
        if len(E.V) <= E.n:
            return orig()
        r0 = 0.0 if (E.theta is None or len(E.V) < E.n) else float(E.ritz()[1].min())
        nprev = E.n if E.ndiag > 0 else 0
        B, BD = eig._mat(E.V), eig._mat(E.VD)
        err = BD - D @ B
        nd = E.ndiag
        orig()
        if E.ndiag > nd and E.ndiag <= 2:
            C = np.linalg.lstsq(B, eig._mat(E.V[:E.n]), rcond=None)[0]
            new = err[:, nprev:] @ C[nprev:, :]
            ratios.append(np.sqrt(E.krecalc) * np.linalg.norm(new, axis=0).max() / _target(E.eps, r0))
    E.diagonalise = diag
    ov = _Injected(tiny, seed)
    for s in range(solves):
        eig.gmresr_eigsumr(ov, synth.z2_source(tiny["dims"], 40 + s), 1e-10, 1e-3, E, calc=True)
    return ratios


@pytest.mark.parametrize("cfg", [dict(n=6, m=24, krecalc=25), dict(n=6, m=24, krecalc=4),
                                 dict(n=4, m=16, krecalc=25)])
def test_bound_keeps_new_vector_errors_within_targetdelta(tiny, cfg):
    """With every sign call erring by as much as its accuracy allows, the
    error that a cycle's new vectors bring into the eigenvectors stays within
    eq. (targetdelta) over the first two diagonalisations (chi = 1)."""
    ratios = _new_vector_error(tiny, eig.EigSUMR(cfg["n"], cfg["m"], MU, eps=1e-4, krecalc=cfg["krecalc"]))
    assert len(ratios) == 2
    assert max(ratios) < 0.7


class _NoRelaxDivisor(eig.EigSUMR):
    """Planted mistake: the sqrt((m - n) k) divisor left out."""
    def sign_accuracy(self):
        return eig.EigSUMR.sign_accuracy(self) * np.sqrt((self.m - self.n) * self.krecalc)


def test_new_vector_errors_reject_planted(tiny):
    ratios = _new_vector_error(tiny, _NoRelaxDivisor(6, 24, MU, eps=1e-4, krecalc=25))
    assert max(ratios) > 1.0


# --- block collection (several right-hand sides' Krylov vectors, one Alg. 6) ----


def test_canonical_rayleigh_ritz_on_dependent_basis(tiny):
    """With an exactly repeated direction V^H V is singular (Cholesky fails);
    the canonical orthonormalisation gives the Ritz pairs of the basis
    without the repeats."""
    rng = np.random.default_rng(2)
    idx = np.argsort(np.abs(tiny["h"]))[:6]
    V = tiny["Y"][:, idx] @ (rng.normal(size=(6, 6)) + 1j * rng.normal(size=(6, 6)))
    V2 = np.concatenate([V, V[:, :3]], axis=1)
    with pytest.raises(np.linalg.LinAlgError):
        eig.rayleigh_ritz(V2, tiny["D"] @ V2, 4, MU, 0.1)
    _, _, th, _ = eig.rayleigh_ritz(V, tiny["D"] @ V, 4, MU, 0.1)
    v2, vD2, th2, _ = eig.rayleigh_ritz(V2, tiny["D"] @ V2, 4, MU, 0.1, canonical=True)
    assert np.allclose(th2, th, atol=1e-12)
    assert np.allclose(vD2, tiny["D"] @ v2, atol=1e-10)
    assert np.allclose(v2.conj().T @ v2, np.eye(4), atol=1e-10)


def _krylov_pairs(tiny, b, steps):
    """The Alg. 1 basis (q, U q) of `steps` SUMR iterations with the exact U."""
    S = tiny["G5"] @ (2.0 * tiny["D"] - (1 + MU) * np.eye(tiny["D"].shape[0])) / (1 - MU)
    pairs = []
    krylov.sumr(lambda v, eta: g5((S @ v.reshape(-1)).reshape(v.shape)), (1 - MU) / (1 + MU),
                (2.0 / (1 + MU)) * b, 1e-300, maxiter=steps,
                on_step=lambda q, u: pairs.append((q.copy(), 0.5 * (1 - MU) * u + 0.5 * (1 + MU) * q)))
    return pairs


def test_block_collection_ritz_values_interlace(tiny):
    """Krylov vectors of two right-hand sides in one basis: each of the n lowest
    Ritz values of M over the union is at most the same Ritz value over either
    sequence alone (Courant-Fischer on nested subspaces), and with exact images
    the Ritz pairs are exact Rayleigh-Ritz pairs of gamma_5 D."""
    pa = _krylov_pairs(tiny, synth.z2_source(tiny["dims"], 90), 14)
    pb = _krylov_pairs(tiny, synth.z2_source(tiny["dims"], 91), 14)
    n = 5

    def ritz(pairs):
        V = eig._mat([p[0] for p in pairs])
        VD = eig._mat([p[1] for p in pairs])
        return eig.rayleigh_ritz(V, VD, n, MU, 0.1, canonical=True)
    _, _, ta, _ = ritz(pa)
    _, _, tb, _ = ritz(pb)
    v, vD, tab, _ = ritz(pa + pb)
    assert np.all(tab <= ta + 1e-12) and np.all(tab <= tb + 1e-12)
    assert np.allclose(vD, tiny["D"] @ v, atol=1e-10)
    for i in range(n):
        hv = np.vdot(v[:, i], tiny["G5"] @ vD[:, i]).real
        r = np.linalg.norm(tiny["G5"] @ vD[:, i] - hv * v[:, i])
        assert np.min(np.abs(tiny["h"] - hv)) <= r + 1e-12
