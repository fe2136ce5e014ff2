"""Oracle: deflation of the middle solve (Sec. 4), eigSUMR (Sec. 5,
Algs. 5 and 6, the relaxation bound of Sec. 5.1) and eigCG (Sec. 5) on the
relCG middle solve with the spectral preconditioner of Sec. 4.

TEST INFRASTRUCTURE ONLY.

Readings where the paper is silent or garbled (also listed in the design notes):
* Alg. 6 writes the update as (V U^T v); it is read as the Rayleigh-Ritz
  vectors  v_new = V R^{-1} Y[:, :n]  (same for v^D), with E = V^H V = R^H R
  (Cholesky, R upper) and Y the ascending eigenvectors of R^{-H} M R^{-1}.
* The eigenvector residual of Alg. 6 is taken as
  r_i = gamma_5 v^D_i - v_i (v_i, gamma_5 v^D_i)  (Sec. 5.1 definition).
* The pair-splitting constant delta (Sec. 5) is not given: delta = 0.1.
* Eq. (bound): chi multiplies the whole numerator,
  ||delta^D|| < chi (sqrt(eps^2 + r0^2) - r0) / (sqrt((m - n) k) <max|UV|>),
  chi = 1 for the first two diagonalisations and sqrt(n) after; max|UV| is
  taken over new eigenvectors i < n and new Krylov vectors n <= j < m of the
  rotation R^{-1} Y, averaged over the last ten diagonalisations (1 before
  any); the sign accuracy follows as eta = 2 ||delta^D|| / (1 - mu).
* When both the inversion and the eigenvector bound apply, the stricter
  (smaller) sign accuracy is used (Sec. 5.1, third strategy).
* The subspace size m is not given for the inversions: m = n + 40 unless
  set; v^D is recomputed accurately every k diagonalisations and when the
  eigenvector phase ends.
* Standalone eigSUMR eigensolver (Sec. 6, eigenvector calculation): each
  run generates the Alg. 1 basis from its start vector with Alg. 5
  collection, and ends after 24 diagonalisations, when | ||q|| - 1 | > 0.1 or
  |gamma| >= 1, or when every held eigenvector's residual is at most the
  run's target; at the end of a run Alg. 6 closes it, v^D is recomputed
  accurately, and one more Rayleigh-Ritz runs over the current eigenvectors
  and those kept at the previous two restarts (the three-set
  re-diagonalisation of Sec. 5, which the calculating solves of the
  inverters also run once each, at the end of the solve, since every new
  right-hand side restarts the Krylov space).  Those sets overlap more and more as the
  vectors converge, so that Rayleigh-Ritz orthonormalises canonically
  (eigenvectors of V^H V with eigenvalues below 1e-10 of the largest are
  dropped) instead of by Cholesky.  The next run starts from the last q,
  orthogonalised (twice) against the eigenvectors and normalised; its target
  is the larger of the final accuracy and a tenth of the largest residual at
  the restart (the paper sets each run's tolerance below the residual it
  expects next, without a rule).
* eigCG (Sec. 5 describes it in words only): every CG iteration adds two
  basis vectors, the preconditioned direction w = Hhat^{-1} p and H w (the
  paper keeps both p and gamma_5 D p), each scaled to unit norm, with their
  images D w = gamma_5 (H w) and D (H w) = gamma_5 (H H w) taken from the
  two H applications the iteration makes anyway; Alg. 6 (with the same
  pair-splitting M) diagonalises them, at k = m and at the end of each
  middle solve, and the Sec. 5.1 bound caps the CG's sign accuracy as for
  eigSUMR.  The spectral preconditioner of a middle solve is built from the
  eigenvectors held when it starts and stays fixed until it ends (a CG needs
  a fixed operator; GMRESR absorbs the change between middle solves).  Its
  vectors are the Rayleigh-Ritz vectors of H^2 = D^+ D in the span of the n
  held eigenvectors, so that they are orthonormal as Sec. 4's formula needs.
"""
import numpy as np

from .lattice import dot, g5, norm


def _mat(vs):
    return np.stack([v.reshape(-1) for v in vs], axis=1)


class Deflation:
    """Sec. 4: rotate psi' = psi Y so that (psi'_i, gamma_5 D psi'_j) is
    diagonal, then x0 = sum_j alpha_j psi'_j with
    alpha_j = (D psi'_j, b) / (D psi'_j, D psi'_j); D x0 = sum_j alpha_j D psi'_j."""

    def __init__(self, vecs, dvecs):
        P = _mat(vecs)
        DP = _mat(dvecs)
        shape = vecs[0].shape
        H = P.conj().T @ g5(DP.T.reshape((-1,) + shape)).reshape(len(vecs), -1).T
        H = 0.5 * (H + H.conj().T)
        h, Y = np.linalg.eigh(H)
        self.h = h
        self.P = P @ Y
        self.DP = DP @ Y
        self.shape = shape

    def x0(self, b):
        bb = b.reshape(-1)
        num = self.DP.conj().T @ bb
        den = np.einsum("ij,ij->j", self.DP.conj(), self.DP).real
        alpha = num / den
        return (self.P @ alpha).reshape(self.shape)

    def project(self, b):
        """(x0, D x0)."""
        bb = b.reshape(-1)
        alpha = (self.DP.conj().T @ bb) / np.einsum("ij,ij->j", self.DP.conj(), self.DP).real
        return (self.P @ alpha).reshape(self.shape), (self.DP @ alpha).reshape(self.shape)


def rayleigh_ritz(V, VD, n, mu, delta, canonical=False, cut=1e-10):
    """Alg. 6 on the columns of V (basis) and VD (their images under D):
    returns (v, vD, theta, C) with v = V C, vD = VD C, C = R^{-1} Y[:, :n];
    with canonical, R^{-1} is replaced by B = W_k diag(l_k^{-1/2}) over the
    eigenpairs (l, W) of V^H V above cut times the largest (the basis of a
    block collection, whose Krylov sequences are nearly dependent)."""
    E = V.conj().T @ V
    E = 0.5 * (E + E.conj().T)
    N = V.shape[0]
    if canonical:
        lam, W = np.linalg.eigh(E)
        keep = lam > cut * lam.max()
        B = W[:, keep] / np.sqrt(lam[keep])
        G5VD = (g5(VD.T.reshape((VD.shape[1], N // 12, 4, 3))).reshape(VD.shape[1], -1)).T
        M = VD.conj().T @ VD + 2.0 * mu * delta * (V.conj().T @ G5VD)
        G = B.conj().T @ (0.5 * (M + M.conj().T)) @ B
        theta, Y = np.linalg.eigh(0.5 * (G + G.conj().T))
        C = B @ Y[:, :n]
        return V @ C, VD @ C, theta[:n], C
    L = np.linalg.cholesky(E)            # E = L L^H, R = L^H
    R = L.conj().T
    # gamma_5 in canonical layout: spins 2, 3 negated
    G5VD = (g5(VD.T.reshape((VD.shape[1], N // 12, 4, 3))).reshape(VD.shape[1], -1)).T
    M = VD.conj().T @ VD + 2.0 * mu * delta * (V.conj().T @ G5VD)
    M = 0.5 * (M + M.conj().T)
    Rinv = np.linalg.inv(R)
    G = Rinv.conj().T @ M @ Rinv
    G = 0.5 * (G + G.conj().T)
    theta, Y = np.linalg.eigh(G)
    C = Rinv @ Y[:, :n]
    return V @ C, VD @ C, theta[:n], C


class EigSUMR:
    """Alg. 5 inside the SUMR iteration plus Alg. 6 at k = m.

    collect(q, u): v_k = q, v^D_k = (1 - mu)/2 u + (1 + mu)/2 q, u = U q."""

    def __init__(self, n, m, mu, delta=0.1, eps=1e-4, krecalc=25, canonical=False):
        assert m > n
        self.canonical = canonical
        self.n, self.m, self.mu, self.delta = n, m, float(mu), float(delta)
        self.eps, self.krecalc = eps, krecalc
        self.V, self.VD = [], []
        self.ndiag = 0
        self.uv_hist = []
        self.theta = None
        self.shape = None
        self.kept = []   # eigenvector sets (V, VD) kept at the last two restarts

    def collect(self, q, u):
        self.shape = q.shape
        self.V.append(q.copy())
        self.VD.append(0.5 * (1.0 - self.mu) * u + 0.5 * (1.0 + self.mu) * q)
        if len(self.V) == self.m:
            self.diagonalise()

    def diagonalise(self):
        if len(self.V) <= self.n:
            return
        nprev = self.n if self.ndiag > 0 else 0
        v, vD, theta, C = rayleigh_ritz(_mat(self.V), _mat(self.VD), self.n, self.mu, self.delta,
                                        canonical=self.canonical)
        self.V = [v[:, i].reshape(self.shape) for i in range(self.n)]
        self.VD = [vD[:, i].reshape(self.shape) for i in range(self.n)]
        self.theta = theta
        self.ndiag += 1
        if C.shape[0] > nprev:
            self.uv_hist.append(float(np.abs(C[nprev:, :]).max()))
        self.uv_hist = self.uv_hist[-10:]

    def ritz(self):
        """Ritz values (v_i, gamma_5 v^D_i) and residual norms of Alg. 6."""
        vals, res = [], []
        for v, vD in zip(self.V[: self.n], self.VD[: self.n]):
            g = g5(vD)
            h = dot(v, g).real
            vals.append(h)
            res.append(norm(g - h * v))
        return np.array(vals), np.array(res)

    def rediagonalise_kept(self):
        """The three-set re-diagonalisation of Sec. 5 (module notes): Alg. 6's
        Rayleigh-Ritz over the n held eigenvectors and the sets kept at the
        last two restarts; the result is held and kept."""
        if self.theta is None or len(self.V) < self.n:
            return
        n = self.n
        cur = ([v.copy() for v in self.V[:n]], [d.copy() for d in self.VD[:n]])
        v, vD, theta = rediagonalise_sets([cur] + self.kept[::-1], n, self.mu, self.delta)
        self.V = [v[:, i].reshape(self.shape) for i in range(n)]
        self.VD = [vD[:, i].reshape(self.shape) for i in range(n)]
        self.theta = theta
        self.kept = (self.kept + [(list(self.V), list(self.VD))])[-2:]

    def recompute(self, apply_D, eta=1e-13):
        """v^D = D v to high accuracy (after the eigenvector phase / every k)."""
        self.VD = [apply_D(v, eta) for v in self.V]

    def sign_accuracy(self):
        """Eq. (bound) of Sec. 5.1 as a sign accuracy (module notes)."""
        if len(self.V) < self.n or self.theta is None:
            r0 = 0.0
        else:
            r0 = float(self.ritz()[1].min())
        chi = 1.0 if self.ndiag < 2 else np.sqrt(self.n)
        uv = np.mean(self.uv_hist) if self.uv_hist else 1.0
        dd = chi * (np.sqrt(self.eps ** 2 + r0 ** 2) - r0) / (np.sqrt((self.m - self.n) * self.krecalc) * uv)
        return 2.0 * dd / (1.0 - self.mu)

    def deflation(self):
        return Deflation(self.V[: self.n], self.VD[: self.n])


def gmresr_eigsumr(overlap, b, eps, eta_tilde, eig, calc=True, floor=1e-2, maxiter=10000):
    """GMRESR(relSUMR) with eigSUMR (Secs. 3-5): every middle solve starts from
    the deflation projection of the current eigenvector set; while calc is
    true its Krylov vectors are collected (Alg. 5) at the stricter of the
    inversion and eigenvector sign accuracies, and Alg. 6 runs whenever m
    vectors are held and at the end of each middle solve."""
    from . import krylov
    mu = overlap.mu
    bnorm = norm(b)
    rho = (1.0 - mu) / (1.0 + mu)

    def apply_A(u):
        e = min(1e-2, eps * bnorm / (2.0 * (1.0 - mu) * norm(u)))
        return overlap(u, e)

    def middle(r):
        x0 = None
        if len(eig.V) >= eig.n and eig.theta is not None:
            x0 = eig.deflation().x0(r)
        bp = (2.0 / (1.0 + mu)) * r
        bpn = norm(bp)

        def eta_fn(j, res):
            e = eta_tilde if (res is None or res <= 0) else min(floor, eta_tilde * bpn / res)
            if calc:
                e = min(e, eig.sign_accuracy())
            return e

        res = krylov.sumr(overlap.U, rho, bp, eta_tilde, x0=x0, maxiter=maxiter, eta_fn=eta_fn,
                          on_step=(eig.collect if calc else None))
        if calc:
            eig.diagonalise()
            if eig.ndiag and eig.ndiag % eig.krecalc == 0:
                eig.recompute(overlap)
        return res.x, res.iters

    res = krylov.gmresr(apply_A, middle, b, 0.5 * eps)
    if calc:
        eig.rediagonalise_kept()   # each new right-hand side restarts the Krylov space (Sec. 5)
    return res


def spectral_preconditioner(V, VD):
    """Sec. 4's Hhat^{-1} from held vectors V with images VD = D V: the
    Rayleigh-Ritz pairs (m_i, s_i) of H^2 = D^+ D in span(V), found from
    V^H V = R^H R and the eigenpairs (m_i, y_i) of R^{-H} VD^H VD R^{-1}
    (since (H v, H w) = (D v, D w)), with s_i = V R^{-1} y_i orthonormal."""
    from . import krylov
    shape = V[0].shape
    Vm, VDm = _mat(V), _mat(VD)
    E = Vm.conj().T @ Vm
    E = 0.5 * (E + E.conj().T)
    Rinv = np.linalg.inv(np.linalg.cholesky(E).conj().T)
    G = Rinv.conj().T @ (VDm.conj().T @ VDm) @ Rinv
    m, Y = np.linalg.eigh(0.5 * (G + G.conj().T))
    S = Vm @ (Rinv @ Y)
    return krylov.SpectralPreconditioner([S[:, i].reshape(shape) for i in range(S.shape[1])], m)


class EigCG(EigSUMR):
    """eigCG collection on the relCG middle solve (module notes): the two
    unit-norm basis vectors of each CG iteration with their images under D,
    Alg. 6 at k = m; the relaxation bound, recomputation and deflation data
    are those of EigSUMR."""

    def collect_cg(self, w, hw, hhw):
        for v, dv in ((w, g5(hw)), (hw, g5(hhw))):
            s = 1.0 / norm(v)
            self.shape = v.shape
            self.V.append(s * v)
            self.VD.append(s * dv)
            if len(self.V) == self.m:
                self.diagonalise()

    def preconditioner(self):
        """The spectral preconditioner of the n held eigenvectors, or None
        before the first diagonalisation."""
        if self.theta is None:
            return None
        n = min(self.n, len(self.V))
        return spectral_preconditioner(self.V[:n], self.VD[:n])


def gmresr_eigcg(overlap, b, eps, eta_tilde, eig, calc=True, floor=1e-2, maxiter=10000):
    """GMRESR(eigCG): Alg. 3 whose middle solves are the Sec. 4 CGNE for
    H u = gamma_5 r, spectrally preconditioned with the eigenvectors held
    when each middle solve starts; while calc is true each CG iteration's
    vectors are collected (EigCG.collect_cg) at the stricter of the CG and
    eigenvector sign accuracies, and Alg. 6 closes every middle solve."""
    from . import krylov
    mu = overlap.mu
    bnorm = norm(b)

    def apply_A(u):
        e = min(1e-2, eps * bnorm / (2.0 * (1.0 - mu) * norm(u)))
        return overlap(u, e)

    def H(v, eta):
        return g5(overlap(v, eta))

    def middle(r):
        pre = eig.preconditioner()
        res = krylov.cgne(H, g5(r), eta_tilde, precond=pre, eps_A=eta_tilde, floor=floor, maxiter=maxiter,
                          eta_cap=(eig.sign_accuracy if calc else None),
                          on_iter=(eig.collect_cg if calc else None))
        if calc:
            eig.diagonalise()
            if eig.ndiag and eig.ndiag % eig.krecalc == 0:
                eig.recompute(overlap)
        return res.x, res.iters

    res = krylov.gmresr(apply_A, middle, b, 0.5 * eps)
    if calc:
        eig.rediagonalise_kept()
    return res


def rediagonalise_sets(sets, n, mu, delta, cut=1e-10):
    """Rayleigh-Ritz of Alg. 6 (same pair-splitting M) over the union of the
    eigenvector sets [(V, VD), ...], orthonormalised canonically: with
    V^H V = W diag(l) W^H and B = W_k diag(l_k^{-1/2}) over l_k > cut max(l),
    the eigenpairs (theta, Y) of B^H M B give v = V B Y[:, :n]."""
    V = _mat([v for vs, _ in sets for v in vs])
    VD = _mat([d for _, ds in sets for d in ds])
    N = V.shape[0]
    E = V.conj().T @ V
    lam, W = np.linalg.eigh(0.5 * (E + E.conj().T))
    keep = lam > cut * lam.max()
    B = W[:, keep] / np.sqrt(lam[keep])
    G5VD = (g5(VD.T.reshape((VD.shape[1], N // 12, 4, 3))).reshape(VD.shape[1], -1)).T
    M = VD.conj().T @ VD + 2.0 * mu * delta * (V.conj().T @ G5VD)
    G = B.conj().T @ (0.5 * (M + M.conj().T)) @ B
    theta, Y = np.linalg.eigh(0.5 * (G + G.conj().T))
    C = B @ Y[:, :n]
    return V @ C, VD @ C, theta[:n]


class EigensolverRun:
    def __init__(self, applies, ritz, resid, ndiag, rank):
        self.applies, self.ritz, self.resid, self.ndiag, self.rank = applies, ritz, resid, ndiag, rank


def eigsumr_eigensolver(overlap, q0, eig, restarts=10, diag_per_restart=24, relaxed=True, eta_full=1e-12,
                        recompute_eta=1e-13, floor=1e-2):
    """The standalone eigSUMR eigensolver (module notes): runs of the Alg. 1
    basis with Alg. 5 collection at the Sec. 5.1 sign accuracy, never looser
    than floor (relaxed), or at eta_full, each closed by Alg. 6, an accurate v^D and the three-set
    re-diagonalisation; stops when every residual is at most eig.eps as
    given.  Returns one EigensolverRun per restart (U applications so far,
    Ritz values and residuals after it)."""
    n = eig.n
    eps_final = eig.eps
    q = q0 / norm(q0)
    eig.kept = []
    runs = []
    applies = 0
    for _ in range(restarts):
        q_t = q.copy()
        nd0 = eig.ndiag
        while eig.ndiag - nd0 < diag_per_restart:
            u = overlap.U(q, min(floor, eig.sign_accuracy()) if relaxed else eta_full)
            applies += 1
            eig.collect(q, u)
            gamma = dot(q_t, u)
            if abs(gamma) >= 1.0:
                break
            sigma = np.sqrt(1.0 - abs(gamma) ** 2)
            gamma = -gamma
            q = (gamma * q_t + u) / sigma
            q_t = sigma * q_t + np.conj(gamma) * q
            if abs(norm(q) - 1.0) > 0.1:
                break
            if eig.theta is not None and eig.ritz()[1].max() <= eig.eps:
                break
        eig.diagonalise()
        if eig.theta is None or len(eig.V) < n:
            raise RuntimeError("eigensolver: a run ended before the first diagonalisation")
        eig.recompute(overlap, recompute_eta)
        eig.rediagonalise_kept()
        vals, res = eig.ritz()
        runs.append(EigensolverRun(applies, vals, res, eig.ndiag, None))
        if res.max() <= eps_final:
            break
        eig.eps = max(eps_final, 0.1 * res.max())
        for _ in range(2):
            for vi in eig.V:
                q = q - dot(vi, q) * vi
        q = q / norm(q)
    eig.eps = eps_final
    return runs
