"""Oracle: sign function, overlap operator and the nested solvers, FP64 numpy.

TEST INFRASTRUCTURE ONLY.

* ``multishift_cg``  -- the inner inversions of x^2 + sigma_l (paper Sec. 3,
  eq. 7 and the text after it; the paper does not print the algorithm, the
  textbook multi-shift CG recurrences are used: base system the smallest
  shift, shifted residuals r_l = zeta_l r).
* ``SignFunction``   -- sign(K) with the lowest eigenvectors of K treated
  exactly and the Zolotarev approximation on the rest (Sec. 1, eq. 4 and the
  text after it; Sec. 3, eq. 7).
* ``Overlap``        -- D[mu] = (1 + mu + (1 - mu) gamma_5 sign(K)) / 2 (Sec. 1, eq. 1).
* ``sumr``           -- Alg. 2 (with the basis recurrence of Alg. 1) for
  (1 + rho U) x = b, U unitary, run in the printed statement order; the
  relaxation eta_j = eps_A ||b|| / ||r_j|| of Sec. 3 with a floor on the
  accuracy, and the normalisation-monitoring restart of Sec. 2.
* ``gmresr``         -- Alg. 3.
* ``SpectralPreconditioner``, ``cgne``, ``gmresr_cg`` -- the deflated CGNE
  of Sec. 4 (its printed algorithm) with the spectral preconditioner built
  from approximate eigenvectors of H = gamma_5 D[mu], the CG relaxation of
  Sec. 3, and GMRESR(relCG) (Alg. 3 with that middle solve).

Readings where the paper is silent or garbled (each also listed in the design
notes):
* Alg. 2 uses zeta without defining it: zeta = 1.
* Alg. 2 is applied to D[mu] as (1 + rho' U) x = b' with U = gamma_5 sign(K),
  rho' = (1 - mu)/(1 + mu), b' = 2 b / (1 + mu); its residual norm is
  rho' |tau_hat|.
* Sign accuracy eta -> multi-shift stopping rule: shift l is frozen once
  omega_l |zeta_l| ||r|| / (2 sqrt(sigma_l)) <= eta ||b|| / N_Z, which bounds
  the inversion error of the rational function by eta ||b||
  (||K (K^2 + sigma)^{-1}|| <= 1 / (2 sqrt(sigma))).
* CG relaxation (Sec. 3): eta_j = eps_A ||r_0|| sqrt(zeta_j) with zeta_j the
  sum of ||r_i||^-2 over the residuals so far, r_0 the (preconditioned)
  starting residual, capped at the same floor as SUMR; the closing
  x = H Hhat^{-1} x_j uses accuracy eps_A.
* CGNE for the GMRESR middle solve D u = r: D = gamma_5 H, so u solves
  H u = gamma_5 r.
* GMRESR's "compute c with ||A u - c|| < eps ||b|| ||u|| / ||r||": taken
  literally it lets each outer step open a residual gap of up to
  eps ||b|| ||u|| / ||r||, i.e. up to eps ||b|| / mu.  The rule used asks for
  ||A u - c|| <= eps ||b|| / 4 (with ||c|| ~ ||r||), i.e. a sign accuracy
  eps ||b|| / (2 (1 - mu) ||u||), and the outer loop stops at
  ||r|| <= eps ||b|| / 2, so that the true residual stays below eps ||b||.
"""
import numpy as np

from .lattice import axpy, axpby, dot, g5, norm


class MSCGResult:
    def __init__(self, x, iters, shift_iters):
        self.x = x
        self.iters = iters
        self.shift_iters = shift_iters


def multishift_cg(apply_A, sigma, b, tol, maxiter=100000):
    """Solve (A + sigma_l) x_l = b for every shift, A Hermitian non-negative.

    Base system: the smallest shift s0; w = (A + s0) p, alpha = (r, r)/(p, w),
    r <- r - alpha w, beta = (r_new, r_new)/(r, r), p <- r + beta p.  Shift l
    keeps r_l = zeta_l r, with
      zeta_l' = zeta_l zeta_l^old alpha^old /
                [alpha beta^old (zeta_l^old - zeta_l)
                 + zeta_l^old alpha^old (1 + (sigma_l - s0) alpha)],
      alpha_l = alpha zeta_l' / zeta_l,  x_l += alpha_l p_l,
      p_l <- zeta_l' r_new + beta (zeta_l'/zeta_l)^2 p_l,
    started from zeta = zeta^old = 1, alpha^old = 1, beta^old = 0.
    Shift l is frozen (no further updates) once |zeta_l| ||r|| <= tol_l ||b||;
    the iteration ends when every shift is frozen.
    """
    sigma = np.asarray(sigma, dtype=np.float64)
    tol = np.broadcast_to(np.asarray(tol, dtype=np.float64), sigma.shape)
    n = len(sigma)
    base = int(np.argmin(sigma))
    s0 = sigma[base]
    b = np.ascontiguousarray(b, dtype=np.complex128)
    x = [np.zeros_like(b) for _ in range(n)]
    bnorm = norm(b)
    shift_iters = np.zeros(n, dtype=np.int64)
    if bnorm == 0.0:
        return MSCGResult(x, 0, shift_iters)
    r = b.copy()
    p = [b.copy() for _ in range(n)]
    zeta = np.ones(n)
    zeta_old = np.ones(n)
    alpha_old, beta_old = 1.0, 0.0
    rr = dot(r, r).real
    active = np.ones(n, dtype=bool)
    it = 0
    while active.any() and it < maxiter:
        w = apply_A(p[base]) + s0 * p[base]
        alpha = rr / dot(p[base], w).real
        zeta_new = zeta.copy()
        for l in range(n):
            if not active[l]:
                continue
            zeta_new[l] = (zeta[l] * zeta_old[l] * alpha_old) / (
                alpha * beta_old * (zeta_old[l] - zeta[l])
                + zeta_old[l] * alpha_old * (1.0 + (sigma[l] - s0) * alpha))
            alpha_l = alpha * zeta_new[l] / zeta[l]
            axpy(alpha_l, p[l], x[l])                   # x_l = x_l + alpha_l p_l
        axpy(-alpha, w, r)                              # r = r - alpha w
        rr_new = dot(r, r).real
        beta = rr_new / rr
        for l in range(n):
            if not active[l]:
                continue
            beta_l = beta * (zeta_new[l] / zeta[l]) ** 2
            axpby(zeta_new[l], r, beta_l, p[l])         # p_l = zeta_l' r + beta_l p_l
            zeta_old[l] = zeta[l]
            zeta[l] = zeta_new[l]
            shift_iters[l] += 1
        alpha_old, beta_old, rr = alpha, beta, rr_new
        it += 1
        rn = np.sqrt(rr)
        for l in range(n):
            if active[l] and abs(zeta[l]) * rn <= tol[l] * bnorm:
                active[l] = False
    return MSCGResult(x, it, shift_iters)


def shift_tolerances(zolo, eta):
    """Per-shift stopping targets that bound the rational function's
    inversion error by eta ||b|| (see the module notes)."""
    return eta * 2.0 * np.sqrt(zolo.sigma) / (zolo.nz * zolo.omega)


class LowModes:
    """Lowest eigenpairs (lambda_i, psi_i) of K, treated exactly in sign(K)."""

    def __init__(self, evals, evecs):
        self.evals = np.asarray(evals, dtype=np.float64)
        self.evecs = np.asarray(evecs, dtype=np.complex128)   # [n, V, 4, 3]

    def __len__(self):
        return len(self.evals)


class SignFunction:
    """sign(K) psi ~= sum_i sign(lambda_i) psi_i (psi_i, psi)
                     + eps(K) (1 - sum_i psi_i psi_i^dagger) psi,
    eps(K) = K sum_l omega_l (K^2 + sigma_l)^{-1} (Sec. 1 eq. 4; Sec. 3 eq. 7)."""

    def __init__(self, kern, zolo, lowmodes=None):
        self.kern = kern
        self.zolo = zolo
        self.low = lowmodes
        self.calls = 0
        self.mscg_iters = 0

    def __call__(self, psi, eta):
        psi = np.asarray(psi, dtype=np.complex128).reshape(self.kern.shape)
        exact = np.zeros_like(psi)
        perp = psi.copy()
        if self.low is not None and len(self.low):
            for lam, v in zip(self.low.evals, self.low.evecs):
                c = dot(v, psi)
                perp = perp - c * v
                exact = exact + np.sign(lam) * c * v
        res = multishift_cg(self.kern.K2s, self.zolo.sigma, perp,
                            shift_tolerances(self.zolo, eta))
        y = np.zeros_like(psi)
        for w, xl in zip(self.zolo.omega, res.x):
            y = y + w * xl
        self.calls += 1
        self.mscg_iters += res.iters
        return self.kern.K(y) + exact


class Overlap:
    """D[mu] = (1 + mu + (1 - mu) gamma_5 sign(K)) / 2  (Sec. 1, eq. 1)."""

    def __init__(self, sign, mu):
        self.sign = sign
        self.mu = float(mu)

    def U(self, psi, eta):
        """The unitary part gamma_5 sign(K) psi."""
        return g5(self.sign(psi, eta))

    def __call__(self, psi, eta):
        return 0.5 * (1.0 + self.mu) * psi + 0.5 * (1.0 - self.mu) * self.U(psi, eta)

    def adjoint(self, psi, eta):
        """D^dagger = gamma_5 D gamma_5 (Sec. 1)."""
        return g5(self(g5(psi), eta))


class SUMRResult:
    def __init__(self, x, iters, resid, restarts, history):
        self.x = x
        self.iters = iters
        self.resid = resid
        self.restarts = restarts
        self.history = history


def sumr(apply_U, rho, b, tol, x0=None, maxiter=10000, eta_fn=None,
         norm_restart=0.1, on_step=None):
    """Alg. 2: solve (1 + rho U) x = b, U unitary, to ||b - (1 + rho U) x|| <= tol ||b||.

    apply_U(v, eta) applies U with accuracy eta.  eta_fn(j, resid) gives the
    accuracy for iteration j from the current residual norm; the default is
    full accuracy 1e-15.  on_step(q, u) is called with the basis vector q_j and
    u = U q_j of every iteration (the eigSUMR hook of Alg. 5).
    The statements of the loop body are executed in the printed order; zeta = 1.
    Restart (Sec. 2; threshold of Sec. 6): when | ||q|| - 1 | > norm_restart or
    |gamma| >= 1, the current x becomes x0 and the algorithm starts again.
    """
    if eta_fn is None:
        def eta_fn(j, res):
            return 1e-15
    bnorm = norm(b)
    x = np.zeros_like(b) if x0 is None else x0.copy()
    history = []
    total = 0
    restarts = 0
    if bnorm == 0.0:
        return SUMRResult(np.zeros_like(b), 0, 0.0, 0, history)
    zeta = 1.0
    while True:
        if x0 is None and total == 0 and restarts == 0:
            rt = b.copy()
        else:
            rt = b - (x + rho * apply_U(x, eta_fn(total, None)))
        delta = norm(rt)
        if delta <= tol * bnorm:
            return SUMRResult(x, total, delta, restarts, history)
        phi_hat = 1.0 / delta
        tau_hat = delta / rho
        omega = np.zeros_like(b)
        q_old = np.zeros_like(b)
        p = np.zeros_like(b)
        phi = 0.0
        s = 0.0
        q = rt / delta
        q_t = q.copy()
        lam = 0.0
        r_p = 0.0
        r = 1.0
        gamma = 1.0
        c = 1.0
        c_dag = 1.0
        sigma = 1.0
        restart = False
        while True:
            resid = rho * abs(tau_hat)
            history.append(resid)
            if resid <= tol * bnorm:
                return SUMRResult(x, total, resid, restarts, history)
            if total >= maxiter:
                return SUMRResult(x, total, resid, restarts, history)
            r_pp = r
            u = apply_U(q, eta_fn(total, resid))
            if on_step is not None:
                on_step(q, u)
            gamma = dot(q_t, u)
            if abs(gamma) >= 1.0:
                restart = True
                break
            sigma = np.sqrt(1.0 - abs(gamma) ** 2)
            alpha = gamma * delta
            gamma = -gamma
            r_p = alpha * phi + s * zeta / rho
            r_hat = alpha * phi_hat + c_dag * zeta / rho
            nrm = np.sqrt(abs(r_hat) ** 2 + sigma ** 2)
            c_dag = r_hat / nrm
            c = np.conj(c_dag)
            s = -sigma / nrm
            r = s * sigma - c * r_hat
            tau = -c * tau_hat
            tau_hat = s * tau_hat
            eta = tau / r
            kappa = r_p / r_pp
            omega_old = omega
            omega = alpha * p + kappa * (q_old - omega)
            p = p + lam * (q_old - omega_old)
            x = x + eta * (q - omega)
            delta = sigma * delta
            phi = s * np.conj(gamma) / delta - c * phi_hat
            lam = phi / r
            phi_hat = s * phi_hat + c_dag * np.conj(gamma) / delta
            q_old = q
            q = (gamma * q_t + u) / sigma
            q_t = sigma * q_t + np.conj(gamma) * q
            total += 1
            if abs(norm(q) - 1.0) > norm_restart:
                restart = True
                break
        if restart:
            restarts += 1
            if restarts > 50:
                return SUMRResult(x, total, None, restarts, history)


def sumr_overlap(overlap, b, tol, x0=None, eps_A=None, floor=1e-2, maxiter=10000, on_step=None):
    """relSUMR for D[mu] x = b (Alg. 2 with the Sec. 3 relaxation).

    eta_j = min(floor, eps_A ||b|| / ||r_j||); eps_A defaults to tol.
    The residual is tracked in the units of the scaled system, whose residual
    is (2/(1+mu)) times that of D[mu] x = b.
    """
    mu = overlap.mu
    rho = (1.0 - mu) / (1.0 + mu)
    bp = (2.0 / (1.0 + mu)) * b
    bpn = norm(bp)
    eps_A = tol if eps_A is None else eps_A

    def eta_fn(j, res):
        if res is None or res <= 0.0:
            return eps_A
        return min(floor, eps_A * bpn / res)

    return sumr(overlap.U, rho, bp, tol, x0=x0, maxiter=maxiter, eta_fn=eta_fn,
                on_step=on_step)


def gmres_dense(A, b, m):
    """Full GMRES iterate of dimension m for dense A (Krylov basis by
    Arnoldi with modified Gram-Schmidt; least squares by numpy)."""
    n = len(b)
    Q = np.zeros((n, m + 1), dtype=np.complex128)
    Hm = np.zeros((m + 1, m), dtype=np.complex128)
    beta = np.linalg.norm(b)
    Q[:, 0] = b / beta
    for j in range(m):
        w = A @ Q[:, j]
        for i in range(j + 1):
            Hm[i, j] = np.vdot(Q[:, i], w)
            w = w - Hm[i, j] * Q[:, i]
        Hm[j + 1, j] = np.linalg.norm(w)
        Q[:, j + 1] = w / Hm[j + 1, j]
    e1 = np.zeros(m + 1, dtype=np.complex128)
    e1[0] = beta
    y = np.linalg.lstsq(Hm, e1, rcond=None)[0]
    return Q[:, :m] @ y


class GMRESRResult:
    def __init__(self, x, steps, resid, middle_iters):
        self.x = x
        self.steps = steps
        self.resid = resid
        self.middle_iters = middle_iters


def gmresr(apply_A, middle, b, eps, max_steps=50):
    """Alg. 3.  apply_A(u) returns c = A u to the accuracy the outer loop
    needs (module notes); middle(r) returns an approximate solution u of
    A u = r (the preconditioner) and its iteration count.  Stops at
    ||r|| <= eps ||b|| (the caller passes the tightened eps)."""
    x = np.zeros_like(b)
    r = b.copy()
    C, Uv = [], []
    bnorm = norm(b)
    steps = 0
    middle_iters = []
    while norm(r) > eps * bnorm and steps < max_steps:
        u, its = middle(r)
        middle_iters.append(its)
        c = apply_A(u)
        for Cj, Uj in zip(C, Uv):
            beta = dot(Cj, c)
            c = c - beta * Cj
            u = u - beta * Uj
        nc = norm(c)
        c = c / nc
        u = u / nc
        C.append(c)
        Uv.append(u)
        alpha = dot(c, r)
        x = x + alpha * u
        r = r - alpha * c
        steps += 1
    return GMRESRResult(x, steps, norm(r), middle_iters)


def gmresr_sumr(overlap, b, eps, eta_tilde, floor=1e-2, deflation=None, maxiter=10000):
    """GMRESR(relSUMR): Alg. 3 with relSUMR (Alg. 2, Sec. 3 relaxation) as the
    preconditioner; the outer c = D u uses the sign accuracy of the module
    notes; ``deflation`` (optional) gives the middle solve's starting vector
    (Sec. 4)."""
    mu = overlap.mu
    bnorm = norm(b)

    def apply_A(u):
        eta = min(1e-2, eps * bnorm / (2.0 * (1.0 - mu) * norm(u)))
        return overlap(u, eta)

    def middle(r):
        x0 = None if deflation is None else deflation.x0(r)
        res = sumr_overlap(overlap, r, eta_tilde, x0=x0, eps_A=eta_tilde, floor=floor,
                           maxiter=maxiter)
        return res.x, res.iters

    return gmresr(apply_A, middle, b, 0.5 * eps)


class SpectralPreconditioner:
    """Hhat^{-1} = 1 + sum_i |psi_i><psi_i| (c / sqrt(m_i) - 1)  (Sec. 4), with
    psi_i orthonormal approximate eigenvectors of H^2 and m_i their Ritz
    values (psi_i, H^2 psi_i); c = sqrt(3)/2 as in the paper.  Applied on both
    sides of H^2: with exact eigenvectors the n smallest eigenvalues of
    Hhat^{-1} H^2 Hhat^{-1} become c^2 and the rest stay."""

    def __init__(self, psis, ritz, c=np.sqrt(3.0) / 2.0):
        self.psis = [np.asarray(p) for p in psis]
        self.ritz = [float(m) for m in ritz]
        self.c = float(c)

    def __call__(self, v):
        out = v.copy()
        for p, m in zip(self.psis, self.ritz):
            out = out + (self.c / np.sqrt(m) - 1.0) * dot(p, v) * p
        return out


class CGResult:
    def __init__(self, x, iters, resid):
        self.x, self.iters, self.resid = x, iters, resid


def cgne(apply_H, b, tol, precond=None, eps_A=None, floor=1e-2, maxiter=10000, eta_cap=None, on_iter=None):
    """The preconditioned CGNE of Sec. 4 for H x = b (H Hermitian):
    r_0 = p_0 = Hhat^{-1} b, x_0 = 0; per iteration z = Hhat^{-1} H^2
    Hhat^{-1} p, alpha = (r, r) / (r, z), r -= alpha z, x += alpha p,
    beta = (r', r') / (r, r), p = r' + beta p; until ||r|| < tol ||b||; then
    x = H Hhat^{-1} x.  apply_H(v, eta) applies H with sign accuracy eta,
    relaxed as in Sec. 3 for CG (module notes).

    eigCG (Sec. 5) hooks: eta_cap() bounds each iteration's sign accuracy
    from above (the eigenvector bound of Sec. 5.1), and on_iter(w, Hw, HHw)
    receives the preconditioned direction w = Hhat^{-1} p with its two
    images under H."""
    P = precond if precond is not None else (lambda v: v)
    eps_A = tol if eps_A is None else eps_A
    bn = norm(b)
    r = P(b)
    p = r.copy()
    x = np.zeros_like(b)
    rr = dot(r, r).real
    r0n = np.sqrt(rr)
    zeta = 1.0 / rr if rr > 0 else 0.0
    it = 0
    while np.sqrt(rr) >= tol * bn and it < maxiter:
        eta = min(floor, eps_A * r0n * np.sqrt(zeta))
        if eta_cap is not None:
            eta = min(eta, eta_cap())
        w = P(p)
        hw = apply_H(w, eta)
        hhw = apply_H(hw, eta)
        if on_iter is not None:
            on_iter(w, hw, hhw)
        z = P(hhw)
        alpha = rr / dot(r, z)
        r = r - alpha * z
        x = x + alpha * p
        rr_new = dot(r, r).real
        beta = rr_new / rr
        p = r + beta * p
        rr = rr_new
        zeta += 1.0 / rr if rr > 0 else 0.0
        it += 1
    return CGResult(apply_H(P(x), eps_A), it, np.sqrt(rr))


def gmresr_cg(overlap, b, eps, eta_tilde, floor=1e-2, precond=None, maxiter=10000):
    """GMRESR(relCG): Alg. 3 with the Sec. 4 CGNE as the preconditioner for
    D u = r (H u = gamma_5 r, H = gamma_5 D), optionally with the spectral
    preconditioner; the outer c = D u as in gmresr_sumr."""
    mu = overlap.mu
    bnorm = norm(b)

    def apply_A(u):
        eta = min(1e-2, eps * bnorm / (2.0 * (1.0 - mu) * norm(u)))
        return overlap(u, eta)

    def H(v, eta):
        return g5(overlap(v, eta))

    def middle(r):
        res = cgne(H, g5(r), eta_tilde, precond=precond, eps_A=eta_tilde, floor=floor, maxiter=maxiter)
        return res.x, res.iters

    return gmresr(apply_A, middle, b, 0.5 * eps)
