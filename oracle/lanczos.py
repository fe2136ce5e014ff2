"""Oracle: sign(K) psi by the two-pass Lanczos method (the Lanczos approach to
the matrix sign function that Sec. 1 cites after eq. 4, as an alternative to
rational approximations; the paper gives no formula for it).

TEST INFRASTRUCTURE ONLY.

sign(K) = K (K^2)^{-1/2}.  On the part psi_perp of psi orthogonal to the
exactly treated low modes:
  pass 1: Lanczos on A = K^2 from q_1 = psi_perp / ||psi_perp||,
          w = A q_j - beta_{j-1} q_{j-1}, alpha_j = (q_j, w),
          w = w - alpha_j q_j, beta_j = ||w||, q_{j+1} = w / beta_j,
          building the tridiagonal T_j (alpha on the diagonal, beta beside it),
          without keeping the q_j;  y_j = ||psi_perp|| T_j^{-1/2} e_1 from the
          eigendecomposition of T_j;
  stop:   once lambda_max ||y_j - (y_{j-1}, 0)|| <= eta ||psi|| (the change of
          the last step, times the largest |lambda| of K since the result is
          K times the Lanczos approximation), or at maxiter;
  pass 2: the same recurrence from q_1 with the stored alpha_j, beta_j
          regenerates q_1 .. q_k and accumulates x = sum_j y_j q_j;
  result: sign(K) psi = K x + sum_i sign(lambda_i) psi_i (psi_i, psi).
Reading (the paper is silent on it): the stopping rule above.
"""
import numpy as np

from .lattice import dot, norm


class LanczosResult:
    def __init__(self, out, iters, converged):
        self.out, self.iters, self.converged = out, iters, converged


def _inv_sqrt_e1(alpha, beta):
    """T^{-1/2} e_1 for the symmetric tridiagonal T = tridiag(beta, alpha, beta)."""
    k = len(alpha)
    T = np.diag(np.asarray(alpha, dtype=np.float64))
    if k > 1:
        T += np.diag(np.asarray(beta[: k - 1], dtype=np.float64), 1) + np.diag(np.asarray(beta[: k - 1]), -1)
    th, S = np.linalg.eigh(T)
    return S @ (S[0, :] / np.sqrt(th))


def lanczos_sign(kern, psi, eta, lmax, lowmodes=None, maxiter=5000):
    """sign(K) psi to accuracy eta (module notes); lmax bounds |lambda| of K."""
    psi = np.asarray(psi, dtype=np.complex128).reshape(kern.shape)
    exact = np.zeros_like(psi)
    perp = psi.copy()
    if lowmodes is not None and len(lowmodes):
        for lam, v in zip(lowmodes.evals, lowmodes.evecs):
            c = dot(v, psi)
            perp = perp - c * v
            exact = exact + np.sign(lam) * c * v
    pn = norm(perp)
    if pn == 0.0:
        return LanczosResult(exact, 0, True)
    # pass 1: the tridiagonal matrix only
    alpha, beta = [], []
    q = perp / pn
    q_old = np.zeros_like(q)
    b_old = 0.0
    y_prev = None
    converged = False
    while len(alpha) < maxiter:
        w = kern.K2s(q) - b_old * q_old
        a = dot(q, w).real
        w = w - a * q
        b = norm(w)
        alpha.append(a)
        beta.append(b)
        y = pn * _inv_sqrt_e1(alpha, beta)
        if y_prev is not None:
            change = np.linalg.norm(y - np.concatenate([y_prev, [0.0]]))
            if lmax * change <= eta * norm(psi):
                converged = True
                break
        y_prev = y
        if b == 0.0:
            converged = True
            break
        q_old, q = q, w / b
        b_old = b
    k = len(alpha)
    y = pn * _inv_sqrt_e1(alpha, beta)
    # pass 2: regenerate the Lanczos vectors and accumulate x = sum_j y_j q_j
    q = perp / pn
    q_old = np.zeros_like(q)
    x = y[0] * q
    for j in range(k - 1):
        w = kern.K2s(q) - (beta[j - 1] if j > 0 else 0.0) * q_old - alpha[j] * q
        q_old, q = q, w / beta[j]
        x = x + y[j + 1] * q
    return LanczosResult(kern.K(x) + exact, k, converged)
