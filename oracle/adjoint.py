"""Oracle: derivatives of S = Re(chi^H D[mu] psi), FP64 numpy.

TEST INFRASTRUCTURE ONLY.

The paper does not differentiate the overlap operator; this follows from its
definitions: D[mu] (Sec. 1, eq. 1), the kernel K = gamma_5 D_W(-rho) (Sec. 1,
eq. 2) and the rational sign function
    eps(K) = K sum_l omega_l X_l,   X_l = (K^2 + sigma_l)^{-1}
(Sec. 1, eq. 4 and Sec. 3, eq. 7), with no exactly treated low modes (the
link derivative of the low-mode projection is not provided).

* dS/dpsi (the gradient as d/dRe + i d/dIm) = D^dagger chi = gamma_5 D gamma_5 chi.
* Links, each entry of U_mu(x) an independent complex variable (the hopping
  term uses U and U^dagger).  With chi' = gamma_5 chi, a_l = X_l psi and
  b_l = X_l K chi',
      dS = (1 - mu)/2 Re sum_l omega_l [chi'^H dK a_l - b_l^H dK K a_l
                                        - (K b_l)^H dK a_l],
  using d X_l = -X_l (dK K + K dK) X_l, and dK = -gamma_5 dH / 2.
  For Re(alpha^H gamma_5 dH beta), with alpha' = gamma_5 alpha, the
  gradient on the link (y, mu) is the colour matrix
      T(alpha', beta)_ab = sum_s [((1 - gamma_mu) alpha')(y)_sa conj(beta(y+mu)_sb)
                                  + beta(y)_sa conj(((1 + gamma_mu) alpha')(y+mu)_sb)],
  the first term from U_mu(y) psi(y+mu) in H, the second from
  U_mu(y)^dagger psi(y) in (H psi)(y+mu).
"""
import numpy as np

from .krylov import Overlap, SignFunction, multishift_cg
from .lattice import WilsonKernel, dot, g5, gamma


def action(dims, U, rho, zolo, mu, psi, chi, eta=1e-15):
    """S = Re(chi^H D[mu] psi) with the Zolotarev sign function, no low modes."""
    k = WilsonKernel(dims, U, rho)
    D = Overlap(SignFunction(k, zolo), mu)
    return dot(chi, D(psi, eta)).real


def psi_gradient(dims, U, rho, zolo, mu, chi, eta=1e-15):
    """dS/dpsi = D^dagger chi (S is linear in psi)."""
    k = WilsonKernel(dims, U, rho)
    return Overlap(SignFunction(k, zolo), mu).adjoint(chi, eta)


def _fwd(field, dims, mu):
    """field(y + mu) for a site-major field [V, ...] (x fastest, periodic)."""
    Lx, Ly, Lz, Lt = (int(d) for d in dims)
    f = field.reshape((Lt, Lz, Ly, Lx) + field.shape[1:])
    return np.roll(f, -1, axis=3 - mu).reshape(field.shape)


def outer_T(dims, alpha_p, beta):
    """T(alpha', beta) for every link: array [V, 4, 3, 3] (see module notes)."""
    G = gamma()
    one = np.eye(4)
    V = alpha_p.shape[0]
    out = np.zeros((V, 4, 3, 3), np.complex128)
    for mu in range(4):
        pm = np.einsum("st,vta->vsa", one - G[mu], alpha_p)
        pp = np.einsum("st,vta->vsa", one + G[mu], alpha_p)
        out[:, mu] = (np.einsum("vsa,vsb->vab", pm, np.conj(_fwd(beta, dims, mu)))
                      + np.einsum("vsa,vsb->vab", beta, np.conj(_fwd(pp, dims, mu))))
    return out


def link_gradient(dims, U, rho, zolo, mu, psi, chi, tol=1e-15):
    """dS/dU (as d/dRe U + i d/dIm U, entry by entry), array [V, 4, 3, 3]."""
    k = WilsonKernel(dims, U, rho)
    psi = np.asarray(psi, np.complex128).reshape(k.shape)
    chi_p = g5(np.asarray(chi, np.complex128).reshape(k.shape))
    a = multishift_cg(k.K2s, zolo.sigma, psi, tol).x
    b = multishift_cg(k.K2s, zolo.sigma, k.K(chi_p), tol).x
    acc = np.zeros((k.V, 4, 3, 3), np.complex128)
    for w, al, bl in zip(zolo.omega, a, b):
        acc += w * (outer_T(dims, g5(chi_p), al)
                    - outer_T(dims, g5(bl), k.K(al))
                    - outer_T(dims, g5(k.K(bl)), al))
    # Re(alpha^H dK beta) = -Re(alpha^H gamma_5 dH beta)/2
    return -0.25 * (1.0 - mu) * acc
