"""Pins for the oracle's derivatives of S = Re(chi^H D[mu] psi) (derived from
Sec. 1 eqs. 1, 2, 4 and Sec. 3 eq. 7): central finite differences of S itself,
which the oracle evaluates with its sign function, and the dense adjoint of
the rational-function operator."""
import numpy as np
import pytest

import synth
from oracle import adjoint
from oracle.lattice import WilsonKernel, dot, norm
from oracle.zolotarev import Zolotarev

# odd and even extents, so that a forward/backward neighbour mix-up cannot
# cancel (on an extent of 2 the two neighbours coincide)
DIMS = (3, 4, 3, 4)
RHO, MU = 1.4, 0.07


@pytest.fixture(scope="module")
def case():
    U = synth.gauge_field(DIMS, 3, 0.3)
    z = Zolotarev(8, 0.3, 8.0 - RHO)
    psi = synth.gaussian_source(DIMS, 61)
    chi = synth.gaussian_source(DIMS, 62)
    return U, z, psi, chi


def test_psi_gradient_dense():
    """D^dagger chi against the dense matrix of
    (1 + mu)/2 + (1 - mu)/2 gamma_5 K sum_l omega_l (K^2 + sigma_l)^{-1}."""
    dims = (2, 2, 2, 2)
    U = synth.gauge_field(dims, 4, 0.3)
    z = Zolotarev(8, 0.3, 8.0 - RHO)
    k = WilsonKernel(dims, U, RHO)
    K = k.dense("K")
    n = K.shape[0]
    R = sum(w * np.linalg.inv(K @ K + s * np.eye(n)) for w, s in zip(z.omega, z.sigma))
    G5 = np.kron(np.eye(k.V), np.kron(np.diag([1.0, 1, -1, -1]), np.eye(3)))
    D = 0.5 * (1 + MU) * np.eye(n) + 0.5 * (1 - MU) * G5 @ K @ R
    chi = synth.gaussian_source(dims, 5)
    got = adjoint.psi_gradient(dims, U, RHO, z, MU, chi)
    ref = D.conj().T @ chi.reshape(-1)
    assert norm(got.reshape(-1) - ref) / norm(ref) < 1e-12


def test_psi_gradient_fd(case):
    """S is linear in psi, so a central difference is exact up to the sign
    function's accuracy."""
    U, z, psi, chi = case
    g = adjoint.psi_gradient(DIMS, U, RHO, z, MU, chi)
    rng = np.random.default_rng(7)
    e = rng.normal(size=psi.shape) + 1j * rng.normal(size=psi.shape)
    h = 1e-3
    fd = (adjoint.action(DIMS, U, RHO, z, MU, psi + h * e, chi)
          - adjoint.action(DIMS, U, RHO, z, MU, psi - h * e, chi)) / (2 * h)
    pred = np.vdot(g, e).real
    assert abs(fd - pred) <= 1e-10 * abs(pred)


def test_link_gradient_fd(case):
    """Central differences along random complex directions on 50 single links
    and on all links at once agree with the formula."""
    U, z, psi, chi = case
    G = adjoint.link_gradient(DIMS, U, RHO, z, MU, psi, chi)
    V = U.shape[0]
    rng = np.random.default_rng(8)
    h = 1e-5

    def fd(E):
        return (adjoint.action(DIMS, U + h * E, RHO, z, MU, psi, chi)
                - adjoint.action(DIMS, U - h * E, RHO, z, MU, psi, chi)) / (2 * h)

    scale = np.abs(G).max()
    for link in rng.choice(4 * V, 50, replace=False):
        s, mu = divmod(int(link), 4)
        E = np.zeros_like(U)
        E[s, mu] = rng.normal(size=(3, 3)) + 1j * rng.normal(size=(3, 3))
        pred = np.vdot(G[s, mu], E[s, mu]).real
        assert abs(fd(E) - pred) <= 1e-6 * scale, (s, mu)
    E = rng.normal(size=U.shape) + 1j * rng.normal(size=U.shape)
    pred = np.vdot(G, E).real
    assert abs(fd(E) - pred) <= 1e-7 * abs(pred)


def test_link_gradient_terms_needed(case):
    """Each of the three terms carries weight: dropping any one of them moves
    the gradient by far more than the finite-difference agreement above."""
    U, z, psi, chi = case
    G = adjoint.link_gradient(DIMS, U, RHO, z, MU, psi, chi)
    k = WilsonKernel(DIMS, U, RHO)
    from oracle.krylov import multishift_cg
    from oracle.lattice import g5
    chi_p = g5(chi)
    a = multishift_cg(k.K2s, z.sigma, psi, 1e-15).x
    b = multishift_cg(k.K2s, z.sigma, k.K(chi_p), 1e-15).x
    c = -0.25 * (1 - MU)
    t1 = sum(w * adjoint.outer_T(DIMS, g5(chi_p), al) for w, al in zip(z.omega, a))
    t2 = sum(w * adjoint.outer_T(DIMS, g5(bl), k.K(al)) for w, al, bl in zip(z.omega, a, b))
    t3 = sum(w * adjoint.outer_T(DIMS, g5(k.K(bl)), al) for w, al, bl in zip(z.omega, a, b))
    assert np.allclose(G, c * (t1 - t2 - t3), rtol=0, atol=1e-13 * np.abs(G).max())
    for t in (t1, t2, t3):
        assert norm(c * t) > 1e-2 * norm(G)
