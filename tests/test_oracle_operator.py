"""Pins for the oracle's Wilson kernel (paper Sec. 1, eq. 2): facts fixed by
the mathematics, not by the oracle itself."""
import numpy as np
import pytest

import synth
from oracle.lattice import WilsonKernel, dot, g5, gamma, norm

pytestmark = pytest.mark.filterwarnings("ignore")


def test_gamma_algebra():
    g = gamma()
    eye = np.eye(4)
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)           # Hermitian
        assert np.allclose(g[mu] @ g[mu], eye)              # gamma_mu^2 = 1
        for nu in range(4):
            if nu != mu:
                assert np.allclose(g[mu] @ g[nu] + g[nu] @ g[mu], 0)
    assert np.allclose(g[4], g[0] @ g[1] @ g[2] @ g[3])
    assert np.allclose(g[4], np.diag([1, 1, -1, -1]))       # chiral basis


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 2, 4)])
def test_free_field_spectrum(dims):
    """Unit links: D_W(p) = sum(1 - cos p) - rho + i sum gamma sin p, whose
    eigenvalues are A +- i B, each six-fold (2 spin x 3 colour)."""
    rho = 1.4
    k = WilsonKernel(dims, synth.unit_gauge(dims), rho)
    ev = np.linalg.eigvals(k.dense("dw"))
    ref = []
    for n in np.ndindex(*dims):
        p = 2 * np.pi * np.array(n) / np.array(dims)
        A = np.sum(1 - np.cos(p)) - rho
        B = np.sqrt(np.sum(np.sin(p) ** 2))
        ref += [A + 1j * B] * 6 + [A - 1j * B] * 6
    key = lambda z: (round(z.real, 9), round(z.imag, 9))
    assert np.allclose(sorted(ev, key=key), sorted(np.array(ref), key=key), atol=1e-11)


def test_free_field_plane_wave():
    """D_W e^{ipx} chi = [sum(1 - cos p) - rho + i sum_mu gamma_mu sin p_mu] chi e^{ipx}
    on a lattice with four different extents (catches axis and sign mix-ups)."""
    dims = (4, 6, 2, 8)
    rho = 1.4
    k = WilsonKernel(dims, synth.unit_gauge(dims), rho)
    g = gamma()
    rng = np.random.default_rng(0)
    chi = rng.normal(size=(4, 3)) + 1j * rng.normal(size=(4, 3))
    coords = np.array(list(np.ndindex(*dims[::-1])))[:, ::-1]   # x fastest
    for n in [(1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1), (1, 2, 1, 3)]:
        p = 2 * np.pi * np.array(n) / np.array(dims)
        phase = np.exp(1j * coords @ p)
        psi = phase[:, None, None] * chi[None]
        M = (np.sum(1 - np.cos(p)) - rho) * np.eye(4) + 1j * sum(g[m] * np.sin(p[m]) for m in range(4))
        ref = phase[:, None, None] * (M @ chi)[None]
        assert np.allclose(k.dw(psi), ref, atol=1e-12)


def _random_kernel(dims=(4, 2, 2, 4), seed=3, eps=0.5):
    return WilsonKernel(dims, synth.gauge_field(dims, seed, eps), 1.4)


def test_gamma5_hermiticity():
    """D_W^dagger = gamma_5 D_W gamma_5, so K = gamma_5 D_W is Hermitian (Sec. 1)."""
    k = _random_kernel()
    Dw = k.dense("dw")
    G5 = np.kron(np.eye(k.V), np.kron(np.diag([1, 1, -1, -1]), np.eye(3)))
    assert np.allclose(Dw.conj().T, G5 @ Dw @ G5, atol=1e-13)
    Kd = k.dense("K")
    assert np.allclose(Kd, Kd.conj().T, atol=1e-13)


def test_gauge_covariance():
    """U_mu(x) -> g(x) U_mu(x) g(x+mu)^dagger, psi -> g psi gives D_W psi -> g D_W psi."""
    dims = (4, 2, 6, 2)
    V = int(np.prod(dims))
    U = synth.gauge_field(dims, 5, 0.7)
    gx = synth.gauge_field(dims, 6, 1.0)[:, 0]          # one random SU(3) per site
    coords = np.array(list(np.ndindex(*dims[::-1])))[:, ::-1]
    def idx(c):
        c = c % np.array(dims)
        return c[:, 0] + dims[0] * (c[:, 1] + dims[1] * (c[:, 2] + dims[2] * c[:, 3]))
    Ug = np.empty_like(U)
    for mu in range(4):
        e = np.zeros(4, int)
        e[mu] = 1
        fwd = idx(coords + e)
        Ug[:, mu] = gx @ U[:, mu] @ gx[fwd].conj().transpose(0, 2, 1)
    psi = synth.gaussian_source(dims, 7)
    psig = np.einsum("xab,xsb->xsa", gx, psi)
    out = WilsonKernel(dims, U, 1.4).dw(psi)
    outg = WilsonKernel(dims, Ug, 1.4).dw(psig)
    assert np.allclose(outg, np.einsum("xab,xsb->xsa", gx, out), atol=1e-12)


def test_norm_bound():
    """||D_W(-rho)|| <= 8 - rho for unitary links (each hop pair has norm <= 1)."""
    k = _random_kernel()
    lam = np.linalg.eigvalsh(k.dense("K"))
    assert np.abs(lam).max() <= 8 - 1.4 + 1e-12


def test_sampled_sites_match_full():
    dims = (4, 4, 2, 6)
    k = WilsonKernel(dims, synth.gauge_field(dims, 9, 0.3), 1.4)
    psi = synth.gaussian_source(dims, 1)
    sites = np.array([0, 1, 17, 100, k.V - 1])
    assert np.array_equal(k.K_sites(psi, sites), k.K(psi)[sites])
