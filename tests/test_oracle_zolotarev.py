"""Pins for the oracle's Zolotarev coefficients (paper Sec. 3, eq. 7)."""
import numpy as np
import pytest

from oracle.zolotarev import Zolotarev


@pytest.mark.parametrize("nz,ratio", [(2, 100.0), (3, 30.0), (6, 100.0), (8, 300.0), (12, 1000.0)])
def test_equioscillation(nz, ratio):
    """Optimality (Chebyshev alternation): |eps| - 1 takes the values -+Delta
    alternately at 2 N_Z + 1 points of [a, b], and nowhere exceeds Delta."""
    z = Zolotarev(nz, 1.0, ratio)
    locs, vals = z.extrema()
    dev = vals - 1.0
    assert len(dev) == 2 * nz + 1
    assert np.allclose(np.abs(dev), z.delta, rtol=1e-6, atol=1e-15)
    assert np.all(np.sign(dev[1:]) == -np.sign(dev[:-1]))
    x = np.exp(np.linspace(0.0, np.log(ratio), 20001))
    assert np.max(np.abs(z(x) - 1.0)) <= z.delta * (1 + 1e-6) + 1e-15


def test_nz1_closed_form():
    """N_Z = 1: eps(x) = w x/(x^2 + s) equioscillates at a, sqrt(s), b only if s = a b."""
    a, b = 0.3, 5.0
    z = Zolotarev(1, a, b)
    assert z.sigma[0] == pytest.approx(a * b, rel=1e-13)
    assert z(a) == pytest.approx(z(b), rel=1e-13)


@pytest.mark.parametrize("nz,a,b", [(16, 0.5, 6.6), (20, 0.05, 6.6), (8, 1.0, 10.0)])
def test_partial_fractions(nz, a, b):
    z = Zolotarev(nz, a, b)
    assert np.all(z.omega > 0) and np.all(z.sigma > 0)
    x = np.exp(np.linspace(np.log(a) - 1, np.log(b) + 1, 3001))
    assert np.allclose(z(x), z.product(x), rtol=1e-12, atol=0)
    assert np.allclose(z(-x), -z(x))                      # odd in x


def test_order_for_double_precision():
    """N_Z ~ 20 gives the sign function to double precision (Sec. 3)."""
    assert Zolotarev(20, 1.0, 100.0).delta < 1e-12
    deltas = [Zolotarev(n, 1.0, 100.0).delta for n in (4, 8, 12, 16)]
    assert all(d2 < d1 for d1, d2 in zip(deltas, deltas[1:]))
