"""Oracle: Zolotarev optimal rational approximation to sign(x).

TEST INFRASTRUCTURE ONLY.

Paper Sec. 3, eq. 7: eps(x) = sum_{l=1}^{N_Z} omega_l x / (x^2 + sigma_l), with
|eps| oscillating between 1 - Delta and 1 + Delta for a < |x| < b; the paper
states that the coefficients and Delta follow from Jacobi elliptic functions
of N_Z, a and b, and cites the literature for the formula.  The formula used
here (Zolotarev's solution in product form, then partial fractions):

  k = a/b, k' = sqrt(1 - k^2), K' = K(k')  (complete elliptic integral)
  c_l = sn^2(l K'/(2 N_Z); k') / cn^2(l K'/(2 N_Z); k'),  l = 1 .. 2 N_Z - 1
  R(x) = d x prod_{l=1}^{N_Z-1} (x^2 + k^2 c_{2l}) / prod_{l=1}^{N_Z} (x^2 + k^2 c_{2l-1})
         for x = lambda / b in [k, 1]
  d chosen so that max R + min R = 2 on [k, 1];  Delta = (max - min)/(max + min)
  sigma_l = a^2 c_{2l-1},
  omega_l = b d prod_i (k^2 c_{2i} - k^2 c_{2l-1}) / prod_{i != l} (k^2 c_{2i-1} - k^2 c_{2l-1})

The Jacobi elliptic functions are SciPy's (which take the parameter m = k'^2).
max and min of R on [k, 1] are taken over its alternation points
x_j = k / dn(j K'/(2 N_Z); k'); the tests check on a dense grid that R has no
larger excursion anywhere else.
"""
import numpy as np
from scipy.special import ellipj, ellipk


def _c_coeffs(nz, k):
    kp2 = 1.0 - k * k
    Kp = ellipk(kp2)
    l = np.arange(1, 2 * nz)
    sn, cn, _, _ = ellipj(l * Kp / (2 * nz), kp2)
    return (sn * sn) / (cn * cn)          # c_1 .. c_{2 nz - 1}


def product_form(x, nz, k, d=1.0):
    """R(x) in the product form above (x = lambda / b)."""
    c = _c_coeffs(nz, k)
    x = np.asarray(x, dtype=np.float64)
    num = np.ones_like(x)
    den = np.ones_like(x)
    for l in range(1, nz):
        num = num * (x * x + k * k * c[2 * l - 1])      # c_{2l}
    for l in range(1, nz + 1):
        den = den * (x * x + k * k * c[2 * l - 2])      # c_{2l-1}
    return d * x * num / den


def alternation_points(nz, k):
    """x_j = k / dn(j K'/(2 N_Z); k'), j = 0 .. 2 N_Z: the 2 N_Z + 1 points of
    [k, 1] (both end points included) where Zolotarev's R(x) takes its
    extreme values, alternately 1 - Delta and 1 + Delta."""
    kp2 = 1.0 - k * k
    Kp = ellipk(kp2)
    j = np.arange(0, 2 * nz + 1)
    _, _, dn, _ = ellipj(j * Kp / (2 * nz), kp2)
    x = k / dn
    x[0], x[-1] = k, 1.0
    return x


class Zolotarev:
    """Coefficients {N_Z, a, b, omega_l, sigma_l, Delta} (paper Sec. 3, eq. 7)."""

    def __init__(self, nz, a, b):
        assert nz >= 1 and 0.0 < a < b
        self.nz, self.a, self.b = int(nz), float(a), float(b)
        k = a / b
        self.k = k
        c = _c_coeffs(nz, k)
        self.c = c
        vals = product_form(alternation_points(nz, k), nz, k)
        rmax, rmin = vals.max(), vals.min()
        self.d = 2.0 / (rmax + rmin)
        self.delta = (rmax - rmin) / (rmax + rmin)
        odd = k * k * c[0::2]        # k^2 c_{2l-1}, l = 1..nz
        even = k * k * c[1::2]       # k^2 c_{2l},   l = 1..nz-1
        omega = np.empty(nz)
        for l in range(nz):
            num = np.prod(even - odd[l])
            den = np.prod(np.delete(odd, l) - odd[l])
            omega[l] = b * self.d * num / den
        self.omega = omega
        self.sigma = a * a * c[0::2]

    def __call__(self, lam):
        """eps(lambda) = lambda sum_l omega_l / (lambda^2 + sigma_l)."""
        lam = np.asarray(lam, dtype=np.float64)
        out = np.zeros_like(lam)
        for w, s in zip(self.omega, self.sigma):
            out = out + w / (lam * lam + s)
        return lam * out

    def product(self, lam):
        lam = np.asarray(lam, dtype=np.float64)
        return product_form(lam / self.b, self.nz, self.k, self.d)

    def extrema(self):
        """(locations, values) of eps at its 2 N_Z + 1 alternation points in [a, b]."""
        x = alternation_points(self.nz, self.k)
        return x * self.b, product_form(x, self.nz, self.k, self.d)
