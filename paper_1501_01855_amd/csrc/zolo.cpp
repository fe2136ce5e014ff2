// Zolotarev optimal rational approximation to sign(x) on a <= |x| <= b
// (paper Sec. 3, eq. 7; the paper cites the literature for the formula):
//
//   k = a/b, k' = sqrt(1 - k^2), K' = K(k')
//   c_l = sn^2(l K'/(2 N_Z); k') / cn^2(l K'/(2 N_Z); k'),   l = 1 .. 2 N_Z - 1
//   R(x) = d x prod_{l<N_Z} (x^2 + k^2 c_{2l}) / prod_{l<=N_Z} (x^2 + k^2 c_{2l-1}),  x = lambda/b
//   R equioscillates at x_j = k / dn(j K'/(2 N_Z); k'), j = 0 .. 2 N_Z;
//   d makes max + min = 2 there, delta = (max - min)/(max + min);
//   sigma_l = a^2 c_{2l-1},  omega_l = b d prod_i (k^2 c_{2i} - k^2 c_{2l-1})
//                                      / prod_{i != l} (k^2 c_{2i-1} - k^2 c_{2l-1}).
//
// Elliptic functions by the arithmetic-geometric mean: K(m) = pi / (2 AGM(1,
// sqrt(1 - m))), and sn, cn, dn by the descending Landen (AGM) recurrence of
// Abramowitz & Stegun 16.4.
#include <cmath>

#include "common.h"

namespace ovl {

static double ellip_K(double m)
{
    double a = 1.0, b = std::sqrt(1.0 - m);
    for (int i = 0; i < 64 && std::fabs(a - b) > 1e-16 * a; ++i) {
        const double an = 0.5 * (a + b);
        b = std::sqrt(a * b);
        a = an;
    }
    return M_PI / (2.0 * a);
}

static void ellip_j(double u, double m, double &sn, double &cn, double &dn)
{
    if (m < 1e-300) {
        sn = std::sin(u);
        cn = std::cos(u);
        dn = 1.0;
        return;
    }
    double a[32], c[32];
    a[0] = 1.0;
    c[0] = std::sqrt(m);
    double b = std::sqrt(1.0 - m);
    int n = 0;
    while (std::fabs(c[n]) > 1e-17 * a[n] && n < 30) {
        a[n + 1] = 0.5 * (a[n] + b);
        c[n + 1] = 0.5 * (a[n] - b);
        b = std::sqrt(a[n] * b);
        ++n;
    }
    double phi = std::ldexp(a[n] * u, n);
    double phi1 = phi;
    for (int i = n; i > 0; --i) {
        phi1 = phi;
        phi = 0.5 * (phi + std::asin(c[i] * std::sin(phi) / a[i]));
    }
    sn = std::sin(phi);
    cn = std::cos(phi);
    dn = n > 0 ? cn / std::cos(phi1 - phi) : 1.0;
}

void zolotarev(int nz, double a, double b, ovl_zolo &out)
{
    OVL_REQUIRE(nz >= 1 && nz <= OVL_MAX_NZ, OVL_ERR_ARG, "n_z out of range");
    OVL_REQUIRE(a > 0.0 && b > a && std::isfinite(b), OVL_ERR_ARG, "need 0 < a < b");
    const double k = a / b;
    const double m = 1.0 - k * k;   // parameter of the complementary modulus k'
    const double Kp = ellip_K(m);
    std::vector<double> c(2 * nz);   // c[l], l = 1 .. 2 nz - 1
    for (int l = 1; l < 2 * nz; ++l) {
        double sn, cn, dn;
        ellip_j(l * Kp / (2.0 * nz), m, sn, cn, dn);
        c[l] = (sn * sn) / (cn * cn);
    }
    auto R = [&](double x) {
        double num = 1.0, den = 1.0;
        for (int l = 1; l < nz; ++l) num *= x * x + k * k * c[2 * l];
        for (int l = 1; l <= nz; ++l) den *= x * x + k * k * c[2 * l - 1];
        return x * num / den;
    };
    double rmax = -1e300, rmin = 1e300;
    for (int j = 0; j <= 2 * nz; ++j) {
        double x;
        if (j == 0) {
            x = k;
        } else if (j == 2 * nz) {
            x = 1.0;
        } else {
            double sn, cn, dn;
            ellip_j(j * Kp / (2.0 * nz), m, sn, cn, dn);
            x = k / dn;
        }
        const double r = R(x);
        rmax = std::fmax(rmax, r);
        rmin = std::fmin(rmin, r);
    }
    const double d = 2.0 / (rmax + rmin);
    out.n_z = nz;
    out.a = a;
    out.b = b;
    out.delta = (rmax - rmin) / (rmax + rmin);
    for (int l = 1; l <= nz; ++l) {
        const double ol = k * k * c[2 * l - 1];
        double num = 1.0, den = 1.0;
        for (int i = 1; i < nz; ++i) num *= k * k * c[2 * i] - ol;
        for (int i = 1; i <= nz; ++i)
            if (i != l) den *= k * k * c[2 * i - 1] - ol;
        out.omega[l - 1] = b * d * num / den;
        out.sigma[l - 1] = a * a * c[2 * l - 1];
    }
    for (int l = nz; l < OVL_MAX_NZ; ++l) {
        out.omega[l] = 0.0;
        out.sigma[l] = 0.0;
    }
}

}  // namespace ovl
