// Kernel low modes: the n_low eigenpairs of K with the smallest |lambda|,
// which the sign function treats exactly (paper Sec. 1 after eq. 4; Sec. 3:
// a^2 is the largest squared eigenvalue so deflated).  Set-up work, once per
// gauge field.
//
// Method: Chebyshev-filtered subspace iteration (Zhou & Saad) on K^2 in FP64
// with a block of nb > n_low vectors.  Each sweep applies the degree-m
// Chebyshev polynomial that damps [a_cut, b_up] of the K^2 spectrum
// (b_up = (8 - rho)^2 bounds it for unitary links, a_cut is the largest Ritz
// value of the block), orthonormalises the block by Cholesky QR (twice), and
// does a Rayleigh-Ritz step with K^2 (whose wanted eigenvalues are the
// smallest of a positive spectrum; a Rayleigh-Ritz step with the indefinite K
// would produce spurious Ritz values inside its spectral gap).  Once the
// leading K^2 pairs have converged, K is diagonalised inside their span to
// obtain eigenvectors of K with signed eigenvalues.  The multi-field stencil
// applies K to the whole block in one launch.  Stops when every wanted pair
// has ||K v - lambda v|| <= tol.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "context.h"
#include "dense.h"
#include "kernels.h"
#include "ops.h"

namespace ovl {

using dense::zc;

static void applyK(Context &c, double rho, const double2 *X, double2 *Y, int nb)
{
    stencil(c, EPI_K, OVL_F64, X, Y, nb, rho, 0.0, nullptr, nullptr);
}

// G[i][j] = (X_i, Y_j), nx x ny
static std::vector<zc> gram(Context &c, const double2 *X, int nx, const double2 *Y, int ny)
{
    std::vector<cplx<double>> d;
    gram_f64(c, X, nx, Y, ny, false, d);
    std::vector<zc> G(d.size());
    for (size_t i = 0; i < d.size(); ++i) G[i] = zc(d[i].re, d[i].im);
    return G;
}

// Z_k = sum_j W[j][k] Y_j, W is nY x nZ
static void rotate(Context &c, const double2 *Y, int nY, const std::vector<zc> &W, double2 *Z, int nZ)
{
    std::vector<cplx<double>> w(W.size());
    for (size_t i = 0; i < W.size(); ++i) w[i] = {W[i].real(), W[i].imag()};
    rotate_f64(c, Y, nY, w, nZ, Z, 0.0);
}

// Y <- Y R^{-1} with Y^H Y = R^H R (into Q), twice for orthogonality to rounding.
static void chol_qr(Context &c, double2 *Y, double2 *Q, int nb)
{
    for (int pass = 0; pass < 2; ++pass) {
        const std::vector<zc> G = gram(c, Y, nb, Y, nb);
        std::vector<zc> R;
        OVL_REQUIRE(dense::cholesky_upper(nb, G, R), OVL_ERR_BREAKDOWN,
                    "low-mode block lost rank (Cholesky QR failed)");
        rotate(c, Y, nb, dense::inv_upper(nb, R), Q, nb);
        copy_fields(c, Q, Y, nb, OVL_F64);
    }
}

void lowmodes_compute(Context &c, double rho, int n_low, double tol, double *evals, double *lmax)
{
    const Geom &g = c.g;
    const size_t FB = field_bytes(g, OVL_F64);
    // a block well beyond n_low: synthetic near-unit gauge fields have
    // clusters of dozens of almost degenerate low modes (the doublers)
    const int nb = (int)std::min<int64_t>(n_low + std::max(48, n_low), 12 * g.V - 1);
    OVL_REQUIRE(n_low < nb, OVL_ERR_ARG, "n_low too large for this lattice");
    double2 *X = (double2 *)c.buf("lm_X", FB * nb);
    double2 *Y = (double2 *)c.buf("lm_Y", FB * nb);
    double2 *Z = (double2 *)c.buf("lm_Z", FB * nb);
    double2 *T = (double2 *)c.buf("lm_T", FB * nb);
    double2 *T2 = (double2 *)c.buf("lm_T2", FB * nb);
    double *canon = (double *)c.buf("lm_canon", FB);
    for (int i = 0; i < nb; ++i) {
        source_generate(c, OVL_SRC_GAUSS, 0x5EED0000ull + (uint64_t)i, 0, 0, 0, canon);
        pack_spinor(c, canon, X + (size_t)i * 12 * g.V, 1, OVL_F64);
    }
    const double b_up = (8.0 - rho) * (8.0 - rho) * 1.0001;
    const int degree = 32;
    double a_cut = 0.0;
    bool converged = false;
    std::vector<double> theta;
    for (int sweep = 0; sweep < 200 && !converged; ++sweep) {
        if (sweep > 0) {
            // Chebyshev filter of K^2 damping [a_cut, b_up] (scaled three-term recurrence)
            const double e = 0.5 * (b_up - a_cut), cc = 0.5 * (b_up + a_cut);
            double sigma = e / (0.0 - cc);
            const double tau = 2.0 / sigma;
            applyK(c, rho, X, T2, nb);
            applyK(c, rho, T2, T, nb);                      // T = K^2 X
            lincomb3_f64(c, sigma / e, T, -cc * sigma / e, X, 0.0, nullptr, Y, nb);
            for (int i = 2; i <= degree; ++i) {
                const double sn = 1.0 / (tau - sigma);
                applyK(c, rho, Y, T2, nb);
                applyK(c, rho, T2, T, nb);                  // T = K^2 Y
                lincomb3_f64(c, 2.0 * sn / e, T, -2.0 * sn * cc / e, Y, -sigma * sn, X, Z, nb);
                std::swap(X, Y);                            // X <- Y
                std::swap(Y, Z);                            // Y <- Y_new
                sigma = sn;
            }
            copy_fields(c, Y, X, nb, OVL_F64);
        }
        chol_qr(c, X, Z, nb);
        // Rayleigh-Ritz with K^2 (the wanted end of a positive spectrum)
        applyK(c, rho, X, T, nb);                           // T  = K X
        applyK(c, rho, T, T2, nb);                          // T2 = K^2 X
        std::vector<double> w2;
        std::vector<zc> W;
        dense::eigh(nb, gram(c, X, nb, T2, nb), w2, W);
        rotate(c, X, nb, W, Y, nb);
        rotate(c, T, nb, W, Z, nb);
        rotate(c, T2, nb, W, T, nb);
        std::swap(X, Y);            // X: Ritz vectors of K^2
        std::swap(T, Z);            // T: K X ; Z: K^2 X
        int nc = 0;                 // leading converged K^2 pairs
        while (nc < nb) {
            lincomb3_f64(c, 1.0, Z + (size_t)nc * 12 * g.V, -w2[nc], X + (size_t)nc * 12 * g.V, 0.0, nullptr, T2, 1);
            std::vector<double> n2;
            norm2_f64(c, T2, 1, n2);
            if (!(std::sqrt(n2[0]) <= tol * std::max(1.0, w2[nc]))) break;
            ++nc;
        }
        a_cut = std::min(w2[nb - 1], 0.5 * b_up);
        if (nc < n_low) continue;
        // eigenvectors of K inside the converged K^2 subspace (signs of lambda)
        std::vector<double> th;
        std::vector<zc> Wk;
        dense::eigh(nc, gram(c, X, nc, T, nc), th, Wk);
        std::vector<int> ord(nc);
        std::iota(ord.begin(), ord.end(), 0);
        std::sort(ord.begin(), ord.end(), [&](int a, int b) { return std::fabs(th[a]) < std::fabs(th[b]); });
        std::vector<zc> Wo((size_t)nc * n_low);
        theta.assign(n_low, 0.0);
        for (int k = 0; k < n_low; ++k) {
            theta[k] = th[ord[k]];
            for (int j = 0; j < nc; ++j) Wo[(size_t)j * n_low + k] = Wk[(size_t)j * nc + ord[k]];
        }
        rotate(c, X, nc, Wo, Y, n_low);
        rotate(c, T, nc, Wo, T2, n_low);
        double worst = 0.0;
        for (int k = 0; k < n_low; ++k) {
            lincomb3_f64(c, 1.0, T2 + (size_t)k * 12 * g.V, -theta[k], Y + (size_t)k * 12 * g.V, 0.0, nullptr,
                         Z + (size_t)k * 12 * g.V, 1);
            std::vector<double> n2;
            norm2_f64(c, Z + (size_t)k * 12 * g.V, 1, n2);
            worst = std::max(worst, std::sqrt(n2[0]));
        }
        converged = worst <= tol;
    }
    OVL_REQUIRE(converged, OVL_ERR_NOT_CONVERGED, "low-mode eigensolver did not reach its tolerance");
    c.lowmodes_changed();
    if (c.low) {
        OVL_HIP(hipStreamSynchronize(c.stream));
        OVL_HIP(hipFree(c.low));
        c.bytes_held -= (int64_t)FB * c.n_low;
        c.low = nullptr;
    }
    OVL_HIP(hipMalloc(&c.low, FB * n_low));
    c.bytes_held += (int64_t)FB * n_low;
    copy_fields(c, Y, c.low, n_low, OVL_F64);
    c.n_low = n_low;
    c.low_evals = theta;
    OVL_HIP(hipStreamSynchronize(c.stream));
    if (evals)
        for (int k = 0; k < n_low; ++k) evals[k] = theta[k];
    if (lmax) *lmax = 8.0 - rho;
}

}  // namespace ovl

namespace ovl {

// Symmetric tridiagonal T (diagonal a[0..n), off-diagonal b[0..n-1)): the
// number of eigenvalues below x by the Sturm sequence of the LDL^T pivots.
static int sturm_below(const std::vector<double> &a, const std::vector<double> &b, int n, double x)
{
    int cnt = 0;
    double d = 1.0;
    for (int i = 0; i < n; ++i) {
        d = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / d : 0.0);
        if (d == 0.0) d = -1e-300;
        if (d < 0.0) ++cnt;
    }
    return cnt;
}

// The k-th smallest eigenvalue of T by bisection inside its Gershgorin bounds.
static double tri_eig(const std::vector<double> &a, const std::vector<double> &b, int n, int k)
{
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < n; ++i) {
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(std::fabs(lo), std::fabs(hi)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (sturm_below(a, b, n, mid) > k) hi = mid;
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}

// |last component| of the unit eigenvector of T for eigenvalue th, by two
// steps of inverse iteration (tridiagonal solves with partial pivoting).
static double tri_evec_last(const std::vector<double> &a, const std::vector<double> &b, int n, double th)
{
    std::vector<double> y(n, 1.0 / std::sqrt((double)n));
    const double shift = th * (1.0 - 1e-13) - 1e-300;
    for (int pass = 0; pass < 2; ++pass) {
        // Gaussian elimination on (T - shift) z = y, rows i, i+1 swapped when needed
        std::vector<double> d(n), u(n, 0.0), w(n, 0.0), r = y;
        for (int i = 0; i < n; ++i) d[i] = a[i] - shift;
        std::vector<double> lo(n > 0 ? n - 1 : 0);
        for (int i = 0; i + 1 < n; ++i) {
            u[i] = b[i];
            lo[i] = b[i];
        }
        // U has diagonal d, superdiagonals u, w (from pivoting)
        for (int i = 0; i + 1 < n; ++i) {
            if (std::fabs(lo[i]) > std::fabs(d[i])) {   // swap rows i and i+1
                std::swap(d[i], lo[i]);
                const double t1 = u[i];
                u[i] = d[i + 1];
                d[i + 1] = t1;
                if (i + 2 < n) {
                    w[i] = u[i + 1];
                    u[i + 1] = 0.0;
                }
                std::swap(r[i], r[i + 1]);
            }
            const double m = d[i] != 0.0 ? lo[i] / d[i] : 0.0;
            d[i + 1] -= m * u[i];
            if (i + 2 < n) u[i + 1] -= m * w[i];
            r[i + 1] -= m * r[i];
        }
        std::vector<double> z(n);
        for (int i = n - 1; i >= 0; --i) {
            double t = r[i];
            if (i + 1 < n) t -= u[i] * z[i + 1];
            if (i + 2 < n) t -= w[i] * z[i + 2];
            z[i] = t / (d[i] != 0.0 ? d[i] : 1e-300);
        }
        double nn = 0.0;
        for (double v : z) nn += v * v;
        nn = std::sqrt(nn);
        for (int i = 0; i < n; ++i) y[i] = z[i] / nn;
    }
    return std::fabs(y[n - 1]);
}

// Ends of the spectrum of K^2 by Lanczos (FP64, one vector, no
// re-orthogonalisation: the extreme Ritz values converge regardless, and
// the smallest one decreases monotonically towards lambda_min^2).  Set-up
// for the Zolotarev interval when no kernel modes are treated exactly.
// Every ten steps the extreme eigenvalues of the tridiagonal matrix are
// found by bisection; the run stops when the smallest has moved by less than
// 1e-10 (relative) over two such checks.
void kernel_interval(Context &c, double rho, int max_iter, double *lmin, double *lmin_err, double *lmax)
{
    const Geom &g = c.g;
    const size_t FB = field_bytes(g, OVL_F64);
    double2 *v = (double2 *)c.buf("li_v", FB);
    double2 *vp = (double2 *)c.buf("li_vp", FB);
    double2 *w = (double2 *)c.buf("li_w", FB);
    double2 *t = (double2 *)c.buf("li_t", FB);
    double *canon = (double *)c.buf("lm_canon", FB);
    source_generate(c, OVL_SRC_GAUSS, 0x5EED1A00ull, 0, 0, 0, canon);
    pack_spinor(c, canon, t, 1, OVL_F64);
    std::vector<double> n2;
    norm2_f64(c, t, 1, n2);
    lincomb3_f64(c, 1.0 / std::sqrt(n2[0]), t, 0.0, t, 0.0, nullptr, v, 1);
    zero_fields(c, vp, 1, OVL_F64);   // read (times 0) by the first step
    std::vector<double> alpha, beta;   // T = tridiag(beta, alpha, beta)
    double bprev = 0.0, th_min = 0.0, th_max = 0.0, last = -1.0;
    int stable = 0;
    for (int j = 0; j < max_iter; ++j) {
        stencil(c, EPI_K, OVL_F64, v, t, 1, rho, 0.0, nullptr, nullptr);
        stencil(c, EPI_K, OVL_F64, t, w, 1, rho, 0.0, nullptr, nullptr);   // w = K^2 v
        std::vector<cplx<double>> d;
        dot_f64(c, v, w, 1, d);
        const double a = d[0].re;
        lincomb3_f64(c, 1.0, w, -a, v, -bprev, vp, t, 1);                  // t = w - a v - b_prev v_prev
        norm2_f64(c, t, 1, n2);
        const double b = std::sqrt(n2[0]);
        alpha.push_back(a);
        beta.push_back(b);
        const int n = (int)alpha.size();
        if (n % 10 == 0 || j == max_iter - 1 || b == 0.0) {
            th_min = tri_eig(alpha, beta, n, 0);
            th_max = tri_eig(alpha, beta, n, n - 1);
            if (last > 0.0 && std::fabs(last - th_min) <= 1e-10 * th_min) ++stable;
            else stable = 0;
            last = th_min;
            if (stable >= 2 || b == 0.0) break;
        }
        std::swap(vp, v);                                                  // v_prev <- v
        lincomb3_f64(c, 1.0 / b, t, 0.0, t, 0.0, nullptr, v, 1);           // v <- t / b
        bprev = b;
    }
    OVL_HIP(hipStreamSynchronize(c.stream));
    const int n = (int)alpha.size();
    *lmin = std::sqrt(std::max(th_min, 0.0));
    if (lmin_err) *lmin_err = beta[n - 1] * tri_evec_last(alpha, beta, n, th_min);   // |beta_n y_n|
    if (lmax) *lmax = std::sqrt(std::max(th_max, 0.0));
}

}  // namespace ovl
