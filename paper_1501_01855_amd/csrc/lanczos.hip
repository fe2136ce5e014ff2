// sign(K) psi by the two-pass Lanczos method (the Lanczos approach to the
// matrix sign function cited in the paper's Sec. 1 after eq. 4), FP64.
//
// sign(K) = K (K^2)^{-1/2}.  On psi_perp (psi with the exactly treated low
// modes removed): pass 1 runs Lanczos on K^2 from q_1 = psi_perp/||psi_perp||
// keeping only the tridiagonal T (alpha_j, beta_j); every ten steps the
// coefficients y = ||psi_perp|| T^{-1/2} e_1 are evaluated on the host, and
// the pass stops once lambda_max ||y - y_prev|| <= eta ||psi||.  Pass 2
// repeats the recurrence with the stored alpha, beta (no inner products) to
// regenerate q_1 .. q_k and accumulates x = sum_j y_j q_j; the result is
// K x plus the low modes' exact part.  Vector work per step: two stencil
// launches and one three-term combination (pass 1 adds a dot product and a
// norm, pass 2 one axpy), independent of the number of poles.
//
// T^{-1/2} e_1 on the host: T is symmetric positive definite with its
// eigenvalues (Ritz values of K^2) inside [a^2, b^2] of the Zolotarev interval
// passed in, so 1/sqrt(t) = sum_l omega_l / (t + sigma_l) of a 32-pole
// Zolotarev approximation on [a, b] (error below 1e-15 there) and
// T^{-1/2} e_1 = sum_l omega_l (T + sigma_l)^{-1} e_1, each a tridiagonal solve.
#include <algorithm>
#include <cmath>

#include "context.h"
#include "kernels.h"
#include "ops.h"

namespace ovl {

// (T + s) z = e_1 for the symmetric tridiagonal T = tridiag(b, a, b), s > 0
// (positive definite, so the Thomas recurrence is stable).
static void tri_shift_solve(const std::vector<double> &a, const std::vector<double> &b, int k, double s,
                            std::vector<double> &z)
{
    std::vector<double> cp(k), dp(k);
    double den = a[0] + s;
    cp[0] = k > 1 ? b[0] / den : 0.0;
    dp[0] = 1.0 / den;
    for (int i = 1; i < k; ++i) {
        den = a[i] + s - b[i - 1] * cp[i - 1];
        cp[i] = i + 1 < k ? b[i] / den : 0.0;
        dp[i] = (0.0 - b[i - 1] * dp[i - 1]) / den;
    }
    z.assign(k, 0.0);
    z[k - 1] = dp[k - 1];
    for (int i = k - 2; i >= 0; --i) z[i] = dp[i] - cp[i] * z[i + 1];
}

static void inv_sqrt_e1(const ovl_zolo &zz, const std::vector<double> &a, const std::vector<double> &b, int k,
                        double scale, std::vector<double> &y)
{
    y.assign(k, 0.0);
    std::vector<double> z;
    for (int l = 0; l < zz.n_z; ++l) {
        tri_shift_solve(a, b, k, zz.sigma[l], z);
        for (int i = 0; i < k; ++i) y[i] += scale * zz.omega[l] * z[i];
    }
}

void sign_lanczos(Context &c, double rho, const ovl_zolo &z, const double2 *in, double2 *out, int nf, double eta,
                  int maxiter, ovl_stats *st)
{
    const Geom &g = c.g;
    const size_t FB = field_bytes(g, OVL_F64);
    const int64_t fs = 12 * g.V;
    double2 *perp = (double2 *)c.buf("lz_perp", FB);
    double2 *q = (double2 *)c.buf("lz_q", FB);
    double2 *qp = (double2 *)c.buf("lz_qp", FB);
    double2 *t = (double2 *)c.buf("lz_t", FB);
    double2 *w = (double2 *)c.buf("lz_w", FB);
    double2 *x = (double2 *)c.buf("lz_x", FB);
    ovl_zolo zz{};
    zolotarev(32, z.a, z.b, zz);   // 1/sqrt on [a^2, b^2], the spectrum of T
    const double lmax = z.b;
    for (int f = 0; f < nf; ++f) {
        const double2 *psi = in + f * fs;
        double2 *o = out + f * fs;
        std::vector<double> n2;
        norm2_f64(c, psi, 1, n2);
        const double psin = std::sqrt(n2[0]);
        OVL_REQUIRE(std::isfinite(psin), OVL_ERR_BREAKDOWN, "Lanczos sign: non-finite input");
        // the low modes: c_i = (v_i, psi), psi_perp = psi - sum c_i v_i
        std::vector<cplx<double>> cl;
        copy_fields(c, psi, perp, 1, OVL_F64);
        if (c.n_low > 0) {
            multidot_f64(c, c.low, c.n_low, psi, 1, cl);
            std::vector<cplx<double>> neg(cl.size());
            for (size_t i = 0; i < cl.size(); ++i) neg[i] = {-cl[i].re, -cl[i].im};
            multiaxpy_f64(c, c.low, c.n_low, neg.data(), perp, 1);
        }
        norm2_f64(c, perp, 1, n2);
        const double pn = std::sqrt(n2[0]);
        zero_fields(c, x, 1, OVL_F64);
        int k = 0;
        std::vector<double> al, be, y, yprev;
        if (pn > 0.0) {
            // pass 1
            lincomb3_f64(c, 1.0 / pn, perp, 0.0, perp, 0.0, nullptr, q, 1);
            zero_fields(c, qp, 1, OVL_F64);
            double bprev = 0.0;
            bool done = false;
            while (!done) {
                OVL_REQUIRE(k < maxiter, OVL_ERR_NOT_CONVERGED, "Lanczos sign: iteration limit");
                stencil(c, EPI_K, OVL_F64, q, t, 1, rho, 0.0, nullptr, nullptr);
                stencil(c, EPI_K, OVL_F64, t, w, 1, rho, 0.0, nullptr, nullptr);   // w = K^2 q
                std::vector<cplx<double>> d;
                dot_f64(c, q, w, 1, d);
                const double aj = d[0].re;
                lincomb3_f64(c, 1.0, w, -aj, q, -bprev, qp, t, 1);   // t = w - a q - b_prev q_prev
                norm2_f64(c, t, 1, n2);
                const double bj = std::sqrt(n2[0]);
                OVL_REQUIRE(std::isfinite(aj) && std::isfinite(bj), OVL_ERR_BREAKDOWN, "Lanczos sign: non-finite step");
                al.push_back(aj);
                be.push_back(bj);
                ++k;
                if (k % 10 == 0 || bj == 0.0) {
                    inv_sqrt_e1(zz, al, be, k, pn, y);
                    if (!yprev.empty()) {
                        double ch = 0.0;
                        for (int i = 0; i < k; ++i) {
                            const double dd = y[i] - (i < (int)yprev.size() ? yprev[i] : 0.0);
                            ch += dd * dd;
                        }
                        done = lmax * std::sqrt(ch) <= eta * psin;
                    }
                    yprev = y;
                    if (bj == 0.0) done = true;
                }
                if (!done) {
                    std::swap(qp, q);                                              // q_prev <- q
                    lincomb3_f64(c, 1.0 / bj, t, 0.0, t, 0.0, nullptr, q, 1);      // q <- t / b
                    bprev = bj;
                }
            }
            // pass 2: x = sum_j y_j q_j over the regenerated vectors
            lincomb3_f64(c, 1.0 / pn, perp, 0.0, perp, 0.0, nullptr, q, 1);
            zero_fields(c, qp, 1, OVL_F64);
            lincomb3_f64(c, y[0], q, 0.0, q, 0.0, nullptr, x, 1);
            for (int j = 0; j + 1 < k; ++j) {
                stencil(c, EPI_K, OVL_F64, q, t, 1, rho, 0.0, nullptr, nullptr);
                stencil(c, EPI_K, OVL_F64, t, w, 1, rho, 0.0, nullptr, nullptr);
                lincomb3_f64(c, 1.0 / be[j], w, -al[j] / be[j], q, -(j > 0 ? be[j - 1] : 0.0) / be[j], qp, t, 1);
                std::swap(qp, q);   // q_prev <- q_j
                std::swap(q, t);    // q <- q_{j+1}
                lincomb3_f64(c, 1.0, x, y[j + 1], q, 0.0, nullptr, w, 1);
                std::swap(x, w);
            }
        }
        stencil(c, EPI_K, OVL_F64, x, o, 1, rho, 0.0, nullptr, nullptr);           // K x
        if (c.n_low > 0) {
            std::vector<cplx<double>> ex(cl.size());
            for (int i = 0; i < c.n_low; ++i) {
                const double sg = c.low_evals[i] < 0.0 ? -1.0 : 1.0;
                ex[i] = {sg * cl[i].re, sg * cl[i].im};
            }
            multiaxpy_f64(c, c.low, c.n_low, ex.data(), o, 1);
        }
        if (st) {
            st->mscg_iters += k;
            st->dslash_calls[OVL_F64] += 4 * (int64_t)k - 1;
            st->sign_calls[OVL_F64] += 1;
        }
    }
    OVL_HIP(hipStreamSynchronize(c.stream));
    // the buffers swapped above belong to the context's pool: restore nothing
    // (each call takes them by name again)
}

}  // namespace ovl
