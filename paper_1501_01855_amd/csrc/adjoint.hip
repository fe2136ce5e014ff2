// Derivatives of S = sum_f Re(chi_f^H D[mu] psi_f) with respect to psi and to
// the links, for D[mu] with the rational sign function
//   eps(K) = K sum_l omega_l X_l,  X_l = (K^2 + sigma_l)^{-1}
// (Sec. 1 eqs. 1, 2, 4 and Sec. 3 eq. 7; the exactly treated low modes are not
// differentiated, so the context must hold none).  Gradients are d/dRe + i d/dIm,
// each link entry an independent complex variable:
//   dS/dpsi = gamma_5 D gamma_5 chi
//   dS/dU_mu(y) = -(1 - mu)/4 sum_l omega_l [T(chi', a_l) - T(b_l, K a_l) - T(K b_l, a_l)]
// with chi' = gamma_5 chi, a_l = X_l psi, b_l = X_l K chi' (from
// dX_l = -X_l (dK K + K dK) X_l and dK = -gamma_5 dH / 2), and for spinor fields
// (alpha, beta) the colour matrix on link (y, mu)
//   T(alpha, beta)_ab = sum_{t=0,1} [ (P+ alpha(y))_ta conj((P- beta(y+mu))_tb)
//                                   + (P+ beta(y))_ta conj((P- alpha(y+mu))_tb) ],
// where P-+ psi = psi_up -+ A_mu psi_down is the upper half of (1 -+ gamma_mu) psi.
// The lower half of (1 -+ gamma_mu) psi is a unitary image of the upper one,
// so the two-spin sum equals the four-spin contraction of the definition.
//
// Cost: two multi-shift solves that keep every shifted solution, 2 N_Z kernel
// applications and one pass of the force kernel below.
#include "context.h"
#include "fields.h"
#include "kernels.h"
#include "mscg_state.h"
#include "ops.h"

namespace ovl {

struct ForceCoef {
    double w[NZMAX];   // -(1 - mu)/4 omega_l
};

// h = psi_up + A psi_down (PLUS) or psi_up - A psi_down
template <int MU, bool PLUS, typename R>
__device__ __forceinline__ void half_proj(const cplx<R> v[12], cplx<R> h[6])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cplx<R> a0, a1;
        apply_A<MU>(v[6 + c], v[9 + c], a0, a1);
        if constexpr (PLUS) {
            h[c] = v[c] + a0;
            h[3 + c] = v[3 + c] + a1;
        } else {
            h[c] = v[c] - a0;
            h[3 + c] = v[3 + c] - a1;
        }
    }
}

// acc_ab += w sum_t x_ta conj(y_tb)
template <typename R>
__device__ __forceinline__ void outer_acc(double w, const cplx<R> x[6], const cplx<R> y[6], cplx<double> acc[9])
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const cplx<R> t = cmul_conj(y[b], x[a]) + cmul_conj(y[3 + b], x[3 + a]);
            acc[a * 3 + b].re += w * (double)t.re;
            acc[a * 3 + b].im += w * (double)t.im;
        }
}

template <int MU, typename ST>
__device__ __forceinline__ void force_dir(const ST *chip, const ST *a, const ST *b, const ST *ka, const ST *kb,
                                          int64_t lstride, const ForceCoef &k, int nz, int64_t V, int64_t s,
                                          int64_t sf, double2 *__restrict__ G, bool accumulate)
{
    using R = typename Planes<ST>::R;
    cplx<double> acc[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) acc[i] = {0.0, 0.0};
    cplx<R> v[12], cp[6], cm[6];
    ld_sp(chip, V, s, v);
    half_proj<MU, true>(v, cp);    // P+ chi'(y)
    ld_sp(chip, V, sf, v);
    half_proj<MU, false>(v, cm);   // P- chi'(y+mu)
    for (int l = 0; l < nz; ++l) {
        const double w = k.w[l];
        const int64_t o = l * lstride;
        cplx<R> ap[6], am[6], xp[6], xm[6];
        ld_sp(a + o, V, s, v);
        half_proj<MU, true>(v, ap);    // P+ a_l(y)
        ld_sp(a + o, V, sf, v);
        half_proj<MU, false>(v, am);   // P- a_l(y+mu)
        ld_sp(kb + o, V, s, v);
        half_proj<MU, true>(v, xp);    // P+ K b_l(y)
        ld_sp(kb + o, V, sf, v);
        half_proj<MU, false>(v, xm);   // P- K b_l(y+mu)
        // T(chi', a_l) - T(K b_l, a_l) = (P+ chi' - P+ K b_l) (x) P- a_l + P+ a_l (x) (P- chi' - P- K b_l)
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            xp[c] = cp[c] - xp[c];
            xm[c] = cm[c] - xm[c];
        }
        outer_acc(w, xp, am, acc);
        outer_acc(w, ap, xm, acc);
        // - T(b_l, K a_l)
        ld_sp(b + o, V, s, v);
        half_proj<MU, true>(v, xp);    // P+ b_l(y)
        ld_sp(ka + o, V, sf, v);
        half_proj<MU, false>(v, am);   // P- K a_l(y+mu)
        outer_acc(-w, xp, am, acc);
        ld_sp(ka + o, V, s, v);
        half_proj<MU, true>(v, ap);    // P+ K a_l(y)
        ld_sp(b + o, V, sf, v);
        half_proj<MU, false>(v, xm);   // P- b_l(y+mu)
        outer_acc(-w, ap, xm, acc);
    }
    double2 *g = G + (s * 4 + MU) * 9;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        double2 o = make_double2(acc[i].re, acc[i].im);
        if (accumulate) {
            const double2 p = g[i];
            o.x += p.x;
            o.y += p.y;
        }
        g[i] = o;
    }
}

// One thread per site, all four link directions; G canonical [V][4][3][3].
// Field arguments point at the field of one right-hand side; shift l of
// a, b, ka, kb is lstride elements further on.
template <typename ST>
__global__ __launch_bounds__(256) void k_link_force(const ST *__restrict__ chip, const ST *__restrict__ a,
                                                    const ST *__restrict__ b, const ST *__restrict__ ka,
                                                    const ST *__restrict__ kb, int64_t lstride, ForceCoef k, int nz,
                                                    Geom g, double2 *__restrict__ G, int accumulate)
{
    const int64_t V = g.V;
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= V) return;
    int32_t co[4];
    int64_t r = s;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        co[m] = (int32_t)(r % g.L[m]);
        r /= g.L[m];
    }
    co[3] = (int32_t)r;
    int64_t sf[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) sf[m] = co[m] + 1 == g.L[m] ? s - (int64_t)(g.L[m] - 1) * g.stride[m] : s + g.stride[m];
    force_dir<0>(chip, a, b, ka, kb, lstride, k, nz, V, s, sf[0], G, accumulate != 0);
    force_dir<1>(chip, a, b, ka, kb, lstride, k, nz, V, s, sf[1], G, accumulate != 0);
    force_dir<2>(chip, a, b, ka, kb, lstride, k, nz, V, s, sf[2], G, accumulate != 0);
    force_dir<3>(chip, a, b, ka, kb, lstride, k, nz, V, s, sf[3], G, accumulate != 0);
}

template <typename ST>
static void link_force_t(Context &c, double rho, double mu, const ovl_zolo &z, const void *psi, const void *chip,
                         double2 *dU, int nf, double eta, int prec, int maxiter, ovl_stats *st)
{
    const Geom &g = c.g;
    const int nz = z.n_z;
    const size_t FB = field_bytes(g, prec);
    const int64_t fs = fstride<ST>(g.V);   // elements of ST per field
    ST *t = (ST *)c.buf("adj_t", FB * nf);
    ST *xa = (ST *)c.buf("adj_xa", FB * nf * nz);
    ST *xb = (ST *)c.buf("adj_xb", FB * nf * nz);
    ST *ka = (ST *)c.buf("adj_ka", FB * nf * nz);
    ST *kb = (ST *)c.buf("adj_kb", FB * nf * nz);
    std::vector<double> e(nf, eta);
    stencil(c, EPI_K, prec, chip, t, nf, rho, 0.0, nullptr, nullptr);   // K chi'
    shifts_mscg(c, rho, z, psi, xa, nf, e.data(), prec, maxiter, st);   // a_l = X_l psi
    shifts_mscg(c, rho, z, t, xb, nf, e.data(), prec, maxiter, st);     // b_l = X_l K chi'
    stencil(c, EPI_K, prec, xa, ka, nf * nz, rho, 0.0, nullptr, nullptr);
    stencil(c, EPI_K, prec, xb, kb, nf * nz, rho, 0.0, nullptr, nullptr);
    if (st) st->dslash_calls[prec] += nf * (1 + 2 * nz);
    ForceCoef k{};
    for (int l = 0; l < nz; ++l) k.w[l] = -0.25 * (1.0 - mu) * z.omega[l];
    const int64_t lstride = (int64_t)nf * fs;
    for (int f = 0; f < nf; ++f) {
        const int64_t o = (int64_t)f * fs;
        k_link_force<ST><<<site_blocks(g), 256, 0, c.stream>>>((const ST *)chip + o, xa + o, xb + o, ka + o, kb + o,
                                                              lstride, k, nz, g, dU, f > 0);
        OVL_HIP(hipGetLastError());
    }
}

void overlap_adjoint(Context &c, double rho, double mu, const ovl_zolo &z, const double2 *psi, const double2 *chi,
                     double2 *dpsi, double2 *dU, int nf, double eta, int prec, int maxiter, ovl_stats *st)
{
    OVL_REQUIRE(c.n_low == 0, OVL_ERR_UNSUPPORTED,
                "the derivative of the exact low-mode part is not provided; remove the low modes first");
    OVL_REQUIRE(prec == OVL_F64 || prec == OVL_F32, OVL_ERR_UNSUPPORTED, "the adjoint runs in FP64 or FP32");
    const size_t FB64 = field_bytes(c.g, OVL_F64) * nf;
    double2 *chip = (double2 *)c.buf("adj_chip", FB64);
    copy_fields(c, chi, chip, nf, OVL_F64);
    gamma5_f64(c, chip, nf);   // chi' = gamma_5 chi
    if (dpsi) {                // D^dagger chi = gamma_5 D chi'
        overlap_f64(c, rho, mu, z, chip, dpsi, nf, eta, prec, maxiter, st);
        gamma5_f64(c, dpsi, nf);
    }
    if (!dU) return;
    if (prec == OVL_F64) {
        link_force_t<double2>(c, rho, mu, z, psi, chip, dU, nf, eta, prec, maxiter, st);
    } else {
        const size_t FB = field_bytes(c.g, prec) * nf;
        void *p32 = c.buf("adj_psi32", FB);
        void *c32 = c.buf("adj_chi32", FB);
        convert_spinor(c, psi, OVL_F64, p32, prec, nf);
        convert_spinor(c, chip, OVL_F64, c32, prec, nf);
        link_force_t<float4>(c, rho, mu, z, p32, c32, dU, nf, eta, prec, maxiter, st);
    }
}

}  // namespace ovl
