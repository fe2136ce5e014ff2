// The overlap operator and the nested solver:
//   D[mu] = (1 + mu + (1 - mu) gamma_5 sign(K)) / 2          (paper Sec. 1, eq. 1)
//   relSUMR: Alg. 2 (basis recurrence of Alg. 1) for (1 + rho' U) x = b',
//            U = gamma_5 sign(K), rho' = (1 - mu)/(1 + mu), b' = 2 b/(1 + mu),
//            sign accuracy eta_j = min(floor, eps_A ||b'|| / ||r_j||)   (Sec. 3)
//   GMRESR:  Alg. 3 around relSUMR, outer vectors and residual in FP64.
//
// nf right-hand sides are solved together: every vector operation runs on all
// nf fields in one launch (per-field coefficients passed by value), and every
// sign-function call applies the multi-shift CG to all active fields at once,
// so one gauge-link read serves all of them.  Each right-hand side keeps its
// own scalar recurrences (on the host: a few complex numbers per iteration),
// its own accuracy and its own convergence; finished fields are masked out.
// The sign function's precision follows the strictest accuracy asked for
// among the active fields (Sec. 3: single precision once the accuracy is
// looser than a threshold; here also an FP16-storage level).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>

#include "context.h"
#include "fields.h"
#include "kernels.h"
#include "ops.h"

namespace ovl {

using zc = std::complex<double>;
static constexpr int MAXF = 16;

// out = a in + b gamma_5 s   (flat FP64 fields, n = 12 V complex each)
__global__ __launch_bounds__(256) void k_overlap_combine(const double2 *__restrict__ in,
                                                         const double2 *__restrict__ s, double2 *__restrict__ out,
                                                         double a, double b, int64_t V)
{
    const int f = blockIdx.y;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= 12 * V) return;
    const int64_t o = (int64_t)f * 12 * V + i;
    const double g = (i >= 6 * V) ? -b : b;   // planes 6..11 are spins 2, 3
    const double2 x = in[o], y = s[o];
    out[o] = make_double2(a * x.x + g * y.x, a * x.y + g * y.y);
}

static int prec_for(const ovl_solver_params &p, double eta)
{
    if (eta >= p.half_threshold) return OVL_HALF;
    if (eta >= p.f32_threshold) return OVL_F32;
    return OVL_F64;
}

static double min_active(const double *eta, int nf)
{
    double m = 1e300;
    for (int f = 0; f < nf; ++f)
        if (eta[f] > 0.0) m = std::min(m, eta[f]);
    return m;
}

// With the adaptive option: the fewest poles n <= z.n_z whose rational
// approximation error Delta(n) on [z.a, z.b] is at most eta / 4 (eta the
// strictest accuracy asked for); the multi-shift CG then gets eta - Delta(n)
// per field, so that the call's error stays within eta (Sec. 3: the error of
// the sign function is bounded by the larger of the approximation and the
// inversion errors).  Returns z itself when no smaller order qualifies.
static const ovl_zolo &zolo_for_accuracy(Context &c, const ovl_zolo &z, double eta_min)
{
    if (!c.adaptive_nz || !(eta_min < 1e300) || !(z.a > 0.0) || !(z.b > z.a)) return z;
    if (c.zolo_ab[0] != z.a || c.zolo_ab[1] != z.b) {
        c.zolo_by_n.clear();
        c.zolo_ab[0] = z.a;
        c.zolo_ab[1] = z.b;
    }
    for (int n = 2; n < z.n_z; ++n) {
        auto it = c.zolo_by_n.find(n);
        if (it == c.zolo_by_n.end()) {
            ovl_zolo zn{};
            zolotarev(n, z.a, z.b, zn);
            it = c.zolo_by_n.emplace(n, zn).first;
        }
        if (it->second.delta <= 0.25 * eta_min) return it->second;
    }
    return z;
}

// s = sign(K) in (FP64 packed in/out) with the multi-shift CG in precision
// prec.  Counters: with per_field, st has nf entries and field f's work goes
// to st[f]; otherwise st is one aggregate.  With lo non-null, a result in
// FP32 or FP16 storage is left where *lo points (its precision in *lo_prec)
// and s is not written; a result computed in FP64 is in s and *lo is null.
static void sign_f64(Context &c, double rho, const ovl_zolo &zin, const double2 *in, double2 *s, int nf,
                     const double *eta_in, int prec, int maxiter, ovl_stats *st, bool per_field,
                     const void **lo = nullptr, int *lo_prec = nullptr)
{
    if (lo) *lo = nullptr;
    const ovl_zolo &z = zolo_for_accuracy(c, zin, min_active(eta_in, nf));
    std::vector<double> eta_v(eta_in, eta_in + nf);
    if (&z != &zin)
        for (double &e : eta_v)
            if (e > 0.0) e -= z.delta;   // >= 3/4 of the accuracy asked for
    const double *eta = eta_v.data();
    ovl_stats *agg = per_field ? nullptr : st;
    // A multi-shift CG that breaks down in reduced precision (the curvature
    // (p, (K^2 + sigma) p) of a direction near the bottom of the spectrum is
    // below the storage rounding of K^2 p) is redone one precision up; the
    // accuracy asked for is unchanged.
    while (true) {
        try {
            if (prec == OVL_F64) {
                sign_mscg(c, rho, z, in, s, nf, eta, prec, maxiter, agg);
            } else {
                const size_t FB = field_bytes(c.g, prec) * nf;
                void *a = c.buf("u_lo_in", FB);
                void *b = c.buf("u_lo_out", FB);
                convert_spinor(c, in, OVL_F64, a, prec, nf);
                sign_mscg(c, rho, z, a, b, nf, eta, prec, maxiter, agg);
                if (lo) {
                    *lo = b;
                    *lo_prec = prec;
                } else {
                    convert_spinor(c, b, prec, s, OVL_F64, nf);
                }
            }
            break;
        } catch (const Error &e) {
            if (e.code != OVL_ERR_BREAKDOWN || prec == OVL_F64) throw;
            prec = prec == OVL_HALF ? OVL_F32 : OVL_F64;
            c.precision_retries += 1;
        }
    }
    if (per_field && st)
        for (int f = 0; f < nf; ++f)
            if (eta[f] > 0.0) {
                const int64_t it = f < (int)c.last_field_iters.size() ? c.last_field_iters[f] : 0;
                st[f].mscg_iters += it;
                st[f].dslash_calls[prec] += 2 * it + 1;
                st[f].sign_calls[prec] += 1;
            }
}

// u = gamma_5 s for a sign call's output s in FP32 or FP16 storage, widened to
// FP64, with each block's partial sums of (x, u) = sum conj(x) u: the
// widening, gamma_5 and the dot (q~, U q) that follows every application of
// U in Alg. 2, in one pass over the fields.
static constexpr int WD_BLOCKS = 512;   // blocks per field of the fused pass
template <typename ST>
__global__ __launch_bounds__(256) void k_widen_g5_dot(const ST *__restrict__ in, double2 *__restrict__ u,
                                                      const double2 *__restrict__ x, int64_t V, double *partial)
{
    const int f = blockIdx.y;
    const ST *inf = in + f * fstride<ST>(V);
    double re = 0.0, im = 0.0;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < V; s += (int64_t)gridDim.x * blockDim.x) {
        cplx<float> v[12];
        ld_sp(inf, V, s, v);
        const int64_t o = (int64_t)f * 12 * V + s;
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const double sg = c < 6 ? 1.0 : -1.0;   // gamma_5 = diag(1, 1, -1, -1) on the spins
            const double ur = sg * (double)v[c].re, ui = sg * (double)v[c].im;
            u[o + c * V] = make_double2(ur, ui);
            const double2 a = x[o + c * V];
            re += a.x * ur + a.y * ui;
            im += a.x * ui - a.y * ur;
        }
    }
    __shared__ double lds[4];
    const double tr = block_sum<256>(re, lds);
    const double ti = block_sum<256>(im, lds);
    if (threadIdx.x == 0) {
        partial[((int64_t)f * 2 + 0) * gridDim.x + blockIdx.x] = tr;
        partial[((int64_t)f * 2 + 1) * gridDim.x + blockIdx.x] = ti;
    }
}

// u = gamma_5 sign(K) q for the fields with eta[f] > 0.  The active fields
// are grouped by the precision their own accuracy calls for, and each group
// runs its own sign call (its own Zolotarev order with the adaptive option):
// a field whose middle solve has just restarted at a tight accuracy does not
// pull the others up to FP32 or FP64.
// With dx non-null, also (dx_f, u_f) for every field into *dot (an FP32 /
// FP16 result is widened, gamma_5 applied and the dot taken in one pass).
static void unitary_f64(Context &c, double rho, const ovl_zolo &z, const double2 *q, double2 *u, int nf,
                        const double *eta, const ovl_solver_params &prm, ovl_stats *st,
                        const double2 *dx = nullptr, std::vector<std::complex<double>> *dot = nullptr)
{
    int want[MAXF], present[3] = {0, 0, 0};
    for (int f = 0; f < nf; ++f) {
        want[f] = eta[f] > 0.0 ? prec_for(prm, eta[f]) : -1;
        if (want[f] >= 0) present[want[f]] += 1;
    }
    const int groups = (present[0] > 0) + (present[1] > 0) + (present[2] > 0);
    if (groups <= 1) {
        const void *lo = nullptr;
        int lp = OVL_F64;
        sign_f64(c, rho, z, q, u, nf, eta, prec_for(prm, min_active(eta, nf)), prm.max_mscg, st, true,
                 dx ? &lo : nullptr, &lp);
        if (lo) {
            const int64_t V = c.g.V;
            double *part = (double *)c.buf("u_wdot_part", sizeof(double) * WD_BLOCKS * 2 * nf);
            if (lp == OVL_F32)
                k_widen_g5_dot<float4><<<dim3(WD_BLOCKS, nf), 256, 0, c.stream>>>((const float4 *)lo, u, dx, V, part);
            else
                k_widen_g5_dot<h8><<<dim3(WD_BLOCKS, nf), 256, 0, c.stream>>>((const h8 *)lo, u, dx, V, part);
            OVL_HIP(hipGetLastError());
            const double *h = sum_partials_host(c, part, WD_BLOCKS, 2 * nf);
            dot->resize(nf);
            for (int f = 0; f < nf; ++f) (*dot)[f] = {h[2 * f], h[2 * f + 1]};
            return;
        }
    } else {
        // each group's call writes every field of its output (the others'
        // unspecified), so it goes to a scratch set and its own fields are copied out
        const size_t FB = field_bytes(c.g, OVL_F64);
        double2 *tmp = (double2 *)c.buf("u_group", FB * nf);
        for (int p = 0; p < 3; ++p) {
            if (!present[p]) continue;
            double eg[MAXF];
            for (int f = 0; f < nf; ++f) eg[f] = want[f] == p ? eta[f] : 0.0;
            sign_f64(c, rho, z, q, tmp, nf, eg, p, prm.max_mscg, st, true);
            for (int f = 0; f < nf; ++f)
                if (want[f] == p) copy_fields(c, tmp + (size_t)f * 12 * c.g.V, u + (size_t)f * 12 * c.g.V, 1, OVL_F64);
        }
    }
    gamma5_f64(c, u, nf);
    if (dx) {
        std::vector<cplx<double>> d;
        dot_f64(c, dx, u, nf, d);
        dot->resize(nf);
        for (int f = 0; f < nf; ++f) (*dot)[f] = {d[f].re, d[f].im};
    }
}

static void overlap_impl(Context &c, double rho, double mu, const ovl_zolo &z, const double2 *in, double2 *out,
                         int nf, const double *eta, int prec, int maxiter, ovl_stats *st, bool per_field)
{
    double2 *s = (double2 *)c.buf("ov_s", field_bytes(c.g, OVL_F64) * nf);
    sign_f64(c, rho, z, in, s, nf, eta, prec, maxiter, st, per_field);
    const int64_t V = c.g.V;
    k_overlap_combine<<<dim3((unsigned)((12 * V + 255) / 256), nf), 256, 0, c.stream>>>(
        in, s, out, 0.5 * (1.0 + mu), 0.5 * (1.0 - mu), V);
    OVL_HIP(hipGetLastError());
}

void overlap_f64(Context &c, double rho, double mu, const ovl_zolo &z, const double2 *in, double2 *out, int nf,
                 const double *eta, int prec, int maxiter, ovl_stats *st)
{
    overlap_impl(c, rho, mu, z, in, out, nf, eta, prec, maxiter, st, false);
}

void overlap_f64(Context &c, double rho, double mu, const ovl_zolo &z, const double2 *in, double2 *out, int nf,
                 double eta, int prec, int maxiter, ovl_stats *st)
{
    std::vector<double> e(nf, eta);
    overlap_impl(c, rho, mu, z, in, out, nf, e.data(), prec, maxiter, st, false);
}

// One fused SUMR vector step per field (the vector statements of Alg. 2, in order):
//   omega_old = omega; omega = alpha p + kappa (q_old - omega)
//   p = p + lambda (q_old - omega_old)
//   x = x + eta (q - omega)
//   q_old = q; q = (gamma q_t + u)/sigma; q_t = sigma q_t + conj(gamma) q
// and ||q_new||^2 per block.  Fields with act[f] = 0 are left untouched.
struct SumrCoef {
    double ar[MAXF], ai[MAXF], kr[MAXF], ki[MAXF], lr[MAXF], li[MAXF], er[MAXF], ei[MAXF], gr[MAXF], gi[MAXF],
        sigma[MAXF];
    int act[MAXF];
};

__global__ __launch_bounds__(256) void k_sumr_step(SumrCoef k, double2 *__restrict__ x, double2 *__restrict__ p,
                                                   double2 *__restrict__ om, double2 *__restrict__ qold,
                                                   double2 *__restrict__ q, double2 *__restrict__ qt,
                                                   const double2 *__restrict__ u, int64_t n, double *partial)
{
    const int f = blockIdx.y;
    double nn = 0.0;
    if (k.act[f]) {
        const cplx<double> alpha{k.ar[f], k.ai[f]}, kappa{k.kr[f], k.ki[f]}, lam{k.lr[f], k.li[f]},
            eta{k.er[f], k.ei[f]}, gam{k.gr[f], k.gi[f]};
        const double sg = k.sigma[f], is = 1.0 / sg;
        const int64_t o = (int64_t)f * n;
        for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
             i += (int64_t)gridDim.x * blockDim.x) {
            const int64_t j = o + i;
            const double2 pv = p[j], ov = om[j], qo = qold[j], qv = q[j], tv = qt[j], uv = u[j], xv = x[j];
            const cplx<double> P{pv.x, pv.y}, O{ov.x, ov.y}, QO{qo.x, qo.y}, Q{qv.x, qv.y}, T{tv.x, tv.y},
                U{uv.x, uv.y}, X{xv.x, xv.y};
            const cplx<double> On = alpha * P + kappa * (QO - O);
            const cplx<double> Pn = P + lam * (QO - O);
            const cplx<double> Xn = X + eta * (Q - On);
            const cplx<double> Qn = is * (gam * T + U);
            const cplx<double> Tn = sg * T + cmul_conj(gam, Qn);
            om[j] = make_double2(On.re, On.im);
            p[j] = make_double2(Pn.re, Pn.im);
            x[j] = make_double2(Xn.re, Xn.im);
            qold[j] = qv;
            q[j] = make_double2(Qn.re, Qn.im);
            qt[j] = make_double2(Tn.re, Tn.im);
            nn += Qn.re * Qn.re + Qn.im * Qn.im;
        }
    }
    __shared__ double lds[4];
    const double t = block_sum<256>(nn, lds);
    if (threadIdx.x == 0) partial[(int64_t)f * gridDim.x + blockIdx.x] = t;
}

static void norms(Context &c, const double2 *x, int nf, std::vector<double> &out)
{
    norm2_f64(c, x, nf, out);
    for (auto &v : out) v = std::isnan(v) ? v : std::sqrt(std::max(0.0, v));   // a NaN stays visible
}

static void dots(Context &c, const double2 *x, const double2 *y, int nf, std::vector<zc> &out)
{
    std::vector<cplx<double>> d;
    dot_f64(c, x, y, nf, d);
    out.resize(nf);
    for (int f = 0; f < nf; ++f) out[f] = zc(d[f].re, d[f].im);
}

// y_f = a_f x_f + b_f y_f over nf fields (a_f = 0, b_f = 1 leaves field f as is)
static void axpby(Context &c, const std::vector<zc> &a, const double2 *x, const std::vector<zc> &b, double2 *y,
                  int nf)
{
    std::vector<cplx<double>> ca(nf), cb(nf);
    for (int f = 0; f < nf; ++f) {
        ca[f] = {a[f].real(), a[f].imag()};
        cb[f] = {b[f].real(), b[f].imag()};
    }
    axpby_f64(c, ca.data(), x, cb.data(), y, nf);
}

struct SumrField {
    zc phi_hat, tau_hat, phi, s, lam, c_dag, cc;
    double r = 1.0, delta = 0.0, bn = 0.0, resid = 0.0;
    int iters = 0, restarts = 0;
    bool active = false, need_init = true;
};

// relSUMR for (1 + rho U) x_f = bp_f on the fields with mask[f], x holding x0
// (zero when x_zero).  Ax0 (nullable) holds (1 + rho U) x0 when the caller
// knows it (the deflated start supplies it from the stored D psi', Sec. 4),
// which saves a sign call.  collect: feed every active field's (q, U q) to
// eigSUMR (Alg. 5; several fields only in block collection) and use the
// stricter of the inversion and eigenvector sign accuracies (Sec. 5.1).
static void sumr(Context &c, const ovl_zolo &z, const ovl_solver_params &prm, double rhoK, double rho,
                 const double2 *bp, double2 *x, int nf, const std::vector<int> &mask, bool x_zero,
                 const double2 *Ax0, double tol, double epsA, bool collect, ovl_stats *st)
{
    const size_t FB = field_bytes(c.g, OVL_F64);
    double2 *rt = (double2 *)c.buf("s_rt", FB * nf);
    double2 *p = (double2 *)c.buf("s_p", FB * nf);
    double2 *om = (double2 *)c.buf("s_om", FB * nf);
    double2 *q = (double2 *)c.buf("s_q", FB * nf);
    double2 *qold = (double2 *)c.buf("s_qold", FB * nf);
    double2 *qt = (double2 *)c.buf("s_qt", FB * nf);
    double2 *u = (double2 *)c.buf("s_u", FB * nf);
    const int64_t n = 12 * c.g.V;
    const int nblk = 256;
    double *part = (double *)c.buf("s_part", sizeof(double) * nblk * nf);
    const double zeta = 1.0;

    std::vector<SumrField> F(nf);
    std::vector<double> bn;
    norms(c, bp, nf, bn);
    for (int f = 0; f < nf; ++f) {
        F[f].bn = bn[f];
        F[f].active = mask[f] != 0 && bn[f] > 0.0;
        F[f].resid = bn[f];
    }
    bool first = true;
    auto eta_for = [&](const SumrField &sf) {
        double e = std::fmin(prm.relax_floor, epsA * sf.bn / sf.resid);
        if (collect) e = std::fmin(e, eig_sign_accuracy(c));
        return e;
    };
    std::vector<double> eta(nf, 0.0);
    while (true) {
        // (re)initialise the fields that need it: r~ = b - (1 + rho U) x
        bool any_init = false;
        std::vector<int> init(nf, 0);
        for (int f = 0; f < nf; ++f) {
            init[f] = F[f].active && F[f].need_init;
            any_init = any_init || init[f];
        }
        if (any_init) {
            std::vector<zc> ca(nf, 0.0), cb(nf, 1.0);
            for (int f = 0; f < nf; ++f)
                if (init[f]) {
                    ca[f] = 1.0;
                    cb[f] = 0.0;
                }
            axpby(c, ca, bp, cb, rt, nf);   // rt = bp on the (re)starting fields
            const bool need_ux = !(first && x_zero) && !(first && Ax0 != nullptr);
            if (first && !x_zero && Ax0 != nullptr) {
                std::vector<zc> a2(nf, 0.0), b2(nf, 1.0);
                for (int f = 0; f < nf; ++f)
                    if (init[f]) a2[f] = -1.0;
                axpby(c, a2, Ax0, b2, rt, nf);
            } else if (need_ux) {
                for (int f = 0; f < nf; ++f) eta[f] = init[f] ? eta_for(F[f]) : 0.0;
                unitary_f64(c, rhoK, z, x, u, nf, eta.data(), prm, st);
                std::vector<zc> a1(nf, 0.0), a2(nf, 0.0), b1(nf, 1.0);
                for (int f = 0; f < nf; ++f)
                    if (init[f]) {
                        a1[f] = -1.0;
                        a2[f] = -rho;
                    }
                axpby(c, a1, x, b1, rt, nf);
                axpby(c, a2, u, b1, rt, nf);
            }
            std::vector<double> dl;
            norms(c, rt, nf, dl);
            std::vector<zc> qa(nf, 0.0), qb(nf, 1.0), zz(nf, 0.0), z1(nf, 1.0), a0(nf, 0.0);
            for (int f = 0; f < nf; ++f) {
                SumrField &sf = F[f];
                if (!init[f]) continue;
                if (!std::isfinite(dl[f])) throw Error{OVL_ERR_BREAKDOWN, "SUMR: non-finite residual"};
                sf.delta = dl[f];
                sf.resid = dl[f];
                sf.need_init = false;
                if (dl[f] <= tol * sf.bn) {
                    sf.active = false;
                    continue;
                }
                sf.phi_hat = 1.0 / sf.delta;
                sf.tau_hat = sf.delta / rho;
                sf.phi = 0.0;
                sf.s = 0.0;
                sf.lam = 0.0;
                sf.c_dag = 1.0;
                sf.cc = 1.0;
                sf.r = 1.0;
                qa[f] = 1.0 / sf.delta;
                qb[f] = 0.0;
                a0[f] = 1.0;
                z1[f] = 0.0;
            }
            axpby(c, qa, rt, qb, q, nf);      // q = r~/delta on the (re)started fields
            axpby(c, a0, q, z1, qt, nf);      // q_t = q
            axpby(c, zz, rt, z1, om, nf);     // omega = 0  (0 times the finite r~)
            axpby(c, zz, rt, z1, p, nf);      // p = 0
            axpby(c, zz, rt, z1, qold, nf);   // q_old = 0
        }
        first = false;
        // residual estimates and the active set
        int nact = 0;
        for (int f = 0; f < nf; ++f) {
            SumrField &sf = F[f];
            if (!sf.active) continue;
            sf.resid = rho * std::abs(sf.tau_hat);
            if (sf.resid <= tol * sf.bn || sf.iters >= prm.max_middle || sf.restarts > 50) sf.active = false;
            nact += sf.active;
        }
        if (nact == 0) break;
        for (int f = 0; f < nf; ++f) eta[f] = F[f].active ? eta_for(F[f]) : 0.0;
        std::vector<zc> g;   // (q~, U q), taken with U q
        unitary_f64(c, rhoK, z, q, u, nf, eta.data(), prm, st, qt, &g);
        if (collect)   // Alg. 5: every active field's (q, U q); one field unless collecting as a block
            for (int f = 0; f < nf; ++f)
                if (F[f].active) eig_collect(c, q + (size_t)f * n, u + (size_t)f * n);
        SumrCoef k{};
        for (int f = 0; f < nf; ++f) {
            SumrField &sf = F[f];
            k.act[f] = 0;
            if (!sf.active) continue;
            zc gamma = g[f];
            if (!(std::abs(gamma) < 1.0)) {   // |gamma| >= 1: restart (Sec. 2)
                sf.need_init = true;
                sf.restarts += 1;
                if (st) st[f].restarts += 1;
                continue;
            }
            const double r_pp = sf.r;
            const double sigma = std::sqrt(1.0 - std::norm(gamma));
            const zc alpha = gamma * sf.delta;
            gamma = -gamma;
            const zc r_p = alpha * sf.phi + sf.s * zeta / rho;
            const zc r_hat = alpha * sf.phi_hat + sf.c_dag * zeta / rho;
            const double nrm = std::sqrt(std::norm(r_hat) + sigma * sigma);
            sf.c_dag = r_hat / nrm;
            sf.cc = std::conj(sf.c_dag);
            sf.s = -sigma / nrm;
            const zc rn = sf.s * sigma - sf.cc * r_hat;
            const zc tau = -sf.cc * sf.tau_hat;
            sf.tau_hat = sf.s * sf.tau_hat;
            const zc et = tau / rn;
            const zc kappa = r_p / r_pp;
            k.ar[f] = alpha.real();
            k.ai[f] = alpha.imag();
            k.kr[f] = kappa.real();
            k.ki[f] = kappa.imag();
            k.lr[f] = sf.lam.real();   // lambda of the previous iteration
            k.li[f] = sf.lam.imag();
            k.er[f] = et.real();
            k.ei[f] = et.imag();
            k.gr[f] = gamma.real();
            k.gi[f] = gamma.imag();
            k.sigma[f] = sigma;
            k.act[f] = 1;
            sf.delta = sigma * sf.delta;
            sf.phi = sf.s * std::conj(gamma) / sf.delta - sf.cc * sf.phi_hat;
            sf.r = rn.real();   // real for this recurrence
            sf.lam = sf.phi / rn;
            sf.phi_hat = sf.s * sf.phi_hat + sf.c_dag * std::conj(gamma) / sf.delta;
            sf.iters += 1;
            if (st) st[f].sumr_iters += 1;
        }
        k_sumr_step<<<dim3(nblk, nf), 256, 0, c.stream>>>(k, x, p, om, qold, q, qt, u, n, part);
        OVL_HIP(hipGetLastError());
        // ||q|| monitoring (Sec. 2)
        const double *hq = sum_partials_host(c, part, nblk, nf);
        const std::vector<double> qn2(hq, hq + nf);
        for (int f = 0; f < nf; ++f) {
            if (!k.act[f]) continue;
            if (!std::isfinite(qn2[f])) throw Error{OVL_ERR_BREAKDOWN, "SUMR: non-finite basis vector"};
            if (std::fabs(std::sqrt(qn2[f]) - 1.0) > prm.norm_restart) {
                F[f].need_init = true;
                F[f].restarts += 1;
                if (st) st[f].restarts += 1;
            }
        }
    }
}

// h_f = H w_f = gamma_5 D[mu] w_f for the fields with eta[f] > 0 (sign
// accuracy eta[f], precision from the ladder, FP32 at most: CG works on
// H^2 = D^+ D, whose lowest eigenvalues (about mu^2, 4e-4 at mu = 0.02) are
// below the uncorrelated rounding of FP16 storage (~5e-4 of a site's largest
// component), and the CG then diverges -- seen on the 16^3 x 32 workload;
// SUMR works on D itself, whose singular values are >= mu).
static void apply_H(Context &c, const ovl_zolo &z, const ovl_solver_params &prm, const double2 *w, double2 *h,
                    int nf, const double *eta, ovl_stats *st)
{
    int prec = prec_for(prm, min_active(eta, nf));
    if (prec == OVL_HALF) prec = OVL_F32;
    overlap_impl(c, prm.rho, prm.mu, z, w, h, nf, eta, prec, prm.max_mscg, st, true);
    gamma5_f64(c, h, nf);
}

// relCG: the preconditioned CGNE of Sec. 4 for H x_f = b_f (H = gamma_5 D[mu]
// Hermitian) on the fields with mask[f]:
//   r = p = Hhat^{-1} b, x = 0;
//   z = Hhat^{-1} H^2 Hhat^{-1} p, alpha = (r, r) / (r, z), r -= alpha z,
//   x += alpha p, beta = (r', r') / (r, r), p = r' + beta p, until
//   ||r|| < tol ||b||; then x = H Hhat^{-1} x.
// Each H is applied with the CG relaxation of Sec. 3,
// eta_j = min(floor, epsA ||r_0|| sqrt(sum_{i<=j} ||r_i||^-2)); the closing H
// with accuracy epsA.  Hhat^{-1} is the identity unless precond.
// collect (eigCG, Sec. 5; one field only): every iteration hands w = Hhat^{-1} p,
// H w and H H w to the eigenspace, and the Sec. 5.1 bound caps eta_j.  The
// preconditioner stays the one built when the CG starts, even where the
// collection diagonalises the eigenspace meanwhile (CG needs a fixed operator).
static void cgne(Context &c, const ovl_zolo &z, const ovl_solver_params &prm, const double2 *b, double2 *x, int nf,
                 const std::vector<int> &mask, double tol, double epsA, bool precond, bool collect, ovl_stats *st)
{
    const size_t FB = field_bytes(c.g, OVL_F64);
    double2 *r = (double2 *)c.buf("cg_r", FB * nf);
    double2 *p = (double2 *)c.buf("cg_p", FB * nf);
    double2 *xj = (double2 *)c.buf("cg_x", FB * nf);
    double2 *w = (double2 *)c.buf("cg_w", FB * nf);
    double2 *t = (double2 *)c.buf("cg_t", FB * nf);
    double2 *hh = collect ? (double2 *)c.buf("cg_hh", FB * nf) : w;
    struct Hold {
        EigSpace &e;
        ~Hold() { e.spec_hold = false; }
    } hold{c.eig};
    auto P = [&](const double2 *in, double2 *out) {
        if (precond)
            spectral_apply(c, in, out, nf);
        else if (out != in)
            copy_fields(c, in, out, nf, OVL_F64);
    };
    std::vector<double> bn, rr(nf, 0.0), r0n(nf, 0.0), zeta(nf, 0.0);
    norms(c, b, nf, bn);
    P(b, r);
    if (precond) c.eig.spec_hold = true;
    copy_fields(c, r, p, nf, OVL_F64);
    zero_fields(c, xj, nf, OVL_F64);
    std::vector<int> act(nf, 0), its(nf, 0);
    {
        std::vector<double> n0;
        norms(c, r, nf, n0);
        for (int f = 0; f < nf; ++f) {
            rr[f] = n0[f] * n0[f];
            r0n[f] = n0[f];
            zeta[f] = rr[f] > 0.0 ? 1.0 / rr[f] : 0.0;
            act[f] = mask[f] != 0 && bn[f] > 0.0;
        }
    }
    std::vector<double> eta(nf, 0.0);
    int loops = 0;
    while (true) {
        int nact = 0;
        for (int f = 0; f < nf; ++f) {
            if (act[f] && (std::sqrt(rr[f]) < tol * bn[f] || its[f] >= prm.max_middle)) act[f] = 0;
            nact += act[f];
        }
        if (nact == 0) break;
        const double cap = collect ? eig_sign_accuracy(c) : 1.0;
        for (int f = 0; f < nf; ++f)
            eta[f] = act[f] ? std::fmin(cap, std::fmin(prm.relax_floor, epsA * r0n[f] * std::sqrt(zeta[f]))) : 0.0;
        P(p, w);
        apply_H(c, z, prm, w, t, nf, eta.data(), st);
        apply_H(c, z, prm, t, hh, nf, eta.data(), st);
        if (collect) eig_collect_cg(c, w, t, hh);
        P(hh, t);   // t = Hhat^{-1} H^2 Hhat^{-1} p
        std::vector<zc> rz;
        dots(c, r, t, nf, rz);
        std::vector<zc> ma(nf, 0.0), pa(nf, 0.0), one(nf, 1.0);
        for (int f = 0; f < nf; ++f)
            if (act[f]) {
                if (!(std::abs(rz[f]) > 0.0) || !std::isfinite(std::abs(rz[f])))
                    throw Error{OVL_ERR_BREAKDOWN, "CG: (r, z) zero or non-finite"};
                const zc alpha = rr[f] / rz[f];
                ma[f] = -alpha;
                pa[f] = alpha;
            }
        axpby(c, ma, t, one, r, nf);
        axpby(c, pa, p, one, xj, nf);
        std::vector<double> rn;
        norms(c, r, nf, rn);
        std::vector<zc> a1(nf, 0.0), bb(nf, 1.0);
        for (int f = 0; f < nf; ++f)
            if (act[f]) {
                const double rr_new = rn[f] * rn[f];
                if (!std::isfinite(rr_new)) throw Error{OVL_ERR_BREAKDOWN, "CG: non-finite residual"};
                a1[f] = 1.0;
                bb[f] = rr_new / rr[f];
                rr[f] = rr_new;
                zeta[f] += rr_new > 0.0 ? 1.0 / rr_new : 0.0;
                its[f] += 1;
                if (st) st[f].sumr_iters += 1;
            }
        axpby(c, a1, r, bb, p, nf);   // p = r + beta p
        if (prm.verbose && ++loops % 20 == 0) {
            double worst = 0.0;
            for (int f = 0; f < nf; ++f)
                if (act[f]) worst = std::max(worst, std::sqrt(rr[f]) / bn[f]);
            std::fprintf(stderr, "[ovl] CG iteration %d: %d fields active, largest ||r||/||b|| = %.3e\n", loops, nact,
                         worst);
        }
    }
    // x = H Hhat^{-1} x_j
    P(xj, w);
    for (int f = 0; f < nf; ++f) eta[f] = mask[f] && bn[f] > 0.0 ? epsA : 0.0;
    apply_H(c, z, prm, w, t, nf, eta.data(), st);
    std::vector<zc> a(nf, 0.0), b0(nf, 1.0);
    for (int f = 0; f < nf; ++f)
        if (mask[f] && bn[f] > 0.0) {
            a[f] = 1.0;
            b0[f] = 0.0;
        }
    axpby(c, a, t, b0, x, nf);
}

ovl_status solve_batch(Context &c, const ovl_zolo &z, const ovl_solver_params &prm, const double2 *b, double2 *x,
                       int nf, ovl_stats *st)
{
    OVL_REQUIRE(nf >= 1 && nf <= MAXF, OVL_ERR_ARG, "too many right-hand sides in one batch");
    OVL_REQUIRE(!(prm.eig_calc && nf > 1 && !prm.eig_block), OVL_ERR_ARG,
                "without eig_block, eigSUMR collects from one right-hand side at a time");
    const auto t0 = std::chrono::steady_clock::now();
    const double mu = prm.mu;
    const double rhoK = prm.rho;
    const double rho = (1.0 - mu) / (1.0 + mu);
    const size_t FB = field_bytes(c.g, OVL_F64);
    const int64_t fs = 12 * c.g.V;   // double2 per field
    const int maxo = prm.max_outer;
    double2 *r = (double2 *)c.buf("g_r", FB * nf);
    double2 *uu = (double2 *)c.buf("g_u", FB * nf);
    double2 *cv = (double2 *)c.buf("g_c", FB * nf);
    double2 *bp = (double2 *)c.buf("g_bp", FB * nf);

    zero_fields(c, x, nf, OVL_F64);
    copy_fields(c, b, r, nf, OVL_F64);
    if (prm.eig_calc) {
        eig_configure(c, prm.n_eig, prm.m_eig, mu, prm.delta_split, prm.eig_eps, prm.k_recalc);
        c.eig.canonical = prm.eig_block != 0;
    }
    std::vector<double> bn, rn;
    norms(c, b, nf, bn);
    for (int f = 0; f < nf; ++f)
        OVL_REQUIRE(std::isfinite(bn[f]), OVL_ERR_BREAKDOWN,
                    "right-hand side " + std::to_string(f) + " has a non-finite entry");
    rn = bn;
    std::vector<int> steps(nf, 0), active(nf, 0);
    ovl_status status = OVL_OK;
    std::vector<double2 *> C, Uv;
    while (true) {
        int nact = 0;
        for (int f = 0; f < nf; ++f) {
            const bool want = bn[f] > 0.0 && rn[f] > 0.5 * prm.tol * bn[f];
            active[f] = want && steps[f] < maxo;
            if (want && steps[f] >= maxo) status = OVL_ERR_NOT_CONVERGED;
            nact += active[f];
        }
        if (nact == 0) break;
        const int i = *std::max_element(steps.begin(), steps.end());   // same for every active field
        if ((int)C.size() <= i) {
            C.push_back((double2 *)c.buf("g_C" + std::to_string(i), FB * nf));
            Uv.push_back((double2 *)c.buf("g_U" + std::to_string(i), FB * nf));
        }
        if (prm.middle_cg) {
            // middle solve D u = r with relCG: H u = gamma_5 r (Sec. 4)
            copy_fields(c, r, bp, nf, OVL_F64);
            gamma5_f64(c, bp, nf);
            const bool pre = prm.use_deflation && spectral_available(c);
            const bool collect = prm.eig_calc != 0;
            zero_fields(c, uu, nf, OVL_F64);
            cgne(c, z, prm, bp, uu, nf, active, prm.eta_tilde, prm.eta_tilde, pre, collect, st);
            if (collect) {
                eig_diagonalise(c);   // Alg. 6 closes each calculating middle solve
                if (c.eig.ndiag > 0 && prm.k_recalc > 0 && c.eig.ndiag % prm.k_recalc == 0)
                    eig_recompute(c, rhoK, z, 1e-12, nullptr);
            }
        } else {
        // middle solve D u = r to relative accuracy eta_tilde: (1 + rho U) u = 2 r/(1 + mu)
        {
            std::vector<zc> a(nf, 2.0 / (1.0 + mu)), b0(nf, 0.0);
            axpby(c, a, r, b0, bp, nf);
        }
        zero_fields(c, uu, nf, OVL_F64);
        // deflated start (Sec. 4): u0 from the eigenspace, (1 + rho U) u0 = 2 D u0/(1 + mu)
        const bool defl = prm.use_deflation && c.eig.n > 0 && c.eig.k >= c.eig.n && c.eig.ndiag > 0;
        double2 *Ax0 = nullptr;
        if (defl) {
            Ax0 = (double2 *)c.buf("g_Ax0", FB * nf);
            double2 *Dx0 = (double2 *)c.buf("g_Dx0", FB * nf);
            zero_fields(c, Dx0, nf, OVL_F64);
            for (int f = 0; f < nf; ++f)
                if (active[f]) eig_project(c, r + f * fs, uu + f * fs, Dx0 + f * fs);
            std::vector<zc> a(nf, 2.0 / (1.0 + mu)), b0(nf, 0.0);
            axpby(c, a, Dx0, b0, Ax0, nf);
        }
        const bool collect = prm.eig_calc != 0;
        sumr(c, z, prm, rhoK, rho, bp, uu, nf, active, !defl, Ax0, prm.eta_tilde, prm.eta_tilde, collect, st);
        if (collect) {
            eig_diagonalise(c);   // the closing Alg. 6 of Alg. 5
            if (c.eig.ndiag > 0 && prm.k_recalc > 0 && c.eig.ndiag % prm.k_recalc == 0)
                eig_recompute(c, rhoK, z, 1e-12, nullptr);
        }
        }
        // c = D u, to ||D u - c|| <= eps ||b|| / 4, or with the option to the
        // accuracy Alg. 3 prints, ||D u - c|| < eps ||b|| ||u|| / ||r||.  Since
        // D u - c = (1 - mu)/2 gamma_5 (sign(K) u - s) for a sign approximation
        // s to relative accuracy eta, these are eta = eps ||b|| / (2 (1 - mu) ||u||)
        // and eta = 2 eps ||b|| / ((1 - mu) ||r||).
        std::vector<double> un;
        if (!c.outer_printed) norms(c, uu, nf, un);
        std::vector<double> eta_c(nf, 0.0);
        for (int f = 0; f < nf; ++f)
            if (active[f])
                eta_c[f] = std::fmin(1e-2, c.outer_printed
                                               ? 2.0 * prm.tol * bn[f] / ((1.0 - mu) * std::max(rn[f], 1e-300))
                                               : prm.tol * bn[f] / (2.0 * (1.0 - mu) * std::max(un[f], 1e-300)));
        overlap_impl(c, rhoK, mu, z, uu, cv, nf, eta_c.data(), prec_for(prm, min_active(eta_c.data(), nf)),
                     prm.max_mscg, st, true);
        // modified Gram-Schmidt against C[0..i)
        for (int j = 0; j < i; ++j) {
            std::vector<zc> beta;
            dots(c, C[j], cv, nf, beta);
            std::vector<zc> mb(nf, 0.0), one(nf, 1.0);
            for (int f = 0; f < nf; ++f)
                if (active[f]) mb[f] = -beta[f];
            axpby(c, mb, C[j], one, cv, nf);
            axpby(c, mb, Uv[j], one, uu, nf);
        }
        std::vector<double> cn;
        norms(c, cv, nf, cn);
        std::vector<zc> inv(nf, 0.0), keep(nf, 1.0);
        for (int f = 0; f < nf; ++f)
            if (active[f]) {
                if (!(cn[f] > 0.0) || !std::isfinite(cn[f]))
                    throw Error{OVL_ERR_BREAKDOWN, "GMRESR: zero or non-finite c"};
                inv[f] = 1.0 / cn[f];
                keep[f] = 0.0;
            }
        axpby(c, inv, cv, keep, C[i], nf);
        axpby(c, inv, uu, keep, Uv[i], nf);
        std::vector<zc> alpha;
        dots(c, C[i], r, nf, alpha);
        std::vector<zc> pa(nf, 0.0), ma(nf, 0.0), one(nf, 1.0);
        for (int f = 0; f < nf; ++f)
            if (active[f]) {
                pa[f] = alpha[f];
                ma[f] = -alpha[f];
            }
        axpby(c, pa, Uv[i], one, x, nf);
        axpby(c, ma, C[i], one, r, nf);
        std::vector<double> rnew;
        norms(c, r, nf, rnew);
        for (int f = 0; f < nf; ++f)
            if (active[f]) {
                rn[f] = rnew[f];
                steps[f] += 1;
                if (st) st[f].gmresr_steps += 1;
            }
        if (prm.verbose)
            std::fprintf(stderr, "[ovl] GMRESR step %d: ||r||/||b|| of field 0 = %.3e (sign calls redone one precision up so far: %lld)\n",
                         i + 1, rn[0] / bn[0], (long long)c.precision_retries);
    }
    // a calculating solve ends a Krylov space: the three-set re-diagonalisation (Sec. 5)
    if (prm.eig_calc && c.eig.ndiag > 0 && c.eig.k >= c.eig.n) eig_rediagonalise_sets(c);
    OVL_HIP(hipStreamSynchronize(c.stream));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (st)
        for (int f = 0; f < nf; ++f) {
            st[f].computed_relres = bn[f] > 0.0 ? rn[f] / bn[f] : 0.0;
            st[f].seconds += secs;
        }
    return status;
}

// The standalone eigSUMR eigensolver (Sec. 6, eigenvector calculation).
// Each run generates the Alg. 1 basis of U = gamma_5 sign(K) from its start
// vector and feeds every (q, U q) to Alg. 5; it ends after diag_per_run
// diagonalisations, when | ||q|| - 1 | > norm_restart or |gamma| >= 1, or when
// every held eigenvector's residual is at most the run's target.  Alg. 6
// closes the run, v^D is recomputed to 1e-12, and the three-set
// re-diagonalisation follows.  Sign accuracy: the Sec. 5.1 bound, never
// looser than relax_floor (eta_fixed <= 0), or eta_fixed.  The next run starts from the last q, orthogonalised
// twice against the eigenvectors and normalised, with the target
// max(eig_eps, 0.1 x the largest residual).  Stops when every residual is
// at most eig_eps (OVL_OK) or after max_runs runs (OVL_ERR_NOT_CONVERGED);
// OVL_ERR_BREAKDOWN if a run ends before any diagonalisation has happened.
// Collection continues from what the eigenspace holds when its n, m and mu
// are unchanged (eig_configure), else starts from an empty space.
ovl_status eig_eigensolve(Context &c, const ovl_zolo &z, const ovl_solver_params &prm, const double2 *q0,
                          int max_runs, int diag_per_run, double eta_fixed, int *runs_out, int64_t *applies_hist,
                          double *maxres_hist, ovl_stats *st)
{
    OVL_REQUIRE(max_runs >= 1 && diag_per_run >= 1, OVL_ERR_ARG, "eigensolver: bad run limits");
    OVL_REQUIRE(prm.n_eig >= 1 && 3 * prm.n_eig <= 512, OVL_ERR_ARG,
                "eigensolver: n_eig must be at most 170 (three sets of n are diagonalised together)");
    const auto t0 = std::chrono::steady_clock::now();
    eig_configure(c, prm.n_eig, prm.m_eig, prm.mu, prm.delta_split, prm.eig_eps, prm.k_recalc);
    EigSpace &e = c.eig;
    const int n = e.n;
    e.nsets = 0;
    const double eps_final = prm.eig_eps;
    struct EpsRestore {
        EigSpace &e;
        double v;
        ~EpsRestore() { e.eps = v; }
    } restore{e, eps_final};
    const size_t FB = field_bytes(c.g, OVL_F64);
    double2 *q = (double2 *)c.buf("es_q", FB);
    double2 *qt = (double2 *)c.buf("es_qt", FB);
    double2 *u = (double2 *)c.buf("es_u", FB);
    std::vector<double> nn;
    norms(c, q0, 1, nn);
    OVL_REQUIRE(nn[0] > 0.0 && std::isfinite(nn[0]), OVL_ERR_ARG, "eigensolver: zero or non-finite start vector");
    lincomb3_f64(c, 1.0 / nn[0], q0, 0.0, q0, 0.0, nullptr, q, 1);
    int64_t applies = 0;
    ovl_status status = OVL_ERR_NOT_CONVERGED;
    int runs = 0;
    for (int run = 0; run < max_runs; ++run) {
        copy_fields(c, q, qt, 1, OVL_F64);
        const int nd0 = e.ndiag;
        while (e.ndiag - nd0 < diag_per_run) {
            double eta = eta_fixed > 0.0 ? eta_fixed : std::fmin(prm.relax_floor, eig_sign_accuracy(c));
            unitary_f64(c, prm.rho, z, q, u, 1, &eta, prm, st);
            applies += 1;
            eig_collect(c, q, u);
            std::vector<zc> g;
            dots(c, qt, u, 1, g);
            zc gamma = g[0];
            if (!(std::abs(gamma) < 1.0)) break;
            const double sigma = std::sqrt(1.0 - std::norm(gamma));
            gamma = -gamma;
            // Alg. 1: q = (gamma q~ + U q) / sigma, q~ = sigma q~ + conj(gamma) q
            axpby(c, {gamma / sigma}, qt, {0.0}, q, 1);
            axpby(c, {1.0 / sigma}, u, {1.0}, q, 1);
            axpby(c, {std::conj(gamma)}, q, {sigma}, qt, 1);
            std::vector<double> qn;
            norms(c, q, 1, qn);
            if (!std::isfinite(qn[0])) throw Error{OVL_ERR_BREAKDOWN, "eigensolver: non-finite basis vector"};
            if (std::fabs(qn[0] - 1.0) > prm.norm_restart) break;
            if (!e.resid.empty() && *std::max_element(e.resid.begin(), e.resid.end()) <= e.eps) break;
        }
        eig_diagonalise(c);
        OVL_REQUIRE(e.ndiag > 0 && e.k >= n, OVL_ERR_BREAKDOWN,
                    "eigensolver: a run ended before the first diagonalisation (fewer than n_eig + 1 basis "
                    "vectors before the norm test); lower n_eig");
        eig_recompute(c, prm.rho, z, 1e-12, st);
        eig_rediagonalise_sets(c);
        runs = run + 1;
        const double mr = *std::max_element(e.resid.begin(), e.resid.end());
        if (applies_hist) applies_hist[run] = applies;
        if (maxres_hist) maxres_hist[run] = mr;
        if (prm.verbose)
            std::fprintf(stderr, "[ovl] eigensolver run %d: %lld applications of U, largest residual %.3e\n", run + 1,
                         (long long)applies, mr);
        if (mr <= eps_final) {
            status = OVL_OK;
            break;
        }
        e.eps = std::max(eps_final, 0.1 * mr);
        for (int pass = 0; pass < 2; ++pass) {   // q -= V (V^H q)
            std::vector<cplx<double>> a;
            gram_f64(c, e.V, n, q, 1, false, a);
            for (auto &x : a) x = {-x.re, -x.im};
            rotate_f64(c, e.V, n, a, 1, q, 1.0);
        }
        norms(c, q, 1, nn);
        OVL_REQUIRE(nn[0] > 0.0 && std::isfinite(nn[0]), OVL_ERR_BREAKDOWN,
                    "eigensolver: the restart vector lies in the eigenspace");
        lincomb3_f64(c, 1.0 / nn[0], q, 0.0, q, 0.0, nullptr, u, 1);
        copy_fields(c, u, q, 1, OVL_F64);
    }
    OVL_HIP(hipStreamSynchronize(c.stream));
    if (runs_out) *runs_out = runs;
    if (st) st->sumr_iters += applies;
    if (st) st->seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return status;
}

}  // namespace ovl
