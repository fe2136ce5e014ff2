// The overlap operator and the nested solver:
//   D[mu] = (1 + mu + (1 - mu) gamma_5 sign(K)) / 2          (paper Sec. 1, eq. 1)
//   relSUMR: Alg. 2 (basis recurrence of Alg. 1) for (1 + rho' U) x = b',
//            U = gamma_5 sign(K), rho' = (1 - mu)/(1 + mu), b' = 2 b/(1 + mu),
//            sign accuracy eta_j = min(floor, eps_A ||b'|| / ||r_j||)   (Sec. 3)
//   GMRESR:  Alg. 3 around relSUMR, outer vectors and residual in FP64.
// The SUMR and GMRESR vectors are packed FP64 fields on the device; their
// scalar recurrences (a few complex numbers per iteration) run on the host,
// which reads back one inner product and one norm per SUMR iteration.  The
// sign function's precision follows its requested accuracy (Sec. 3: single
// precision once the accuracy asked for is looser than a threshold).
#include <chrono>
#include <cmath>
#include <complex>

#include "context.h"
#include "fields.h"
#include "kernels.h"
#include "ops.h"

namespace ovl {

using zc = std::complex<double>;

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

// u = gamma_5 sign(K) q (FP64 packed in/out), sign in precision prec.
static void unitary_f64(Context &c, double rho, const ovl_zolo &z, const double2 *q, double2 *u, int nf,
                        double eta, int prec, int maxiter, ovl_stats *st)
{
    if (prec == OVL_F64) {
        sign_mscg(c, rho, z, q, u, nf, eta, prec, maxiter, st);
    } else {
        const size_t FB = field_bytes(c.g, prec) * nf;
        void *a = c.buf("u_lo_in", FB);
        void *b = c.buf("u_lo_out", FB);
        convert_spinor(c, q, OVL_F64, a, prec, nf);
        sign_mscg(c, rho, z, a, b, nf, eta, prec, maxiter, st);
        convert_spinor(c, b, prec, u, OVL_F64, nf);
    }
    gamma5_f64(c, u, nf);
}

void overlap_f64(Context &c, double rho, double mu, const ovl_zolo &z, const double2 *in, double2 *out,
                 int nf, double eta, int prec, int maxiter, ovl_stats *st)
{
    double2 *s = (double2 *)c.buf("ov_s", field_bytes(c.g, OVL_F64) * nf);
    if (prec == OVL_F64) {
        sign_mscg(c, rho, z, in, s, nf, eta, prec, maxiter, st);
    } else {
        const size_t FB = field_bytes(c.g, prec) * nf;
        void *a = c.buf("u_lo_in", FB);
        void *b = c.buf("u_lo_out", FB);
        convert_spinor(c, in, OVL_F64, a, prec, nf);
        sign_mscg(c, rho, z, a, b, nf, eta, prec, maxiter, st);
        convert_spinor(c, b, prec, s, OVL_F64, nf);
    }
    const int64_t V = c.g.V;
    k_overlap_combine<<<dim3((unsigned)((12 * V + 255) / 256), nf), 256, 0, c.stream>>>(
        in, s, out, 0.5 * (1.0 + mu), 0.5 * (1.0 - mu), V);
    OVL_HIP(hipGetLastError());
}

// One fused SUMR vector step (the vector statements of Alg. 2, in order):
//   omega_old = omega; omega = alpha p + kappa (q_old - omega)
//   p = p + lambda (q_old - omega_old)
//   x = x + eta (q - omega)
//   q_old = q; q = (gamma q_t + u)/sigma; q_t = sigma q_t + conj(gamma) q
// q_new is written over the q_old buffer (the caller swaps the two), and a
// partial ||q_new||^2 is produced.
struct SumrCoef {
    double ar, ai, kr, ki, lr, li, er, ei, gr, gi, sigma;
};

__global__ __launch_bounds__(256) void k_sumr_step(SumrCoef k, double2 *__restrict__ x, double2 *__restrict__ p,
                                                   double2 *__restrict__ om, double2 *__restrict__ qold_qnew,
                                                   const double2 *__restrict__ q, double2 *__restrict__ qt,
                                                   const double2 *__restrict__ u, int64_t n, double *partial)
{
    double nn = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double2 pv = p[i], ov = om[i], qo = qold_qnew[i], qv = q[i], tv = qt[i], uv = u[i], xv = x[i];
        const cplx<double> P{pv.x, pv.y}, O{ov.x, ov.y}, QO{qo.x, qo.y}, Q{qv.x, qv.y}, T{tv.x, tv.y},
            U{uv.x, uv.y}, X{xv.x, xv.y};
        const cplx<double> alpha{k.ar, k.ai}, kappa{k.kr, k.ki}, lam{k.lr, k.li}, eta{k.er, k.ei},
            gam{k.gr, k.gi};
        const cplx<double> On = alpha * P + kappa * (QO - O);
        const cplx<double> Pn = P + lam * (QO - O);
        const cplx<double> Xn = X + eta * (Q - On);
        const double is = 1.0 / k.sigma;
        const cplx<double> Qn = is * (gam * T + U);
        const cplx<double> Tn = k.sigma * T + cmul_conj(gam, Qn);
        om[i] = make_double2(On.re, On.im);
        p[i] = make_double2(Pn.re, Pn.im);
        x[i] = make_double2(Xn.re, Xn.im);
        qold_qnew[i] = make_double2(Qn.re, Qn.im);
        qt[i] = make_double2(Tn.re, Tn.im);
        nn += Qn.re * Qn.re + Qn.im * Qn.im;
    }
    __shared__ double lds[4];
    const double t = block_sum<256>(nn, lds);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

struct SumrOut {
    int iters = 0;
    int restarts = 0;
    double resid = 0.0;
    bool converged = false;
};

static double norm_f64(Context &c, const double2 *x)
{
    std::vector<double> n2;
    norm2_f64(c, x, 1, n2);
    return std::sqrt(n2[0]);
}

static zc dot1(Context &c, const double2 *x, const double2 *y)
{
    std::vector<cplx<double>> d;
    dot_f64(c, x, y, 1, d);
    return zc(d[0].re, d[0].im);
}

// y = a x + b y  (complex scalars, one field)
static void axpby1(Context &c, zc a, const double2 *x, zc b, double2 *y)
{
    cplx<double> ca{a.real(), a.imag()}, cb{b.real(), b.imag()};
    axpby_f64(c, &ca, x, &cb, y, 1);
}

// relSUMR for (1 + rho U) x = bp, starting from x (which holds x0 or zero).
// Ax0 (nullable) is (1 + rho U) x0 when the caller knows it (the deflated
// start supplies it from the stored D psi', Sec. 4), which saves a sign call.
// collect: feed every (q, U q) to eigSUMR (Alg. 5) and use the stricter of the
// inversion and eigenvector sign accuracies (Sec. 5.1).
static SumrOut sumr(Context &c, const ovl_zolo &z, const ovl_solver_params &prm, double rhoK, double rho,
                    const double2 *bp, double2 *x, bool x_is_zero, const double2 *Ax0, double tol, double epsA,
                    bool collect, ovl_stats *st)
{
    const size_t FB = field_bytes(c.g, OVL_F64);
    double2 *rt = (double2 *)c.buf("s_rt", FB);
    double2 *p = (double2 *)c.buf("s_p", FB);
    double2 *om = (double2 *)c.buf("s_om", FB);
    double2 *qa = (double2 *)c.buf("s_qa", FB);
    double2 *qb = (double2 *)c.buf("s_qb", FB);
    double2 *qt = (double2 *)c.buf("s_qt", FB);
    double2 *u = (double2 *)c.buf("s_u", FB);
    const int64_t n = 12 * c.g.V;
    const int nblk = 512;
    double *part = (double *)c.buf("s_part", sizeof(double) * nblk);
    double *res = (double *)c.buf("s_res", sizeof(double));

    const double bn = norm_f64(c, bp);
    SumrOut out;
    if (bn == 0.0) {
        zero_fields(c, x, 1, OVL_F64);
        out.converged = true;
        return out;
    }
    auto eta_for = [&](double resid) {
        double e = std::fmin(prm.relax_floor, epsA * bn / resid);
        if (collect) e = std::fmin(e, eig_sign_accuracy(c));
        return e;
    };
    const double zeta = 1.0;
    double resid = bn;
    bool first = true;
    while (true) {
        // r~ = b - (1 + rho U) x
        if (first && x_is_zero) {
            copy_fields(c, bp, rt, 1, OVL_F64);
        } else if (first && Ax0 != nullptr) {
            copy_fields(c, bp, rt, 1, OVL_F64);
            axpby1(c, zc(-1.0), Ax0, zc(1.0), rt);
        } else {
            const double eta = eta_for(resid);
            unitary_f64(c, rhoK, z, x, u, 1, eta, prec_for(prm, eta), prm.max_mscg, st);
            copy_fields(c, bp, rt, 1, OVL_F64);
            axpby1(c, zc(-1.0), x, zc(1.0), rt);
            axpby1(c, zc(-rho), u, zc(1.0), rt);
        }
        first = false;
        double delta = norm_f64(c, rt);
        if (!std::isfinite(delta)) throw Error{OVL_ERR_BREAKDOWN, "SUMR: non-finite residual"};
        resid = delta;
        if (delta <= tol * bn) {
            out.resid = delta;
            out.converged = true;
            return out;
        }
        zc phi_hat = 1.0 / delta, tau_hat = delta / rho;
        zc phi = 0.0, s = 0.0, lam = 0.0, c_dag = 1.0, cc = 1.0, gamma = 1.0;
        double r = 1.0;
        double sigma = 1.0;
        zero_fields(c, om, 1, OVL_F64);
        zero_fields(c, p, 1, OVL_F64);
        double2 *q = qa, *q_old = qb;
        zero_fields(c, q_old, 1, OVL_F64);
        {
            cplx<double> a{1.0 / delta, 0.0}, b0{0.0, 0.0};
            axpby_f64(c, &a, rt, &b0, q, 1);
        }
        copy_fields(c, q, qt, 1, OVL_F64);
        bool restart = false;
        while (true) {
            resid = rho * std::abs(tau_hat);
            if (resid <= tol * bn) {
                out.resid = resid;
                out.converged = true;
                return out;
            }
            if (out.iters >= prm.max_middle) {
                out.resid = resid;
                return out;
            }
            const double r_pp = r;
            const double eta_j = eta_for(resid);
            unitary_f64(c, rhoK, z, q, u, 1, eta_j, prec_for(prm, eta_j), prm.max_mscg, st);
            if (collect) eig_collect(c, q, u);
            gamma = dot1(c, qt, u);
            if (!(std::abs(gamma) < 1.0)) {
                restart = true;
                break;
            }
            sigma = std::sqrt(1.0 - std::norm(gamma));
            const zc alpha = gamma * delta;
            gamma = -gamma;
            const zc r_p = alpha * phi + s * zeta / rho;
            const zc r_hat = alpha * phi_hat + c_dag * zeta / rho;
            const double nrm = std::sqrt(std::norm(r_hat) + sigma * sigma);
            c_dag = r_hat / nrm;
            cc = std::conj(c_dag);
            s = -sigma / nrm;
            const zc rn = s * sigma - cc * r_hat;
            const zc tau = -cc * tau_hat;
            tau_hat = s * tau_hat;
            const zc eta = tau / rn;
            const zc kappa = r_p / r_pp;
            // vector statements (fused), with lambda from the previous iteration
            SumrCoef k{alpha.real(), alpha.imag(), kappa.real(), kappa.imag(), lam.real(), lam.imag(),
                       eta.real(),   eta.imag(),   gamma.real(), gamma.imag(), sigma};
            k_sumr_step<<<nblk, 256, 0, c.stream>>>(k, x, p, om, q_old, q, qt, u, n, part);
            OVL_HIP(hipGetLastError());
            std::swap(q, q_old);   // q_old <- old q, q <- new q
            delta = sigma * delta;
            phi = s * std::conj(gamma) / delta - cc * phi_hat;
            // r is real in exact arithmetic for this recurrence; keep its modulus-phase form
            r = rn.real();
            lam = phi / rn;
            phi_hat = s * phi_hat + c_dag * std::conj(gamma) / delta;
            out.iters += 1;
            if (st) st->sumr_iters += 1;
            // ||q|| monitoring (Sec. 2)
            sum_partials(c, part, nblk, 1, res);
            double qn2;
            OVL_HIP(hipMemcpyAsync(&qn2, res, sizeof(double), hipMemcpyDeviceToHost, c.stream));
            OVL_HIP(hipStreamSynchronize(c.stream));
            if (!std::isfinite(qn2)) throw Error{OVL_ERR_BREAKDOWN, "SUMR: non-finite basis vector"};
            if (std::fabs(std::sqrt(qn2) - 1.0) > prm.norm_restart) {
                restart = true;
                break;
            }
        }
        if (restart) {
            out.restarts += 1;
            if (st) st->restarts += 1;
            if (out.restarts > 50) {
                out.resid = resid;
                return out;
            }
        }
    }
}

ovl_status solve_one(Context &c, const ovl_zolo &z, const ovl_solver_params &prm, const double2 *b, double2 *x,
                     ovl_stats *st)
{
    const auto t0 = std::chrono::steady_clock::now();
    const double mu = prm.mu;
    const double rhoK = prm.rho;
    const double rho = (1.0 - mu) / (1.0 + mu);
    const size_t FB = field_bytes(c.g, OVL_F64);
    const int maxo = prm.max_outer;
    double2 *Cv = (double2 *)c.buf("g_C", FB * maxo);
    double2 *Uv = (double2 *)c.buf("g_U", FB * maxo);
    double2 *r = (double2 *)c.buf("g_r", FB);
    double2 *uu = (double2 *)c.buf("g_u", FB);
    double2 *cv = (double2 *)c.buf("g_c", FB);
    double2 *bp = (double2 *)c.buf("g_bp", FB);

    zero_fields(c, x, 1, OVL_F64);
    copy_fields(c, b, r, 1, OVL_F64);
    if (prm.eig_calc) eig_configure(c, prm.n_eig, prm.m_eig, mu, prm.delta_split, prm.eig_eps, prm.k_recalc);
    const double bn = norm_f64(c, b);
    if (bn == 0.0) {
        if (st) st->computed_relres = 0.0;
        return OVL_OK;
    }
    double rn = bn;
    int i = 0;
    ovl_status status = OVL_OK;
    while (rn > 0.5 * prm.tol * bn) {
        if (i >= maxo) {
            status = OVL_ERR_NOT_CONVERGED;
            break;
        }
        // middle solve D u = r to relative accuracy eta_tilde: (1 + rho U) u = 2 r/(1 + mu)
        {
            cplx<double> a{2.0 / (1.0 + mu), 0.0}, b0{0.0, 0.0};
            axpby_f64(c, &a, r, &b0, bp, 1);
        }
        // deflated start (Sec. 4): u0 from the eigenspace, (1 + rho U) u0 = 2 D u0/(1 + mu)
        const bool defl = prm.use_deflation && c.eig.k >= c.eig.n && c.eig.n > 0 && c.eig.ndiag > 0;
        double2 *Ax0 = nullptr;
        if (defl) {
            Ax0 = (double2 *)c.buf("g_Ax0", FB);
            double2 *Dx0 = (double2 *)c.buf("g_Dx0", FB);
            eig_project(c, r, uu, Dx0);
            cplx<double> a{2.0 / (1.0 + mu), 0.0}, b0{0.0, 0.0};
            axpby_f64(c, &a, Dx0, &b0, Ax0, 1);
        } else {
            zero_fields(c, uu, 1, OVL_F64);
        }
        const bool collect = prm.eig_calc != 0;
        SumrOut so = sumr(c, z, prm, rhoK, rho, bp, uu, !defl, Ax0, prm.eta_tilde, prm.eta_tilde, collect, st);
        if (collect) {
            eig_diagonalise(c);   // the closing Alg. 6 of Alg. 5
            if (c.eig.ndiag > 0 && prm.k_recalc > 0 && c.eig.ndiag % prm.k_recalc == 0)
                eig_recompute(c, rhoK, z, 1e-12, st);
        }
        (void)so;
        // c = D u, to ||D u - c|| <= eps ||b|| / 4
        const double un = norm_f64(c, uu);
        const double eta_c = std::fmin(1e-2, prm.tol * bn / (2.0 * (1.0 - mu) * un));
        overlap_f64(c, rhoK, mu, z, uu, cv, 1, eta_c, prec_for(prm, eta_c), prm.max_mscg, st);
        // modified Gram-Schmidt against C[0..i)
        for (int j = 0; j < i; ++j) {
            const zc beta = dot1(c, Cv + (size_t)j * 12 * c.g.V, cv);
            axpby1(c, -beta, Cv + (size_t)j * 12 * c.g.V, zc(1.0), cv);
            axpby1(c, -beta, Uv + (size_t)j * 12 * c.g.V, zc(1.0), uu);
        }
        const double cn = norm_f64(c, cv);
        if (!(cn > 0.0) || !std::isfinite(cn)) throw Error{OVL_ERR_BREAKDOWN, "GMRESR: zero or non-finite c"};
        double2 *Ci = Cv + (size_t)i * 12 * c.g.V, *Ui = Uv + (size_t)i * 12 * c.g.V;
        {
            cplx<double> a{1.0 / cn, 0.0}, b0{0.0, 0.0};
            axpby_f64(c, &a, cv, &b0, Ci, 1);
            axpby_f64(c, &a, uu, &b0, Ui, 1);
        }
        const zc alpha = dot1(c, Ci, r);
        axpby1(c, alpha, Ui, zc(1.0), x);
        axpby1(c, -alpha, Ci, zc(1.0), r);
        rn = norm_f64(c, r);
        ++i;
        if (st) st->gmresr_steps += 1;
        if (prm.verbose)
            std::fprintf(stderr, "[ovl] GMRESR step %d: middle iters %d, ||r||/||b|| = %.3e\n", i, so.iters,
                         rn / bn);
    }
    OVL_HIP(hipStreamSynchronize(c.stream));
    if (st) {
        st->computed_relres = rn / bn;
        st->seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return status;
}

}  // namespace ovl
