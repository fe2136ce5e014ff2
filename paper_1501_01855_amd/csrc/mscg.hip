// sign(K) by the Zolotarev partial fractions (paper Sec. 3, eq. 7) with the
// lowest kernel eigenvectors treated exactly (Sec. 1 after eq. 4), the
// shifted inversions of K^2 + sigma_l done by one multi-shift CG.
//
// One CG iteration is six launches on the context's stream, with all of the
// recurrence scalars (alpha, beta, zeta_l, ...) kept in device memory so that
// the host never waits inside the loop:
//   1. t = K p                                  (stencil)
//   2. w = K t + s0 p, partial (p, w)           (stencil + fused dot)
//   3. alpha, zeta_l', alpha_l                  (one block per field)
//   4. r' = r - alpha w, partial ||r'||^2       (fused update + norm)
//   5. beta, beta_l, freezing                   (one block per field)
//   6. y += sum_l omega_l alpha_l p_l,          (one pass over the active
//      p_l = zeta_l' r' + beta_l p_l                shift vectors)
// Only y = sum_l omega_l x_l is stored, never the x_l themselves.  A shift is
// frozen once omega_l |zeta_l| ||r|| / (2 sqrt(sigma_l)) <= eta ||b|| / N_Z,
// which bounds the error of the rational function by eta ||b||.  The host
// polls a per-field stop iteration every few iterations.
#include <cmath>

#include "context.h"
#include "fields.h"
#include "kernels.h"
#include "ops.h"

namespace ovl {

constexpr int NZMAX = OVL_MAX_NZ;

struct MscgScal {
    double rr, alpha, beta, alpha_old, beta_old, b2;
    int iters, breakdown, act_total, pad1;
    double zeta[NZMAX], zeta_old[NZMAX], zn[NZMAX], coef_y[NZMAX], bl[NZMAX];
    int act[NZMAX], act_next[NZMAX];
};

struct MscgConst {
    int nz, base, maxiter, pad;
    double s0;
    double sigma[NZMAX], omega[NZMAX], tol2[NZMAX];
};

// --------------------------------------------------------------- scalar kernels
__device__ double reduce_partials(const double *p, int n, double *lds)
{
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += p[i];
    return block_sum<256>(v, lds);
}

__global__ void k_mscg_init(MscgScal *S, int *stop, const double *partial, int nblk, MscgConst k)
{
    __shared__ double lds[4];
    const int f = blockIdx.x;
    const double b2 = reduce_partials(partial + (int64_t)f * nblk, nblk, lds);
    if (threadIdx.x != 0) return;
    MscgScal &s = S[f];
    s.rr = b2;
    s.b2 = b2;
    s.alpha = 0.0;
    s.beta = 0.0;
    s.alpha_old = 1.0;
    s.beta_old = 0.0;
    s.iters = 0;
    s.breakdown = 0;
    s.act_total = 0;
    for (int l = 0; l < k.nz; ++l) {
        s.zeta[l] = 1.0;
        s.zeta_old[l] = 1.0;
        s.zn[l] = 1.0;
        s.coef_y[l] = 0.0;
        s.bl[l] = 0.0;
        s.act[l] = 1;
        s.act_next[l] = b2 > 0.0 ? 1 : 0;
    }
    stop[f] = b2 > 0.0 ? 0x7fffffff : 0;
}

__global__ void k_mscg_alpha(MscgScal *S, const int *stop, const double *partial, int nblk, int it,
                             MscgConst k)
{
    __shared__ double lds[4];
    const int f = blockIdx.x;
    if (it >= stop[f]) return;
    const double pw = reduce_partials(partial + (int64_t)f * nblk, nblk, lds);
    if (threadIdx.x != 0) return;
    MscgScal &s = S[f];
    int na = 0;
    for (int l = 0; l < k.nz; ++l) {
        s.act[l] = s.act_next[l];
        na += s.act[l];
    }
    s.act_total += na;
    const double alpha = s.rr / pw;
    if (!(pw > 0.0) || !isfinite(alpha)) {
        s.breakdown = 1;
        s.alpha = 0.0;
        for (int l = 0; l < k.nz; ++l) s.coef_y[l] = 0.0;
        return;
    }
    s.alpha = alpha;
    for (int l = 0; l < k.nz; ++l) {
        if (!s.act[l]) continue;
        const double z = s.zeta[l], zo = s.zeta_old[l];
        const double zn = (z * zo * s.alpha_old) /
                          (alpha * s.beta_old * (zo - z) + zo * s.alpha_old * (1.0 + (k.sigma[l] - k.s0) * alpha));
        s.zn[l] = zn;
        s.coef_y[l] = k.omega[l] * (alpha * zn / z);
    }
}

__global__ void k_mscg_beta(MscgScal *S, int *stop, const double *partial, int nblk, int it, MscgConst k)
{
    __shared__ double lds[4];
    const int f = blockIdx.x;
    if (it >= stop[f]) return;
    const double rr_new = reduce_partials(partial + (int64_t)f * nblk, nblk, lds);
    if (threadIdx.x != 0) return;
    MscgScal &s = S[f];
    const double beta = rr_new / s.rr;
    int any = 0;
    for (int l = 0; l < k.nz; ++l) {
        if (!s.act[l]) {
            s.act_next[l] = 0;
            continue;
        }
        const double q = s.zn[l] / s.zeta[l];
        s.bl[l] = beta * q * q;
        s.zeta_old[l] = s.zeta[l];
        s.zeta[l] = s.zn[l];
        const int keep = !(s.zeta[l] * s.zeta[l] * rr_new <= k.tol2[l] * s.b2);
        s.act_next[l] = keep;
        any |= keep;
    }
    s.alpha_old = s.alpha;
    s.beta_old = beta;
    s.beta = beta;
    s.rr = rr_new;
    s.iters += 1;
    if (s.breakdown || !isfinite(rr_new)) {
        s.breakdown = 1;
        any = 0;
    }
    if (!any || s.iters >= k.maxiter) stop[f] = it + 1;
}

// --------------------------------------------------------------- vector kernels
template <typename ST>
__global__ __launch_bounds__(256) void k_norm2(const ST *__restrict__ x, int64_t V, double *partial)
{
    using R = typename Planes<ST>::R;
    constexpr int NP = Planes<ST>::n;
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int f = blockIdx.y;
    double d = 0.0;
    if (s < V) {
        cplx<R> v[12];
        ld_sp(x + (int64_t)f * NP * V, V, s, v);
#pragma unroll
        for (int c = 0; c < 12; ++c) d += (double)v[c].re * (double)v[c].re + (double)v[c].im * (double)v[c].im;
    }
    __shared__ double lds[4];
    const double t = block_sum<256>(d, lds);
    if (threadIdx.x == 0) partial[(int64_t)f * gridDim.x + blockIdx.x] = t;
}

// r' = r - alpha w (r = src on the first iteration); partial ||r'||^2
template <typename ST>
__global__ __launch_bounds__(256) void k_mscg_rupdate(const ST *__restrict__ rin, ST *__restrict__ r,
                                                      const ST *__restrict__ w, const MscgScal *S,
                                                      const int *stop, int it, int64_t V, double *partial)
{
    using R = typename Planes<ST>::R;
    constexpr int NP = Planes<ST>::n;
    const int f = blockIdx.y;
    if (it >= stop[f]) return;
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double d = 0.0;
    if (s < V) {
        const R alpha = (R)S[f].alpha;
        cplx<R> a[12], b[12];
        ld_sp(rin + (int64_t)f * NP * V, V, s, a);
        ld_sp(w + (int64_t)f * NP * V, V, s, b);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            a[c] = a[c] - alpha * b[c];
            d += (double)a[c].re * (double)a[c].re + (double)a[c].im * (double)a[c].im;
        }
        st_sp(r + (int64_t)f * NP * V, V, s, a);
    }
    __shared__ double lds[4];
    const double t = block_sum<256>(d, lds);
    if (threadIdx.x == 0) partial[(int64_t)f * gridDim.x + blockIdx.x] = t;
}

// y += sum_l omega_l alpha_l p_l ; p_l = zeta_l' r + beta_l p_l (active shifts).
// On the first iteration every p_l is the source and y starts at zero.
template <typename ST>
__global__ __launch_bounds__(256) void k_mscg_shift(const ST *__restrict__ src, const ST *__restrict__ r,
                                                    ST *__restrict__ y, ST *__restrict__ p, int nz,
                                                    const MscgScal *S, const int *stop, int it, int64_t V)
{
    using R = typename Planes<ST>::R;
    constexpr int NP = Planes<ST>::n;
    const int f = blockIdx.y;
    if (it >= stop[f]) return;
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= V) return;
    const MscgScal &sc = S[f];
    const int64_t fo = (int64_t)f * NP * V;
    const int64_t pstride = (int64_t)gridDim.y * NP * V;   // shift-major: p[l][f]
    cplx<R> rv[12], yv[12], pv[12];
    ld_sp(r + fo, V, s, rv);
    if (it == 0) {
#pragma unroll
        for (int c = 0; c < 12; ++c) yv[c] = {R(0), R(0)};
        ld_sp(src + fo, V, s, pv);
    } else {
        ld_sp(y + fo, V, s, yv);
    }
    for (int l = 0; l < nz; ++l) {
        if (!sc.act[l]) continue;
        ST *pl = p + l * pstride + fo;
        if (it != 0) ld_sp(pl, V, s, pv);
        const R cy = (R)sc.coef_y[l], zn = (R)sc.zn[l], bl = (R)sc.bl[l];
        cplx<R> nv[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            yv[c] = yv[c] + cy * pv[c];
            nv[c] = zn * rv[c] + bl * pv[c];
        }
        st_sp(pl, V, s, nv);
    }
    st_sp(y + fo, V, s, yv);
}

// ---- low-mode projection (basis FP64 packed [n][12][V], fields in ST)
template <typename ST>
__global__ __launch_bounds__(256) void k_low_dots(const double2 *__restrict__ basis, int n,
                                                  const ST *__restrict__ x, int64_t V, double *partial)
{
    using R = typename Planes<ST>::R;
    constexpr int NP = Planes<ST>::n;
    const int f = blockIdx.y;
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    __shared__ double lds[4];
    cplx<R> xv[12];
    if (s < V) ld_sp(x + (int64_t)f * NP * V, V, s, xv);
    for (int j = 0; j < n; ++j) {
        double dr = 0.0, di = 0.0;
        if (s < V) {
            cplx<double> b[12];
            ld_sp(basis + (int64_t)j * 12 * V, V, s, b);
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                const double xr = xv[c].re, xi = xv[c].im;
                dr += b[c].re * xr + b[c].im * xi;
                di += b[c].re * xi - b[c].im * xr;
            }
        }
        const double tr = block_sum<256>(dr, lds);
        const double ti = block_sum<256>(di, lds);
        if (threadIdx.x == 0) {
            partial[(((int64_t)f * n + j) * 2 + 0) * gridDim.x + blockIdx.x] = tr;
            partial[(((int64_t)f * n + j) * 2 + 1) * gridDim.x + blockIdx.x] = ti;
        }
    }
}

__global__ void k_reduce_rows(const double *partial, int nblk, double *out)
{
    __shared__ double lds[4];
    const double v = reduce_partials(partial + (int64_t)blockIdx.x * nblk, nblk, lds);
    if (threadIdx.x == 0) out[blockIdx.x] = v;
}

// x_perp = x - sum_j c_j v_j ; ex = sum_j sign(lambda_j) c_j v_j
template <typename ST>
__global__ __launch_bounds__(256) void k_low_project(const double2 *__restrict__ basis, int n,
                                                     const double *__restrict__ coef, const double *__restrict__ sgn,
                                                     const ST *__restrict__ x, ST *__restrict__ xp,
                                                     ST *__restrict__ ex, int64_t V)
{
    using R = typename Planes<ST>::R;
    constexpr int NP = Planes<ST>::n;
    const int f = blockIdx.y;
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= V) return;
    cplx<R> xv[12];
    ld_sp(x + (int64_t)f * NP * V, V, s, xv);
    cplx<double> a[12], e[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        a[c] = {(double)xv[c].re, (double)xv[c].im};
        e[c] = {0.0, 0.0};
    }
    for (int j = 0; j < n; ++j) {
        const cplx<double> cj = {coef[((int64_t)f * n + j) * 2], coef[((int64_t)f * n + j) * 2 + 1]};
        const double sj = sgn[j];
        cplx<double> b[12];
        ld_sp(basis + (int64_t)j * 12 * V, V, s, b);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const cplx<double> t = cj * b[c];
            a[c] = a[c] - t;
            e[c] = e[c] + sj * t;
        }
    }
    cplx<R> o[12], oe[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        o[c] = {(R)a[c].re, (R)a[c].im};
        oe[c] = {(R)e[c].re, (R)e[c].im};
    }
    st_sp(xp + (int64_t)f * NP * V, V, s, o);
    st_sp(ex + (int64_t)f * NP * V, V, s, oe);
}

// --------------------------------------------------------------- host driver
template <typename ST>
static void sign_t(Context &c, double rho, const ovl_zolo &z, const void *in, void *out, int nf,
                   double eta, int prec, int maxiter, ovl_stats *st)
{
    const Geom &g = c.g;
    const int64_t V = g.V;
    const size_t FB = field_bytes(g, prec);
    const unsigned nblk = site_blocks(g);
    const dim3 grid(nblk, nf);
    const int nz = z.n_z;
    OVL_REQUIRE(nz >= 1 && nz <= NZMAX, OVL_ERR_ARG, "n_z out of range");
    OVL_REQUIRE(eta > 0.0, OVL_ERR_ARG, "eta must be positive");
    for (int l = 0; l < nz; ++l)
        OVL_REQUIRE(z.sigma[l] > 0.0 && z.omega[l] > 0.0, OVL_ERR_ARG, "Zolotarev coefficients must be positive");

    ST *src = (ST *)c.buf("ms_src", FB * nf);
    ST *ex = (ST *)c.buf("ms_ex", FB * nf);
    ST *r = (ST *)c.buf("ms_r", FB * nf);
    ST *t = (ST *)c.buf("ms_t", FB * nf);
    ST *w = (ST *)c.buf("ms_w", FB * nf);
    ST *y = (ST *)c.buf("ms_y", FB * nf);
    ST *p = (ST *)c.buf("ms_p", FB * nf * nz);
    double *part = (double *)c.buf("ms_part", sizeof(double) * (size_t)nblk * nf * 2 * (c.n_low > 0 ? c.n_low : 1));
    double *coef = (double *)c.buf("ms_coef", sizeof(double) * (size_t)nf * 2 * (c.n_low > 0 ? c.n_low : 1));
    double *sgn = (double *)c.buf("ms_sgn", sizeof(double) * (c.n_low > 0 ? c.n_low : 1));
    MscgScal *S = (MscgScal *)c.buf("ms_scal", sizeof(MscgScal) * nf);
    int *stop = (int *)c.buf("ms_stop", sizeof(int) * nf);

    // 1. low-mode split: src = (1 - P) in, ex = sum sign(lambda) P in
    const bool low = c.n_low > 0;
    if (low) {
        std::vector<double> sg(c.n_low);
        for (int j = 0; j < c.n_low; ++j) sg[j] = c.low_evals[j] >= 0.0 ? 1.0 : -1.0;
        OVL_HIP(hipMemcpyAsync(sgn, sg.data(), sizeof(double) * c.n_low, hipMemcpyHostToDevice, c.stream));
        k_low_dots<ST><<<grid, 256, 0, c.stream>>>(c.low, c.n_low, (const ST *)in, V, part);
        k_reduce_rows<<<nf * c.n_low * 2, 256, 0, c.stream>>>(part, nblk, coef);
        k_low_project<ST><<<grid, 256, 0, c.stream>>>(c.low, c.n_low, coef, sgn, (const ST *)in, src, ex, V);
    } else {
        OVL_HIP(hipMemcpyAsync(src, in, FB * nf, hipMemcpyDeviceToDevice, c.stream));
    }
    OVL_HIP(hipGetLastError());

    // 2. constants
    MscgConst k{};
    k.nz = nz;
    k.maxiter = maxiter;
    int base = 0;
    for (int l = 1; l < nz; ++l)
        if (z.sigma[l] < z.sigma[base]) base = l;
    k.base = base;
    k.s0 = z.sigma[base];
    for (int l = 0; l < nz; ++l) {
        k.sigma[l] = z.sigma[l];
        k.omega[l] = z.omega[l];
        const double tl = eta * 2.0 * std::sqrt(z.sigma[l]) / (nz * z.omega[l]);
        k.tol2[l] = tl * tl;
    }
    zero_fields(c, y, nf, prec);   // y stays zero for a zero source
    k_norm2<ST><<<grid, 256, 0, c.stream>>>(src, V, part);
    k_mscg_init<<<nf, 256, 0, c.stream>>>(S, stop, part, nblk, k);
    OVL_HIP(hipGetLastError());

    // 3. iterations; poll the stop flags every CHUNK iterations, one chunk behind
    const int CHUNK = 8;
    int *hstop = (int *)c.host_stage(sizeof(int) * nf * 2);
    hipEvent_t evs[2] = {c.event(), c.event()};
    const size_t pst = FB * nf;   // bytes between shift vectors
    ST *pbase = (ST *)((char *)p + pst * base);
    int it = 0;
    int pending = -1;   // slot of the chunk awaiting a check
    bool finished = false;
    while (!finished) {
        for (int j = 0; j < CHUNK; ++j, ++it) {
            const ST *pin = it == 0 ? src : pbase;
            stencil(c, EPI_K, prec, pin, t, nf, rho, 0.0, nullptr, nullptr, stop, it);
            stencil(c, EPI_K2DOT, prec, t, w, nf, rho, k.s0, pin, part, stop, it);
            k_mscg_alpha<<<nf, 256, 0, c.stream>>>(S, stop, part, nblk, it, k);
            k_mscg_rupdate<ST><<<grid, 256, 0, c.stream>>>(it == 0 ? src : r, r, w, S, stop, it, V, part);
            k_mscg_beta<<<nf, 256, 0, c.stream>>>(S, stop, part, nblk, it, k);
            PendingEvent pe;
            if (c.prof) c.prof_begin(pe, KERN_SHIFT, prec, 0.0);
            k_mscg_shift<ST><<<grid, 256, 0, c.stream>>>(src, r, y, p, nz, S, stop, it, V);
            if (c.prof) c.prof_end(pe);
            OVL_HIP(hipGetLastError());
        }
        const int slot = (it / CHUNK) & 1;
        OVL_HIP(hipMemcpyAsync(hstop + slot * nf, stop, sizeof(int) * nf, hipMemcpyDeviceToHost, c.stream));
        OVL_HIP(hipEventRecord(evs[slot], c.stream));
        if (pending >= 0) {
            OVL_HIP(hipEventSynchronize(evs[pending]));
            bool all = true;
            for (int f = 0; f < nf; ++f) all = all && hstop[pending * nf + f] != 0x7fffffff;
            if (all) finished = true;
        }
        pending = slot;
        if (it >= maxiter + 2 * CHUNK) finished = true;
    }
    OVL_HIP(hipStreamSynchronize(c.stream));

    // 4. s = K y + ex
    if (low) {
        stencil(c, EPI_KPLUS, prec, y, out, nf, rho, 0.0, ex, nullptr);
    } else {
        stencil(c, EPI_K, prec, y, out, nf, rho, 0.0, nullptr, nullptr);
    }
    OVL_HIP(hipGetLastError());

    std::vector<MscgScal> hs(nf);
    OVL_HIP(hipMemcpyAsync(hs.data(), S, sizeof(MscgScal) * nf, hipMemcpyDeviceToHost, c.stream));
    OVL_HIP(hipStreamSynchronize(c.stream));
    c.prof_collect();
    int64_t iters = 0, act_total = 0;
    bool brk = false, capped = false;
    for (int f = 0; f < nf; ++f) {
        iters += hs[f].iters;
        act_total += hs[f].act_total;
        brk = brk || hs[f].breakdown;
        capped = capped || hs[f].iters >= maxiter;
    }
    if (st) {
        st->mscg_iters += iters;
        st->dslash_calls[prec] += 2 * iters + nf;
        st->sign_calls[prec] += nf;
    }
    c.last_mscg_iters = iters;
    // algorithmic bytes of the shift kernel: r, y in, y out, 2 per active shift
    if (c.prof) c.slots[KERN_SHIFT][prec].bytes += (double)FB * (3.0 * iters + 2.0 * act_total);
    OVL_REQUIRE(!brk, OVL_ERR_BREAKDOWN, "multi-shift CG breakdown (non-positive curvature or NaN)");
    OVL_REQUIRE(!capped, OVL_ERR_NOT_CONVERGED, "multi-shift CG hit its iteration limit");
}

void sign_mscg(Context &c, double rho, const ovl_zolo &z, const void *in, void *out, int nf,
               double eta, int prec, int maxiter, ovl_stats *st)
{
    if (prec == OVL_F64)
        sign_t<double2>(c, rho, z, in, out, nf, eta, prec, maxiter, st);
    else if (prec == OVL_F32)
        sign_t<float4>(c, rho, z, in, out, nf, eta, prec, maxiter, st);
    else
        throw Error{OVL_ERR_UNSUPPORTED, "sign: precision"};
}

}  // namespace ovl
