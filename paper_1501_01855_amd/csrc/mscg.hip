// sign(K) by the Zolotarev partial fractions (paper Sec. 3, eq. 7) with the
// lowest kernel eigenvectors treated exactly (Sec. 1 after eq. 4), the
// shifted inversions of K^2 + sigma_l done by one multi-shift CG.
//
// One CG iteration is four launches on the context's stream; the recurrence
// scalars live in device memory (mscg_state.h) so the host never waits inside
// the loop:
//   1. t = K p                                  (stencil)
//   2. w = K t + s0 p, (p, w) per tile          (stencil + fused dot)
//   3. alpha = rr/(p, w); r' = r - alpha w;     (every block reduces the
//      ||r'||^2 per block                        tile partials itself)
//   4. beta, zeta_l', alpha_l, beta_l;          (one pass over the active
//      y += sum_l omega_l alpha_l p_l,              shift vectors; block 0
//      p_l = zeta_l' r' + beta_l p_l                writes the next state)
// Only y = sum_l omega_l x_l is stored, never the x_l themselves.  A shift is
// frozen once omega_l |zeta_l| ||r|| / (2 sqrt(sigma_l)) <= eta ||b|| / N_Z,
// which bounds the error of the rational function by eta ||b||.  The host
// polls a per-field stop iteration every few iterations.
#include <algorithm>
#include <cmath>

#include "context.h"
#include "fields.h"
#include "kernels.h"
#include "mscg_state.h"
#include "ops.h"

namespace ovl {

static constexpr int UPD_BLOCKS = 1024;   // grid of the update kernels (grid-stride over sites)

struct MscgFinal {
    int iters, breakdown, act_total, pad;
};

__global__ void k_mscg_init(MscgScal *S, int *stop, const double *partial, int nblk, MscgConst k,
                            const double *eta2)
{
    __shared__ double lds[4];
    const int f = blockIdx.x;
    const double b2 = block_allsum(partial + (int64_t)f * nblk, nblk, lds);
    if (threadIdx.x != 0) return;
    MscgScal &s = S[f];   // parity 0
    s.rr = b2;
    // the freezing test uses eta_f^2 ||b||^2; eta_f <= 0 marks a field to skip
    const double e2 = eta2[f];
    s.b2 = e2 > 0.0 ? e2 * b2 : 0.0;
    s.alpha_old = 1.0;
    s.beta_old = 0.0;
    s.iters = 0;
    s.breakdown = 0;
    s.act_total = 0;
    for (int l = 0; l < k.nz; ++l) {
        s.zeta[l] = 1.0;
        s.zeta_old[l] = 1.0;
        s.act[l] = b2 > 0.0 ? 1 : 0;
    }
    stop[f] = (b2 > 0.0 && e2 > 0.0) ? 0x7fffffff : 0;
}

template <typename ST>
__global__ __launch_bounds__(256) void k_norm2(const ST *__restrict__ x, int64_t V, double *partial)
{
    using R = typename Planes<ST>::R;
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int f = blockIdx.y;
    double d = 0.0;
    if (s < V) {
        cplx<R> v[12];
        ld_sp(x + f * fstride<ST>(V), V, s, v);
#pragma unroll
        for (int c = 0; c < 12; ++c) d += (double)v[c].re * (double)v[c].re + (double)v[c].im * (double)v[c].im;
    }
    __shared__ double lds[4];
    const double t = block_sum<256>(d, lds);
    if (threadIdx.x == 0) partial[(int64_t)f * gridDim.x + blockIdx.x] = t;
}

// r' = r - alpha w (r = src on the first iteration), alpha = rr/(p, w) from the
// stencil's tile partials; ||r'||^2 per block.
template <typename ST>
__global__ __launch_bounds__(256) void k_mscg_rupdate(const ST *__restrict__ rin, ST *__restrict__ r,
                                                      const ST *__restrict__ w, const MscgScal *S,
                                                      const int *stop, int it, int64_t V,
                                                      const double *pw_part, int pw_n, double *rr_part)
{
    using R = typename Planes<ST>::R;
    const int f = blockIdx.y;
    if (it >= stop[f]) return;
    __shared__ double lds[4];
    const int nf = gridDim.y;
    const MscgScal &sc = S[(it & 1) * nf + f];
    const double pw = block_allsum(pw_part + (int64_t)f * pw_n, pw_n, lds);
    const double alpha_d = sc.rr / pw;
    const R alpha = (pw > 0.0 && isfinite(alpha_d)) ? (R)alpha_d : R(0);
    double d = 0.0;
    const int64_t o = f * fstride<ST>(V);
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < V; s += (int64_t)gridDim.x * blockDim.x) {
        cplx<R> a[12], b[12];
        ld_sp(rin + o, V, s, a);
        ld_sp(w + o, V, s, b);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            a[c] = a[c] - alpha * b[c];
            d += (double)a[c].re * (double)a[c].re + (double)a[c].im * (double)a[c].im;
        }
        st_sp(r + o, V, s, a);
    }
    const double t = block_sum<256>(d, lds);
    if (threadIdx.x == 0) rr_part[(int64_t)f * gridDim.x + blockIdx.x] = t;
}

// y += sum_l omega_l alpha_l p_l ; p_l = zeta_l' r + beta_l p_l over the active
// shifts (on the first iteration every p_l is the source and y starts at zero).
// With ALL, y holds one solution per shift, shift-major like p, and
// x_l += omega_l alpha_l p_l (the caller passes omega_l = 1).
// Every block derives the iteration's scalars; block 0 stores the next state.
template <typename ST, bool ALL>
__global__ __launch_bounds__(256) void k_mscg_shift(const ST *__restrict__ src, const ST *__restrict__ r,
                                                    ST *__restrict__ y, ST *__restrict__ p, MscgScal *S,
                                                    const MscgConst *kc, int *stop, MscgFinal *fin, int it,
                                                    int64_t V, const double *pw_part, int pw_n,
                                                    const double *rr_part, int rr_n)
{
    using R = typename Planes<ST>::R;
    const int f = blockIdx.y;
    if (it >= stop[f]) return;
    const int nf = gridDim.y;
    __shared__ double lds[4];
    __shared__ double s_cy[NZMAX], s_zn[NZMAX], s_bl[NZMAX];
    __shared__ int s_act[NZMAX];
    __shared__ int s_keep_any;
    const MscgScal &sc = S[(it & 1) * nf + f];
    const double pw = block_allsum(pw_part + (int64_t)f * pw_n, pw_n, lds);
    const double rr_new = block_allsum(rr_part + (int64_t)f * rr_n, rr_n, lds);
    const double alpha = sc.rr / pw;
    const bool ok = pw > 0.0 && isfinite(alpha) && isfinite(rr_new);
    const double beta = rr_new / sc.rr;
    const int nz = kc->nz;
    if (threadIdx.x == 0) s_keep_any = 0;
    __syncthreads();
    if ((int)threadIdx.x < nz) {
        const int l = threadIdx.x;
        const int act = sc.act[l] && ok;
        s_act[l] = act;
        double zn = sc.zeta[l], cy = 0.0, bl = 0.0;
        if (act) {
            const double z = sc.zeta[l], zo = sc.zeta_old[l];
            zn = (z * zo * sc.alpha_old) /
                 (alpha * sc.beta_old * (zo - z) + zo * sc.alpha_old * (1.0 + (kc->sigma[l] - kc->s0) * alpha));
            cy = kc->omega[l] * (alpha * zn / z);
            const double q = zn / z;
            bl = beta * q * q;
        }
        s_zn[l] = zn;
        s_cy[l] = cy;
        s_bl[l] = bl;
        if (blockIdx.x == 0) {
            MscgScal &nx = S[((it + 1) & 1) * nf + f];
            nx.zeta_old[l] = act ? sc.zeta[l] : sc.zeta_old[l];
            nx.zeta[l] = zn;
            const int keep = act && !(zn * zn * rr_new <= kc->tol2[l] * sc.b2);
            nx.act[l] = keep;
            if (keep) atomicOr(&s_keep_any, 1);
        }
    }
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        MscgScal &nx = S[((it + 1) & 1) * nf + f];
        int na = 0;
        for (int l = 0; l < nz; ++l) na += s_act[l];
        nx.rr = rr_new;
        nx.b2 = sc.b2;
        nx.alpha_old = alpha;
        nx.beta_old = beta;
        nx.iters = sc.iters + 1;
        nx.breakdown = sc.breakdown || !ok;
        nx.act_total = sc.act_total + na;
        fin[f] = MscgFinal{nx.iters, nx.breakdown, nx.act_total, 0};
        if (!s_keep_any || nx.breakdown || nx.iters >= kc->maxiter) stop[f] = it + 1;
    }
    if (!ok) return;
    const int64_t fo = f * fstride<ST>(V);
    const int64_t pstride = nf * fstride<ST>(V);   // shift-major: p[l][f]
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < V; s += (int64_t)gridDim.x * blockDim.x) {
        cplx<R> rv[12], yv[12], pv[12];
        ld_sp(r + fo, V, s, rv);
        if (it == 0) {
#pragma unroll
            for (int c = 0; c < 12; ++c) yv[c] = {R(0), R(0)};
            ld_sp(src + fo, V, s, pv);
        } else if constexpr (!ALL) {
            ld_sp(y + fo, V, s, yv);
        }
        for (int l = 0; l < nz; ++l) {
            if (!s_act[l]) continue;
            ST *pl = p + l * pstride + fo;
            if (it != 0) ld_sp(pl, V, s, pv);
            const R cy = (R)s_cy[l], zn = (R)s_zn[l], bl = (R)s_bl[l];
            if constexpr (ALL) {
                ST *xl = y + l * pstride + fo;
                cplx<R> xv[12];
                if (it != 0) {
                    ld_sp(xl, V, s, xv);
                } else {
#pragma unroll
                    for (int c = 0; c < 12; ++c) xv[c] = {R(0), R(0)};
                }
#pragma unroll
                for (int c = 0; c < 12; ++c) xv[c] = xv[c] + cy * pv[c];
                st_sp(xl, V, s, xv);
            } else {
#pragma unroll
                for (int c = 0; c < 12; ++c) yv[c] = yv[c] + cy * pv[c];
            }
            cplx<R> nv[12];
#pragma unroll
            for (int c = 0; c < 12; ++c) nv[c] = zn * rv[c] + bl * pv[c];
            st_sp(pl, V, s, nv);
        }
        if constexpr (!ALL) st_sp(y + fo, V, s, yv);
    }
}

// ---- low-mode projection (basis FP64 packed [n][12][V], fields in ST)
template <typename ST>
__global__ __launch_bounds__(256) void k_low_dots(const double2 *__restrict__ basis, int n,
                                                  const ST *__restrict__ x, int64_t V, double *partial)
{
    using R = typename Planes<ST>::R;
    const int f = blockIdx.y;
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    __shared__ double lds[4];
    cplx<R> xv[12];
    if (s < V) ld_sp(x + f * fstride<ST>(V), V, s, xv);
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
    const double v = block_allsum(partial + (int64_t)blockIdx.x * nblk, nblk, lds);
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
    const int f = blockIdx.y;
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= V) return;
    cplx<R> xv[12];
    ld_sp(x + f * fstride<ST>(V), V, s, xv);
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
    st_sp(xp + f * fstride<ST>(V), V, s, o);
    st_sp(ex + f * fstride<ST>(V), V, s, oe);
}

// --------------------------------------------------------------- host driver
// out = sign(K) in, or (xs != nullptr) every shifted solution
// xs[l][f] = (K^2 + sigma_l)^{-1} in_f, each to |zeta_l| ||r|| <= eta_f ||in_f||,
// with no low-mode split and no final K.
template <typename ST>
static void sign_t(Context &c, double rho, const ovl_zolo &z, const void *in, void *out, int nf,
                   const double *eta, int prec, int maxiter, ovl_stats *st, void *xs = nullptr)
{
    const bool all = xs != nullptr;
    const Geom &g = c.g;
    const int64_t V = g.V;
    const size_t FB = field_bytes(g, prec);
    const unsigned nblk = site_blocks(g);
    const unsigned nblk_max = (unsigned)stencil_tiles_max(g);   // tiles of any stencil variant
    const dim3 grid(nblk, nf);
    const unsigned nupd = std::min<unsigned>(UPD_BLOCKS, nblk);
    const dim3 ugrid(nupd, nf);
    const int nz = z.n_z;
    OVL_REQUIRE(nz >= 1 && nz <= NZMAX, OVL_ERR_ARG, "n_z out of range");
    int nact = 0;
    std::vector<double> eta2(nf);
    for (int f = 0; f < nf; ++f) {
        eta2[f] = eta[f] > 0.0 ? eta[f] * eta[f] : 0.0;
        nact += eta[f] > 0.0;
    }
    for (int l = 0; l < nz; ++l)
        OVL_REQUIRE(z.sigma[l] > 0.0 && z.omega[l] > 0.0, OVL_ERR_ARG, "Zolotarev coefficients must be positive");

    ST *src = (ST *)c.buf("ms_src", FB * nf);
    ST *ex = (ST *)c.buf("ms_ex", FB * nf);
    ST *r = (ST *)c.buf("ms_r", FB * nf);
    ST *t = (ST *)c.buf("ms_t", FB * nf);
    ST *w = (ST *)c.buf("ms_w", FB * nf);
    ST *y = all ? (ST *)xs : (ST *)c.buf("ms_y", FB * nf);
    ST *p = (ST *)c.buf("ms_p", FB * nf * nz);
    const int nl = c.n_low > 0 ? c.n_low : 1;
    double *part = (double *)c.buf("ms_part", sizeof(double) * (size_t)std::max(nblk_max, nblk * 2 * nl) * nf);
    double *rr_part = (double *)c.buf("ms_part2", sizeof(double) * (size_t)nupd * nf);
    double *coef = (double *)c.buf("ms_coef", sizeof(double) * (size_t)nf * 2 * nl);
    double *sgn = (double *)c.buf("ms_sgn", sizeof(double) * nl);
    MscgScal *S = (MscgScal *)c.buf("ms_scal", sizeof(MscgScal) * 2 * nf);
    MscgFinal *fin = (MscgFinal *)c.buf("ms_fin", sizeof(MscgFinal) * nf);
    int *stop = (int *)c.buf("ms_stop", sizeof(int) * nf);
    MscgConst *kdev = (MscgConst *)c.buf("ms_const", sizeof(MscgConst));

    // 1. low-mode split: src = (1 - P) in, ex = sum sign(lambda) P in
    const bool low = c.n_low > 0 && !all;
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

    // 2. constants and initial state
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
        k.omega[l] = all ? 1.0 : z.omega[l];
        const double tl = all ? 1.0 : 2.0 * std::sqrt(z.sigma[l]) / (nz * z.omega[l]);
        k.tol2[l] = tl * tl;
    }
    OVL_HIP(hipMemcpyAsync(kdev, &k, sizeof(MscgConst), hipMemcpyHostToDevice, c.stream));
    zero_fields(c, y, all ? nf * nz : nf, prec);   // stays zero for a zero source
    k_norm2<ST><<<grid, 256, 0, c.stream>>>(src, V, part);
    double *eta2d = (double *)c.buf("ms_eta2", sizeof(double) * nf);
    OVL_HIP(hipMemcpyAsync(eta2d, eta2.data(), sizeof(double) * nf, hipMemcpyHostToDevice, c.stream));
    k_mscg_init<<<nf, 256, 0, c.stream>>>(S, stop, part, nblk, k, eta2d);
    OVL_HIP(hipGetLastError());

    // 3. iterations; poll the stop flags every CHUNK iterations, one chunk behind
    const int CHUNK = 8;
    int *hstop = (int *)c.host_stage(sizeof(int) * nf * 2);
    hipEvent_t evs[2] = {c.event(), c.event()};
    const size_t pst = FB * nf;   // bytes between shift vectors
    ST *pbase = (ST *)((char *)p + pst * base);
    int it = 0;
    int pending = -1;
    bool finished = false;
    while (!finished) {
        for (int j = 0; j < CHUNK; ++j, ++it) {
            const ST *pin = it == 0 ? src : pbase;
            stencil(c, EPI_K, prec, pin, t, nf, rho, 0.0, nullptr, nullptr, stop, it);
            const int ntile = stencil_k2_dot(c, prec, t, w, nf, rho, k.s0, pin, part, stop, it);
            k_mscg_rupdate<ST><<<ugrid, 256, 0, c.stream>>>(it == 0 ? src : r, r, w, S, stop, it, V, part, ntile,
                                                           rr_part);
            PendingEvent pe;
            if (c.prof) c.prof_begin(pe, KERN_SHIFT, prec, 0.0);
            const PendingEvent *ppe = c.prof ? &pe : nullptr;
            if (all)
                launch_k(c.stream, ppe, k_mscg_shift<ST, true>, ugrid, dim3(256), 0, src, r, y, p, S, kdev, stop,
                         fin, it, V, part, ntile, rr_part, (int)nupd);
            else
                launch_k(c.stream, ppe, k_mscg_shift<ST, false>, ugrid, dim3(256), 0, src, r, y, p, S, kdev, stop,
                         fin, it, V, part, ntile, rr_part, (int)nupd);
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

    // 4. s = K y + ex
    if (all) {
    } else if (low) {
        stencil(c, EPI_KPLUS, prec, y, out, nf, rho, 0.0, ex, nullptr);
    } else {
        stencil(c, EPI_K, prec, y, out, nf, rho, 0.0, nullptr, nullptr);
    }
    OVL_HIP(hipGetLastError());

    std::vector<MscgFinal> hs(nf);
    std::vector<int> hstop_final(nf);
    OVL_HIP(hipMemcpyAsync(hs.data(), fin, sizeof(MscgFinal) * nf, hipMemcpyDeviceToHost, c.stream));
    OVL_HIP(hipMemcpyAsync(hstop_final.data(), stop, sizeof(int) * nf, hipMemcpyDeviceToHost, c.stream));
    OVL_HIP(hipStreamSynchronize(c.stream));
    c.prof_collect();
    int64_t iters = 0, act_total = 0;
    bool brk = false, capped = false;
    for (int f = 0; f < nf; ++f) {
        if (hstop_final[f] == 0) continue;   // zero source: no iteration ran
        iters += hs[f].iters;
        act_total += hs[f].act_total;
        brk = brk || hs[f].breakdown;
        capped = capped || hs[f].iters >= maxiter;
    }
    if (st) {
        st->mscg_iters += iters;
        st->dslash_calls[prec] += 2 * iters + (all ? 0 : nact);
        if (!all) st->sign_calls[prec] += nact;
    }
    c.last_mscg_iters = iters;
    c.last_field_iters.assign(nf, 0);
    for (int f = 0; f < nf; ++f)
        if (hstop_final[f] != 0) c.last_field_iters[f] = hs[f].iters;
    // algorithmic bytes of the shift kernel: r, y in, y out, 2 per active shift
    // (with every solution kept: r, and p_l, x_l in and out per active shift)
    if (c.prof) {
        c.slots[KERN_SHIFT][prec].bytes +=
            all ? (double)FB * (1.0 * iters + 4.0 * act_total) : (double)FB * (3.0 * iters + 2.0 * act_total);
        // the two stencils of each executed iteration (K, then K with the
        // shift, the dot and an extra read of p)
        c.slots[KERN_STENCIL][prec].bytes +=
            (double)iters * (stencil_bytes(g, prec, EPI_K) + stencil_bytes(g, prec, EPI_K2DOT));
    }
    OVL_REQUIRE(!brk, OVL_ERR_BREAKDOWN, "multi-shift CG breakdown (non-positive curvature or NaN)");
    OVL_REQUIRE(!capped, OVL_ERR_NOT_CONVERGED, "multi-shift CG hit its iteration limit");
}

void sign_mscg(Context &c, double rho, const ovl_zolo &z, const void *in, void *out, int nf,
               const double *eta, int prec, int maxiter, ovl_stats *st)
{
    if (prec == OVL_F64)
        sign_t<double2>(c, rho, z, in, out, nf, eta, prec, maxiter, st);
    else if (prec == OVL_F32)
        sign_t<float4>(c, rho, z, in, out, nf, eta, prec, maxiter, st);
    else
        sign_t<h8>(c, rho, z, in, out, nf, eta, prec, maxiter, st);
}

void shifts_mscg(Context &c, double rho, const ovl_zolo &z, const void *in, void *xs, int nf, const double *eta,
                 int prec, int maxiter, ovl_stats *st)
{
    OVL_REQUIRE(xs != nullptr, OVL_ERR_ARG, "no output for the shifted solutions");
    if (prec == OVL_F64)
        sign_t<double2>(c, rho, z, in, nullptr, nf, eta, prec, maxiter, st, xs);
    else if (prec == OVL_F32)
        sign_t<float4>(c, rho, z, in, nullptr, nf, eta, prec, maxiter, st, xs);
    else
        throw Error{OVL_ERR_UNSUPPORTED, "shifted solutions are kept in FP64 or FP32 only"};
}

void sign_mscg(Context &c, double rho, const ovl_zolo &z, const void *in, void *out, int nf,
               double eta, int prec, int maxiter, ovl_stats *st)
{
    OVL_REQUIRE(eta > 0.0, OVL_ERR_ARG, "eta must be positive");
    std::vector<double> e(nf, eta);
    sign_mscg(c, rho, z, in, out, nf, e.data(), prec, maxiter, st);
}

}  // namespace ovl
