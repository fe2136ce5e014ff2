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

#include <cstring>
#include <initializer_list>
#include <string>

#include "context.h"
#include "fields.h"
#include "kernels.h"
#include "mscg_state.h"
#include "ops.h"

namespace ovl {


struct MscgFinal {
    int iters, breakdown, act_total, pad;
};

// Host memory the device writes (pinned, mapped): each field's final counts
// and then its stop flag, once, when the field stops, so that polling needs no
// copy commands in the stream.  The host presets the flags to "running"
// before a call; every device store there is followed by a system-scope
// fence.  Data flows only device -> host here: the accuracies travel as a
// kernel argument and the constants by an ordinary copy.
constexpr int MS_MAXF = 64;   // fields of one multi-shift solve
struct MscgPinned {
    int stop[MS_MAXF];
    MscgFinal fin[MS_MAXF];
};
struct MscgEta {
    double e2[MS_MAXF];   // eta_f^2 (0: skip field f)
};

__global__ void k_mscg_init(MscgScal *S, int *stop, const double *partial, int nblk, MscgConst k,
                            MscgEta eta2, int *stop_h, MscgFinal *fin_h)
{
    __shared__ double lds[4];
    const int f = blockIdx.x;
    const double b2 = block_allsum(partial + (int64_t)f * nblk, nblk, lds);
    if (threadIdx.x != 0) return;
    MscgScal &s = S[f];   // parity 0
    s.rr = b2;
    // the freezing test uses eta_f^2 ||b||^2; eta_f <= 0 marks a field to skip
    const double e2 = eta2.e2[f];
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
    const int st0 = (b2 > 0.0 && e2 > 0.0) ? 0x7fffffff : 0;
    stop[f] = st0;
    if (st0 == 0) {   // nothing to iterate: report the field stopped (the host preset "running")
        fin_h[f] = MscgFinal{0, 0, 0, 0};
        __threadfence_system();
        stop_h[f] = 0;
        __threadfence_system();   // the stores are complete before the kernel is
    }
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

// One multi-shift CG step after the two stencils of the iteration:
//   alpha = (r, r) / (p, w)      (p, w) from the stencil's tile partials;
//                                (r, r) exact, from the previous step's blocks
//   r' = r - alpha w             in place; exact ||r'||^2 per block for the next step
//   beta = ||r'||^2 / (r, r)     with ||r'||^2 = (r, r) - 2 alpha Re (r, w)
//                                + alpha^2 (w, w) (the stencil's other partials),
//                                so that no step waits on a grid-wide sum of r'
//   y += sum_l omega_l alpha_l p_l ; p_l = zeta_l' r' + beta_l p_l (active shifts)
// On the first step every p_l is the source and y starts at zero.  With ALL,
// y holds one solution per shift, shift-major like p, and x_l += omega_l
// alpha_l p_l (the caller passes omega_l = 1).  Every block derives the
// step's scalars from the same partial sums in the same order; block 0
// stores the next state.
template <typename ST, bool ALL>
__global__ __launch_bounds__(256) void k_mscg_shift(const ST *__restrict__ src, const ST *__restrict__ rin,
                                                    ST *__restrict__ r, const ST *__restrict__ w,
                                                    ST *__restrict__ y, ST *__restrict__ p, MscgScal *S,
                                                    const MscgConst *kc, int *stop, MscgFinal *fin,
                                                    const int *itb, int itj, int64_t V, const double *part,
                                                    int pw_n, double *rr_part, int rr_n, int *stop_h,
                                                    MscgFinal *fin_h)
{
    using R = typename Planes<ST>::R;
    const int f = blockIdx.y;
    const int it = itb ? *itb + itj : itj;   // the iteration (device base for graph replays)
    if (it >= stop[f]) return;
    const int nf = gridDim.y;
    // exact ||r||^2 partials by iteration parity: read this step's, write the next's
    const double *rr_in = rr_part + (size_t)(it & 1) * rr_n * nf;
    double *rr_out = rr_part + (size_t)((it + 1) & 1) * rr_n * nf;
    __shared__ double lds[4];
    __shared__ double s_cy[NZMAX], s_zn[NZMAX], s_bl[NZMAX];
    __shared__ int s_act[NZMAX];
    __shared__ int s_keep_any;
    const MscgScal &sc = S[(it & 1) * nf + f];
    const int64_t fo = f * fstride<ST>(V);
    const int64_t s0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    // The first site's r and w do not depend on the step's scalars: their
    // loads go out before the sums of partials, and arrive during them.
    SpStored<ST> r_first, w_first;
    if (s0 < V) {
        ld_sp_stored((it == 0 ? src : rin) + fo, V, s0, r_first);
        ld_sp_stored(w + fo, V, s0, w_first);
    }
    // The four sums of partials.  Each thread adds its terms in index order;
    // the loads of PB consecutive terms of each sum are issued together (an
    // index past the end reads the last entry, and adds nothing).
    const double *pf = part + (int64_t)f * 3 * pw_n;
    const double *rf = rr_in + (int64_t)f * rr_n;
    double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
    const int nmax = pw_n > rr_n ? pw_n : rr_n;
    constexpr int PB = 8;
    for (int i0 = threadIdx.x; i0 < nmax; i0 += PB * blockDim.x) {
        double a0[PB], a1[PB], a2[PB], a3[PB];
#pragma unroll
        for (int q = 0; q < PB; ++q) {
            const int i = i0 + q * (int)blockDim.x;
            const int ip = i < pw_n ? i : pw_n - 1, ir = i < rr_n ? i : rr_n - 1;
            a0[q] = pf[ip];
            a1[q] = pf[pw_n + ip];
            a2[q] = pf[2 * pw_n + ip];
            a3[q] = rf[ir];
        }
#pragma unroll
        for (int q = 0; q < PB; ++q) {
            const int i = i0 + q * (int)blockDim.x;
            if (i < pw_n) {
                v0 += a0[q];
                v1 += a1[q];
                v2 += a2[q];
            }
            if (it != 0 && i < rr_n) v3 += a3[q];
        }
    }
    double vv[4] = {v0, v1, v2, v3}, tot[4];
    block_bcast_sum4(vv, tot);
    const double pw = tot[0], rw = tot[1], ww = tot[2];
    const double rr = it == 0 ? sc.rr : tot[3];
    const double alpha = rr / pw;
    const double rr_new = fmax(0.0, rr - 2.0 * alpha * rw + alpha * alpha * ww);
    const bool ok = pw > 0.0 && isfinite(alpha) && isfinite(rr_new);
    const double beta = rr_new / rr;
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
        const MscgFinal fv{nx.iters, nx.breakdown, nx.act_total, 0};
        fin[f] = fv;
        if (!s_keep_any || nx.breakdown || nx.iters >= kc->maxiter) {
            // host memory is written once per field and call, when it stops;
            // the counts reach the host before the flag
            fin_h[f] = fv;
            __threadfence_system();
            stop[f] = it + 1;
            stop_h[f] = it + 1;
            __threadfence_system();   // complete before the kernel is
        }
    }
    if (!ok) return;
    const int64_t pstride = nf * fstride<ST>(V);   // shift-major: p[l][f]
    const R ar = (R)alpha;
    double rn = 0.0;
    // one site, from its loaded r and w
    auto site = [&](int64_t s, cplx<R> (&rv)[12], cplx<R> (&pv)[12]) {
        cplx<R> yv[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) rv[c] = rv[c] - ar * pv[c];
        st_sp(r + fo, V, s, rv);
        as_stored(r, rv, 12);   // continue with r' as stored
#pragma unroll
        for (int c = 0; c < 12; ++c) rn += (double)rv[c].re * (double)rv[c].re + (double)rv[c].im * (double)rv[c].im;
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
    };
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    if (s0 < V) {
        cplx<R> rv[12], pv[12];
        sp_values(r_first, rv);
        sp_values(w_first, pv);
        site(s0, rv, pv);
    }
    for (int64_t s = s0 + step; s < V; s += step) {
        cplx<R> rv[12], pv[12];
        ld_sp((it == 0 ? src : rin) + fo, V, s, rv);
        ld_sp(w + fo, V, s, pv);
        site(s, rv, pv);
    }
    const double t = block_sum<256>(rn, lds);
    if (threadIdx.x == 0) rr_out[(int64_t)f * gridDim.x + blockIdx.x] = t;
}

// Iteration base of graph replays: set, then advanced after each chunk.
__global__ void k_set_it(int *itb, int v)
{
    if (threadIdx.x == 0) *itb = v;
}
__global__ void k_advance(int *itb, int n)
{
    if (threadIdx.x == 0) *itb += n;
}

// ---- low-mode projection (basis [n] packed fields and the fields in the
// storage type ST of the call; sums in FP64)
template <typename ST>
__global__ __launch_bounds__(256) void k_low_dots(const ST *__restrict__ basis, int n,
                                                  const ST *__restrict__ x, int64_t V, double *partial)
{
    using R = typename Planes<ST>::R;
    constexpr int NB = 8;   // basis vectors per pass: their loads are issued together
    const int f = blockIdx.y;
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    __shared__ double lds[2 * NB][4];   // [value][wave]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    cplx<R> xv[12];
    if (s < V) ld_sp(x + f * fstride<ST>(V), V, s, xv);
    for (int j0 = 0; j0 < n; j0 += NB) {
        double d[2 * NB];
#pragma unroll
        for (int q = 0; q < 2 * NB; ++q) d[q] = 0.0;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
            const int j = j0 + q;
            if (s < V && j < n) {
                cplx<R> b[12];
                ld_sp(basis + (int64_t)j * fstride<ST>(V), V, s, b);
                double dr = 0.0, di = 0.0;
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    const double xr = xv[c].re, xi = xv[c].im, br = b[c].re, bi = b[c].im;
                    dr += br * xr + bi * xi;
                    di += br * xi - bi * xr;
                }
                d[2 * q] = dr;
                d[2 * q + 1] = di;
            }
        }
        // block sums of the 2 NB values (fixed order, one LDS pass)
#pragma unroll
        for (int q = 0; q < 2 * NB; ++q)
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) d[q] += __shfl_xor(d[q], off, 64);
        __syncthreads();   // the previous pass has read lds
        if (lane == 0)
#pragma unroll
            for (int q = 0; q < 2 * NB; ++q) lds[q][wave] = d[q];
        __syncthreads();
        const int q = threadIdx.x;
        if (q < 2 * NB && j0 + q / 2 < n) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < 4; ++w) t += lds[q][w];
            const int j = j0 + q / 2;
            partial[(((int64_t)f * n + j) * 2 + (q & 1)) * gridDim.x + blockIdx.x] = t;
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
__global__ __launch_bounds__(256) void k_low_project(const ST *__restrict__ basis, int n,
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
        cplx<R> b[12];
        ld_sp(basis + (int64_t)j * fstride<ST>(V), V, s, b);
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            const cplx<double> t = cj * cplx<double>{(double)b[c].re, (double)b[c].im};
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
// The graph of one chunk of multi-shift iterations (kernel nodes in launch
// order, then the advance of the iteration base), recorded once per launch
// configuration: buffers, constants that are passed by value, the stencil
// launch variants and the field count.  record(j) issues iteration j of the
// chunk through launch_k().
template <typename F>
static hipGraphExec_t chunk_graph(Context &c, int prec, int nf, bool all, int chunk, int *itb, F record,
                                  std::initializer_list<const void *> ptrs, std::initializer_list<double> vals)
{
    std::string key;
    auto put = [&](const void *d, size_t n) { key.append(reinterpret_cast<const char *>(d), n); };
    const int head[6] = {prec, nf, all ? 1 : 0, chunk, stencil_variant(c, EPI_K, prec, nf),
                         stencil_variant(c, EPI_K2DOT, prec, nf)};
    put(head, sizeof(head));
    for (const void *q : ptrs) put(&q, sizeof(q));
    for (double v : vals) put(&v, sizeof(v));
    put(&itb, sizeof(itb));
    auto found = c.graphs.find(key);
    if (found != c.graphs.end()) return found->second;
    GraphRec gr;
    OVL_HIP(hipGraphCreate(&gr.g, 0));
    c.rec = &gr;
    try {
        for (int j = 0; j < chunk; ++j) record(j);
        launch_k(c, nullptr, k_advance, dim3(1), dim3(64), 0, itb, chunk);
    } catch (...) {
        c.rec = nullptr;
        hipGraphDestroy(gr.g);
        throw;
    }
    c.rec = nullptr;
    hipGraphExec_t exec = nullptr;
    const hipError_t e = hipGraphInstantiate(&exec, gr.g, nullptr, nullptr, 0);
    hipGraphDestroy(gr.g);
    OVL_HIP(e);
    c.graphs[key] = exec;
    return exec;
}

// out = sign(K) in, or (xs != nullptr) every shifted solution
// xs[l][f] = (K^2 + sigma_l)^{-1} in_f, each to |zeta_l| ||r|| <= eta_f ||in_f||,
// with no low-mode split and no final K.
//
// The update kernel's grid is the number of its blocks resident on the device
// at once: it strides over the sites, and a larger grid would leave a partial
// second round of blocks running after the first.
template <typename ST, bool ALL>
static unsigned upd_blocks(Context &c, int prec)
{
    int &n = c.upd_per_cu[prec][ALL ? 1 : 0];
    if (n == 0) {
        int b = 0;
        OVL_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_mscg_shift<ST, ALL>, 256, 0));
        n = b > 0 ? b : 1;
    }
    return (unsigned)(n * c.num_cu);
}

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
    const unsigned nupd = std::min<unsigned>(all ? upd_blocks<ST, true>(c, prec) : upd_blocks<ST, false>(c, prec), nblk);
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
    double *part = (double *)c.buf("ms_part", sizeof(double) * (size_t)std::max(3 * nblk_max, nblk * 2 * nl) * nf);
    double *rr_part = (double *)c.buf("ms_part2", sizeof(double) * 2 * (size_t)nupd * nf);   // by step parity
    double *coef = (double *)c.buf("ms_coef", sizeof(double) * (size_t)nf * 2 * nl);
    MscgScal *S = (MscgScal *)c.buf("ms_scal", sizeof(MscgScal) * 2 * nf);
    MscgFinal *fin = (MscgFinal *)c.buf("ms_fin", sizeof(MscgFinal) * nf);
    int *stop = (int *)c.buf("ms_stop", sizeof(int) * nf);
    MscgConst *kdev = (MscgConst *)c.buf("ms_const", sizeof(MscgConst));

    // pinned staging: constants, accuracies, and two slots of polled flags
    OVL_REQUIRE(nf <= MS_MAXF, OVL_ERR_ARG, "too many fields in one multi-shift solve");
    if (!c.ms_pin) {
        OVL_HIP(hipHostMalloc(&c.ms_pin, sizeof(MscgPinned), hipHostMallocMapped | hipHostMallocCoherent));
        std::memset(c.ms_pin, 0, sizeof(MscgPinned));
        for (auto &e : c.ms_ev) OVL_HIP(hipEventCreate(&e));
    }
    volatile MscgPinned &hp = *(volatile MscgPinned *)c.ms_pin;
    MscgPinned *hpd = nullptr;   // the same memory, as the device addresses it
    OVL_HIP(hipHostGetDevicePointer((void **)&hpd, c.ms_pin, 0));

    // 1. low-mode split: src = (1 - P) in, ex = sum sign(lambda) P in, with the
    //    basis stored like the fields (its rounding is that of the call)
    const bool low = c.n_low > 0 && !all;
    if (low) {
        const ST *basis = (const ST *)c.low_basis(prec);
        const double *sgn = c.low_signs();
        k_low_dots<ST><<<grid, 256, 0, c.stream>>>(basis, c.n_low, (const ST *)in, V, part);
        k_reduce_rows<<<nf * c.n_low * 2, 256, 0, c.stream>>>(part, nblk, coef);
        k_low_project<ST><<<grid, 256, 0, c.stream>>>(basis, c.n_low, coef, sgn, (const ST *)in, src, ex, V);
    } else {
        OVL_HIP(hipMemcpyAsync(src, in, FB * nf, hipMemcpyDeviceToDevice, c.stream));
    }
    OVL_HIP(hipGetLastError());

    // 2. constants (uploaded when they change) and initial state
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
    const char *kb = reinterpret_cast<const char *>(&k);
    if (c.ms_const_last.size() != sizeof(k) || std::memcmp(c.ms_const_last.data(), kb, sizeof(k)) != 0) {
        // from pageable memory: the runtime stages the copy before returning
        OVL_HIP(hipMemcpyAsync(kdev, &k, sizeof(MscgConst), hipMemcpyHostToDevice, c.stream));
        c.ms_const_last.assign(kb, kb + sizeof(k));
    }
    zero_fields(c, y, all ? nf * nz : nf, prec);   // stays zero for a zero source
    k_norm2<ST><<<grid, 256, 0, c.stream>>>(src, V, part);
    MscgEta ea{};
    for (int f = 0; f < nf; ++f) {
        ea.e2[f] = eta2[f];
        hp.stop[f] = 0x7fffffff;   // "running" until a kernel writes the field's stop
    }
    k_mscg_init<<<nf, 256, 0, c.stream>>>(S, stop, part, nblk, k, ea, hpd->stop, hpd->fin);
    OVL_HIP(hipGetLastError());

    // 3. iterations; poll the stop flags every CHUNK iterations, one chunk
    //    behind, so the queue never runs dry.  The first chunk is launched
    //    directly (it also settles the stencil launch variants); later chunks
    //    replay a graph of CHUNK iterations whose kernels read the iteration
    //    from *itb, unless profiling (per-launch events) is on.
    const int CHUNK = 4;
    const size_t pst = FB * nf;   // bytes between shift vectors
    ST *pbase = (ST *)((char *)p + pst * base);
    int *itb = (int *)c.buf("ms_itb", sizeof(int));
    auto one_iter = [&](int j, const int *ib) {   // iteration *ib + j (ib null: iteration j)
        const bool zero = ib == nullptr && j == 0;
        const ST *pin = zero ? src : pbase;
        const ST *rin = zero ? src : r;
        stencil(c, EPI_K, prec, pin, t, nf, rho, 0.0, nullptr, nullptr, stop, j, nullptr, ib);
        const int ntile = stencil_k2_dot(c, prec, t, w, nf, rho, k.s0, pin, rin, part, stop, j, ib);
        PendingEvent pe;
        if (c.prof) c.prof_begin(pe, KERN_SHIFT, prec, 0.0);
        const PendingEvent *ppe = c.prof ? &pe : nullptr;
        if (all)
            launch_k(c, ppe, k_mscg_shift<ST, true>, ugrid, dim3(256), 0, src, rin, r, w, y, p, S, kdev, stop, fin,
                     ib, j, V, part, ntile, rr_part, (int)nupd, hpd->stop, hpd->fin);
        else
            launch_k(c, ppe, k_mscg_shift<ST, false>, ugrid, dim3(256), 0, src, rin, r, w, y, p, S, kdev, stop, fin,
                     ib, j, V, part, ntile, rr_part, (int)nupd, hpd->stop, hpd->fin);
        if (c.prof) c.prof_end(pe);
        OVL_HIP(hipGetLastError());
    };
    hipGraphExec_t gexec = nullptr;
    int it = 0;
    int pending = -1;
    bool done = false;
    while (!done) {
        if (it == 0 || c.prof || !c.use_graphs) {
            for (int j = 0; j < CHUNK; ++j) one_iter(it + j, nullptr);
        } else {
            if (!gexec) gexec = chunk_graph(c, prec, nf, all, CHUNK, itb, [&](int j) { one_iter(j, itb); },
                                            {src, r, t, w, y, p, S, kdev, stop, fin, part, rr_part, hpd,
                                             (const void *)(intptr_t)base, (const void *)(intptr_t)nupd},
                                            {rho, k.s0});
            if (it == CHUNK) {
                k_set_it<<<1, 64, 0, c.stream>>>(itb, it);
                OVL_HIP(hipGetLastError());
            }
            OVL_HIP(hipGraphLaunch(gexec, c.stream));
        }
        it += CHUNK;
        const int slot = (it / CHUNK) & 1;
        OVL_HIP(hipEventRecord(c.ms_ev[slot], c.stream));
        if (pending >= 0) {
            // chunk `pending` has completed, so its flags are in host memory
            // (later chunks may have written newer ones: also valid)
            c.spin_wait(c.ms_ev[pending]);
            bool every = true;
            for (int f = 0; f < nf; ++f) every = every && hp.stop[f] != 0x7fffffff;
            if (every) done = true;
        }
        pending = slot;
        if (!done && it >= maxiter + 2 * CHUNK) {   // cannot happen: the kernels stop at maxiter
            OVL_HIP(hipEventSynchronize(c.ms_ev[slot]));
            done = true;
        }
    }

    // 4. s = K y + ex
    if (all) {
    } else if (low) {
        stencil(c, EPI_KPLUS, prec, y, out, nf, rho, 0.0, ex, nullptr);
    } else {
        stencil(c, EPI_K, prec, y, out, nf, rho, 0.0, nullptr, nullptr);
    }
    OVL_HIP(hipGetLastError());

    // every field has stopped: no kernel writes these any more
    std::vector<MscgFinal> hs(nf);
    std::vector<int> hstop_final(nf);
    for (int f = 0; f < nf; ++f) {
        hstop_final[f] = hp.stop[f];
        hs[f].iters = hp.fin[f].iters;
        hs[f].breakdown = hp.fin[f].breakdown;
        hs[f].act_total = hp.fin[f].act_total;
    }
    if (c.prof) c.prof_collect();
    int64_t iters = 0, act_total = 0, launches = 0;
    bool brk = false, capped = false;
    for (int f = 0; f < nf; ++f) {
        if (hstop_final[f] == 0) continue;   // zero source: no iteration ran
        iters += hs[f].iters;
        launches = std::max<int64_t>(launches, hs[f].iters);
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
    // algorithmic bytes of the shift kernel: r, w in, r out, y in, y out and 2
    // per active shift (with every solution kept: r, w, r out, and p_l, x_l in
    // and out per active shift)
    if (c.prof) {
        c.slots[KERN_SHIFT][prec].bytes +=
            all ? (double)FB * (3.0 * iters + 4.0 * act_total) : (double)FB * (5.0 * iters + 2.0 * act_total);
        // the two stencils of each executed iteration (K, then K with the
        // shift, the dot and an extra read of p), the links read once per
        // launch however many fields it carries
        const double G = stencil_link_bytes(g, prec);
        c.slots[KERN_STENCIL][prec].bytes +=
            (double)iters * (stencil_bytes(g, prec, EPI_K) + stencil_bytes(g, prec, EPI_K2DOT) - 2.0 * G) +
            (double)launches * 2.0 * G;
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
