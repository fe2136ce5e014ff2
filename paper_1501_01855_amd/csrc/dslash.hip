// Wilson hopping stencil H and kernel K = gamma_5 [(4 - rho) - H/2]
// (paper Sec. 1, eq. 2) on gfx950, plus layout conversions.
//
// One thread per lattice site, 256 threads (four wave64) per block, one
// right-hand side per grid row.  Each thread gathers the eight neighbour
// spinors, spin-projects them to half spinors (6 complex), multiplies by the
// link (or its adjoint) and reconstructs the lower spin components, so a
// direction costs one 12-complex spinor load, one 9-complex link load and
// 2 x 3 x 3 complex multiply-adds per half spinor.  Neighbour indices are
// computed arithmetically (no index table).  Spinor and link planes are
// site-major, so consecutive lanes issue consecutive 16-byte loads.
#include <algorithm>
#include <type_traits>

#include "context.h"
#include "fields.h"
#include "kernels.h"

namespace ovl {

// ------------------------------------------------------------- layout kernels
__global__ void k_pack_f64(const double2 *__restrict__ canon, double2 *__restrict__ out, int64_t V)
{
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int f = blockIdx.y;
    if (s >= V) return;
    const double2 *src = canon + (int64_t)f * V * 12 + s * 12;
    double2 *dst = out + (int64_t)f * V * 12;
#pragma unroll
    for (int c = 0; c < 12; ++c) dst[c * V + s] = src[c];
}

__global__ void k_unpack_f64(const double2 *__restrict__ in, double2 *__restrict__ canon, int64_t V)
{
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int f = blockIdx.y;
    if (s >= V) return;
    const double2 *src = in + (int64_t)f * V * 12;
    double2 *dst = canon + (int64_t)f * V * 12 + s * 12;
#pragma unroll
    for (int c = 0; c < 12; ++c) dst[c] = src[c * V + s];
}

// packed FP64 <-> packed FP32 (per field)
__global__ void k_f64_to_f32(const double2 *__restrict__ in, float4 *__restrict__ out, int64_t V)
{
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int f = blockIdx.y;
    if (s >= V) return;
    cplx<double> v[12];
    ld_sp(in + (int64_t)f * 12 * V, V, s, v);
    cplx<float> w[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) w[c] = {(float)v[c].re, (float)v[c].im};
    st_sp(out + (int64_t)f * 6 * V, V, s, w);
}

__global__ void k_f32_to_f64(const float4 *__restrict__ in, double2 *__restrict__ out, int64_t V)
{
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int f = blockIdx.y;
    if (s >= V) return;
    cplx<float> v[12];
    ld_sp(in + (int64_t)f * 6 * V, V, s, v);
    cplx<double> w[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) w[c] = {(double)v[c].re, (double)v[c].im};
    st_sp(out + (int64_t)f * 12 * V, V, s, w);
}

__global__ void k_pack_gauge(const double2 *__restrict__ canon, double2 *__restrict__ U64,
                             float2 *__restrict__ U32, __half2 *__restrict__ U16, int64_t V, int64_t Pu)
{
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= V) return;
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const double2 u = canon[s * 36 + mu * 9 + k];
            U64[(mu * 9 + k) * Pu + s] = u;
            U32[(mu * 9 + k) * Pu + s] = make_float2((float)u.x, (float)u.y);
            U16[(mu * 9 + k) * Pu + s] = __floats2half2_rn((float)u.x, (float)u.y);
        }
}

// packed FP64 <-> packed FP16 with per-site scale
__global__ void k_f64_to_h8(const double2 *__restrict__ in, h8 *__restrict__ out, int64_t V)
{
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int f = blockIdx.y;
    if (s >= V) return;
    cplx<double> v[12];
    ld_sp(in + (int64_t)f * 12 * V, V, s, v);
    cplx<float> w[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) w[c] = {(float)v[c].re, (float)v[c].im};
    st_sp(out + f * fstride<h8>(V), V, s, w);
}

__global__ void k_h8_to_f64(const h8 *__restrict__ in, double2 *__restrict__ out, int64_t V)
{
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int f = blockIdx.y;
    if (s >= V) return;
    cplx<float> v[12];
    ld_sp(in + f * fstride<h8>(V), V, s, v);
    cplx<double> w[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) w[c] = {(double)v[c].re, (double)v[c].im};
    st_sp(out + (int64_t)f * 12 * V, V, s, w);
}

void pack_spinor(Context &c, const double *canon, void *packed, int nf, int prec)
{
    const Geom &g = c.g;
    dim3 grid(site_blocks(g), nf);
    if (prec == OVL_F64) {
        k_pack_f64<<<grid, 256, 0, c.stream>>>((const double2 *)canon, (double2 *)packed, g.V);
    } else if (prec == OVL_F32) {
        double2 *tmp = (double2 *)c.buf("pack_tmp", field_bytes(g, OVL_F64) * nf);
        k_pack_f64<<<grid, 256, 0, c.stream>>>((const double2 *)canon, tmp, g.V);
        k_f64_to_f32<<<grid, 256, 0, c.stream>>>(tmp, (float4 *)packed, g.V);
    } else {
        double2 *tmp = (double2 *)c.buf("pack_tmp", field_bytes(g, OVL_F64) * nf);
        k_pack_f64<<<grid, 256, 0, c.stream>>>((const double2 *)canon, tmp, g.V);
        k_f64_to_h8<<<grid, 256, 0, c.stream>>>(tmp, (h8 *)packed, g.V);
    }
    OVL_HIP(hipGetLastError());
}

void unpack_spinor(Context &c, const void *packed, double *canon, int nf, int prec)
{
    const Geom &g = c.g;
    dim3 grid(site_blocks(g), nf);
    if (prec == OVL_F64) {
        k_unpack_f64<<<grid, 256, 0, c.stream>>>((const double2 *)packed, (double2 *)canon, g.V);
    } else if (prec == OVL_F32) {
        double2 *tmp = (double2 *)c.buf("pack_tmp", field_bytes(g, OVL_F64) * nf);
        k_f32_to_f64<<<grid, 256, 0, c.stream>>>((const float4 *)packed, tmp, g.V);
        k_unpack_f64<<<grid, 256, 0, c.stream>>>(tmp, (double2 *)canon, g.V);
    } else {
        double2 *tmp = (double2 *)c.buf("pack_tmp", field_bytes(g, OVL_F64) * nf);
        k_h8_to_f64<<<grid, 256, 0, c.stream>>>((const h8 *)packed, tmp, g.V);
        k_unpack_f64<<<grid, 256, 0, c.stream>>>(tmp, (double2 *)canon, g.V);
    }
    OVL_HIP(hipGetLastError());
}

void convert_spinor(Context &c, const void *src, int sprec, void *dst, int dprec, int nf)
{
    const Geom &g = c.g;
    dim3 grid(site_blocks(g), nf);
    if (sprec == dprec) {
        OVL_HIP(hipMemcpyAsync(dst, src, field_bytes(g, sprec) * nf, hipMemcpyDeviceToDevice, c.stream));
    } else if (sprec == OVL_F64 && dprec == OVL_F32) {
        k_f64_to_f32<<<grid, 256, 0, c.stream>>>((const double2 *)src, (float4 *)dst, g.V);
    } else if (sprec == OVL_F32 && dprec == OVL_F64) {
        k_f32_to_f64<<<grid, 256, 0, c.stream>>>((const float4 *)src, (double2 *)dst, g.V);
    } else if (sprec == OVL_F64 && dprec == OVL_HALF) {
        k_f64_to_h8<<<grid, 256, 0, c.stream>>>((const double2 *)src, (h8 *)dst, g.V);
    } else if (sprec == OVL_HALF && dprec == OVL_F64) {
        k_h8_to_f64<<<grid, 256, 0, c.stream>>>((const h8 *)src, (double2 *)dst, g.V);
    } else {
        throw Error{OVL_ERR_UNSUPPORTED, "convert_spinor: precision pair"};
    }
    OVL_HIP(hipGetLastError());
}

void pack_gauge(Context &c, const double *canon)
{
    const Geom &g = c.g;
    if (!c.U64) {
        OVL_HIP(hipMalloc(&c.U64, (size_t)g.Pu * 36 * sizeof(double2)));
        OVL_HIP(hipMalloc(&c.U32, (size_t)g.Pu * 36 * sizeof(float2)));
        OVL_HIP(hipMalloc(&c.U16, (size_t)g.Pu * 36 * sizeof(__half2)));
        c.bytes_held += (int64_t)g.Pu * 36 * (16 + 8 + 4);
    }
    k_pack_gauge<<<site_blocks(g), 256, 0, c.stream>>>((const double2 *)canon, c.U64, c.U32, (__half2 *)c.U16,
                                                       g.V, g.Pu);
    OVL_HIP(hipGetLastError());
    c.have_gauge = true;
}

// ------------------------------------------------------------- stencil kernel
// TPS threads per site: with TPS = 2 a block covers 128 sites; waves 0-1
// gather directions {x, y} and waves 2-3 directions {z, t} for the same sites
// (no divergence inside a wave), exchange half accumulators through LDS, and
// each thread finishes and stores half of the output spinor -- twice the
// threads for small lattices.
template <int MU, typename R, typename ST, typename GT>
__device__ __forceinline__ void gather_dir(const ST *__restrict__ in, const GT *__restrict__ U, int64_t V, int64_t Pu,
                                           int64_t s,
                                           int32_t c, int32_t Lm, int64_t st, cplx<R> acc[12])
{
    cplx<R> psi[12];
    cplx<R> u[9];
    const int64_t fwd = (c == Lm - 1) ? s - (int64_t)(Lm - 1) * st : s + st;
    const int64_t bwd = (c == 0) ? s + (int64_t)(Lm - 1) * st : s - st;
    ld_sp(in, V, fwd, psi);
    ld_link(U, Pu, MU, s, u);
    hop_term<MU, true>(psi, u, acc);
    ld_sp(in, V, bwd, psi);
    ld_link(U, Pu, MU, bwd, u);
    hop_term<MU, false>(psi, u, acc);
}

// Directions MU0..MU1.  Four directions run as a non-unrolled loop (bounded
// register use); two are unrolled.
template <int MU0, int MU1, typename R, typename ST, typename GT>
__device__ __forceinline__ void gather(const ST *__restrict__ in, const GT *__restrict__ U, int64_t V, int64_t Pu,
                                       int64_t s,
                                       const int32_t co[4], const int32_t Ls[4], const int64_t st[4],
                                       cplx<R> acc[12])
{
    if constexpr (MU1 - MU0 == 1) {
        gather_dir<MU0, R>(in, U, V, Pu, s, co[MU0], Ls[MU0], st[MU0], acc);
        gather_dir<MU1, R>(in, U, V, Pu, s, co[MU1], Ls[MU1], st[MU1], acc);
    } else {
        cplx<R> psi[12];
        cplx<R> u[9];
#pragma unroll 1
        for (int mu = MU0; mu <= MU1; ++mu) {
            const int32_t c = co[mu], Lm = Ls[mu];
            const int64_t fwd = (c == Lm - 1) ? s - (int64_t)(Lm - 1) * st[mu] : s + st[mu];
            const int64_t bwd = (c == 0) ? s + (int64_t)(Lm - 1) * st[mu] : s - st[mu];
            ld_sp(in, V, fwd, psi);
            ld_link(U, Pu, mu, s, u);
            switch (mu) {
            case 0: hop_term<0, true>(psi, u, acc); break;
            case 1: hop_term<1, true>(psi, u, acc); break;
            case 2: hop_term<2, true>(psi, u, acc); break;
            default: hop_term<3, true>(psi, u, acc); break;
            }
            ld_sp(in, V, bwd, psi);
            ld_link(U, Pu, mu, bwd, u);
            switch (mu) {
            case 0: hop_term<0, false>(psi, u, acc); break;
            case 1: hop_term<1, false>(psi, u, acc); break;
            case 2: hop_term<2, false>(psi, u, acc); break;
            default: hop_term<3, false>(psi, u, acc); break;
            }
        }
    }
}

// Site traversal orders (MAP):
//  MAP_LEX    block b takes sites [b n, (b + 1) n) in lexicographic order;
//  MAP_REMAP  the same tiles, but each XCD (blocks are handed to the eight
//             XCDs round-robin) receives a contiguous range of them;
//  MAP_COL    each XCD owns one of eight xyz columns (Geom::cb) and walks it
//             through t, a column slice at a time, so that the t- and
//             z-neighbours of a slice are fetched by the same XCD shortly
//             before or after and meet in its L2.
// Fields run fastest within a tile (the fields of one tile share its links).
enum { MAP_LEX = 0, MAP_REMAP = 1, MAP_COL = 2 };

template <int MAP, int TPS>
__device__ __forceinline__ void site_of_thread(const Geom &g, unsigned &tile, unsigned &f, int64_t &s, int32_t co[4],
                                               bool &valid)
{
    constexpr int SPB = 256 / TPS;   // sites per block
    const int lane = TPS == 2 ? (int)(threadIdx.x & 127) : (int)threadIdx.x;
    if constexpr (MAP == MAP_COL) {
        const unsigned X = gridDim.x, Y = gridDim.y;
        const unsigned lin = blockIdx.y * X + blockIdx.x;
        const unsigned col = lin % 8, k = lin / 8;
        f = k % Y;
        const unsigned rest = k / Y;              // [0, Lt tps)
        const unsigned per_col = X / 8;           // Lt tps
        tile = col * per_col + rest;
        const unsigned tps = per_col / (unsigned)g.L[3];
        const int32_t t = (int32_t)(rest / tps);
        const int32_t local = (int32_t)(rest % tps) * SPB + lane;
        valid = local < g.col_sites;
        const int32_t cx = (int32_t)col % g.cn[0], cy = ((int32_t)col / g.cn[0]) % g.cn[1],
                      cz = (int32_t)col / (g.cn[0] * g.cn[1]);
        co[0] = cx * g.cb[0] + local % g.cb[0];
        co[1] = cy * g.cb[1] + (local / g.cb[0]) % g.cb[1];
        co[2] = cz * g.cb[2] + local / (g.cb[0] * g.cb[1]);
        co[3] = t;
        s = co[0] + (int64_t)g.L[0] * (co[1] + (int64_t)g.L[1] * (co[2] + (int64_t)g.L[2] * co[3]));
    } else {
        tile_of_block<MAP == MAP_REMAP>(tile, f);
        s = (int64_t)tile * SPB + lane;
        valid = s < g.V;
        const int32_t si = valid ? (int32_t)s : 0;
        co[0] = si % g.L[0];
        int32_t rem = si / g.L[0];
        co[1] = rem % g.L[1];
        rem /= g.L[1];
        co[2] = rem % g.L[2];
        co[3] = rem / g.L[2];
    }
}

// With two lanes per site: half h keeps components [6h, 6h+6) of the sum and
// receives the partner's (own half in acc[0..6) afterwards).  Every thread of
// the block must call it.  REUSE: another exchange follows in the same kernel
// (wait until every partner has read).
template <bool REUSE, typename R>
__device__ __forceinline__ void exchange_halves(cplx<R> acc[12], int half)
{
    __shared__ cplx<R> xch[2][6][128];
    const int lane = threadIdx.x & 127;
    const bool hi = half != 0;   // wave-uniform
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        xch[half][c][lane].re = hi ? acc[c].re : acc[6 + c].re;
        xch[half][c][lane].im = hi ? acc[c].im : acc[6 + c].im;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const R mr = hi ? acc[6 + c].re : acc[c].re;
        const R mi = hi ? acc[6 + c].im : acc[c].im;
        const cplx<R> o = xch[1 - half][c][lane];
        acc[c] = {mr + o.re, mi + o.im};
    }
    if constexpr (REUSE) __syncthreads();
}

// Finish site s from the hopping sum acc (this lane's NC components) and store
// it; K2DOT adds its three dot products to part[0..3).
template <typename ST, int EPI, int TPS, typename R>
__device__ __forceinline__ void stencil_epilogue(const StencilArgs<ST> &a, unsigned f, int64_t s, int half,
                                                 const cplx<R> *acc, double part[3])
{
    constexpr int NC = 12 / TPS;
    const int64_t V = a.g.V;
    const ST *in = a.in + f * fstride<ST>(V);
    cplx<R> o[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) o[c] = acc[c];
    ST *out = a.out + f * fstride<ST>(V);
    if constexpr (EPI == EPI_HOP) {
        if constexpr (TPS == 1) st_sp(out, V, s, o); else st_sp_half(out, V, s, half, o);
    } else {
        // D_W psi = (4 - rho) psi - H psi / 2, then gamma_5 (negate spins 2, 3)
        cplx<R> x[NC];
        if constexpr (TPS == 1) ld_sp(in, V, s, x); else ld_sp_half(in, V, s, half, x);
        const R m = (R)a.diag, hh = (R)0.5;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int cg = TPS == 1 ? c : 6 * half + c;
            const cplx<R> d = m * x[c] - hh * o[c];
            o[c] = (cg < 6) ? d : -d;
        }
        if constexpr (EPI == EPI_K2DOT || EPI == EPI_KPLUS) {
            const ST *aux = a.aux + f * fstride<ST>(V);
            if constexpr (TPS == 1) ld_sp(aux, V, s, x); else ld_sp_half(aux, V, s, half, x);
            if constexpr (EPI == EPI_K2DOT) {
                // w = K t + sigma p ; partials (p, w), Re (r, w), (w, w) of w as stored
                const R sg = (R)a.sigma;
#pragma unroll
                for (int c = 0; c < NC; ++c) o[c] = o[c] + sg * x[c];
                cplx<R> ws[NC], rv[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) ws[c] = o[c];
                as_stored(a.out, ws, NC);
                const ST *aux2 = a.aux2 + f * fstride<ST>(V);
                if constexpr (TPS == 1) ld_sp(aux2, V, s, rv); else ld_sp_half(aux2, V, s, half, rv);
                double d0 = 0.0, d1 = 0.0, d2 = 0.0;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const double wr = ws[c].re, wi = ws[c].im;
                    d0 += (double)x[c].re * wr + (double)x[c].im * wi;
                    d1 += (double)rv[c].re * wr + (double)rv[c].im * wi;
                    d2 += wr * wr + wi * wi;
                }
                part[0] += d0;
                part[1] += d1;
                part[2] += d2;
            } else {
#pragma unroll
                for (int c = 0; c < NC; ++c) o[c] = o[c] + x[c];
            }
        }
        if constexpr (TPS == 1) st_sp(out, V, s, o); else st_sp_half(out, V, s, half, o);
    }
}

// K2DOT: one partial of each dot per (field, tile).  Every thread of the block
// must call it.
template <typename ST, int EPI>
__device__ __forceinline__ void store_partials(const StencilArgs<ST> &a, unsigned f, unsigned tile,
                                               const double part[3])
{
    if constexpr (EPI == EPI_K2DOT) {
        __shared__ double lds[4];
        const double t0 = block_sum<256>(part[0], lds);
        const double t1 = block_sum<256>(part[1], lds);
        const double t2 = block_sum<256>(part[2], lds);
        if (threadIdx.x == 0) {
            double *pp = a.partial + (int64_t)f * 3 * gridDim.x + tile;
            pp[0] = t0;
            pp[gridDim.x] = t1;
            pp[2 * gridDim.x] = t2;
        }
    }
}

template <typename ST, typename GT, int EPI, int TPS, int MAP>
__global__ __launch_bounds__(256) void k_stencil(StencilArgs<ST> a, const GT *__restrict__ U)
{
    using R = typename Planes<ST>::R;
    unsigned tile, f;
    int64_t s;
    int32_t co[4];
    bool valid;
    site_of_thread<MAP, TPS>(a.g, tile, f, s, co, valid);
    const int it = a.itb ? *a.itb + a.it : a.it;
    if (a.stop != nullptr && it >= a.stop[f]) return;   // field already converged
    const int64_t V = a.g.V;
    const int half = TPS == 2 ? (int)(threadIdx.x >> 7) : 0;
    const ST *in = a.in + f * fstride<ST>(V);
    double part[3] = {0.0, 0.0, 0.0};
    cplx<R> acc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = {R(0), R(0)};
    if (valid) {
        const int32_t Ls[4] = {a.g.L[0], a.g.L[1], a.g.L[2], a.g.L[3]};
        const int64_t st[4] = {a.g.stride[0], a.g.stride[1], a.g.stride[2], a.g.stride[3]};
        if constexpr (TPS == 1) {
            gather<0, 3, R>(in, U, V, a.g.Pu, s, co, Ls, st, acc);
        } else {
            if (half == 0)
                gather<0, 1, R>(in, U, V, a.g.Pu, s, co, Ls, st, acc);
            else
                gather<2, 3, R>(in, U, V, a.g.Pu, s, co, Ls, st, acc);
        }
    }
    if constexpr (TPS == 2) exchange_halves<false>(acc, half);
    if (valid) stencil_epilogue<ST, EPI, TPS>(a, f, s, half, acc, part);
    store_partials<ST, EPI>(a, f, tile, part);
}

// The same stencil with each thread walking a column of T = Lt / 8 sites in
// t, block lin taking t-chunk lin % 8 (so each XCD, blocks being handed to the
// eight XCDs round-robin, owns one chunk of t for the whole x-y-z volume and
// meets its x, y, z neighbours in its own L2).  The t hops reuse what the
// previous site of the column loaded: the projection (1 + gamma_t) psi(t) and
// the backward term U_t(t)^+ (1 + gamma_t) psi(t) for site t + 1 are carried
// in registers, so psi and U_t are read once per site along t (plus once per
// column for the chunk's first site).  With two lanes per site, half 0
// gathers x, y and half 1 z and t.
template <typename ST, typename GT, int EPI, int TPS>
__global__ __launch_bounds__(256) void k_stencil_tm(StencilArgs<ST> a, const GT *__restrict__ U)
{
    using R = typename Planes<ST>::R;
    constexpr int SPB = 256 / TPS;
    const Geom &g = a.g;
    const unsigned X = gridDim.x, Y = gridDim.y;
    const unsigned lin = blockIdx.y * X + blockIdx.x;
    const unsigned nxyz = X / 8;                  // x-y-z tiles
    const unsigned chunk = lin % 8, k = lin / 8;
    const unsigned f = k % Y, xt = k / Y;
    const unsigned tile = chunk * nxyz + xt;
    const int it = a.itb ? *a.itb + a.it : a.it;
    if (a.stop != nullptr && it >= a.stop[f]) return;
    const int64_t V = g.V, S3 = g.stride[3], Pu = g.Pu;
    const int Lt = g.L[3], T = Lt / 8, t0 = (int)chunk * T;
    const int lane = TPS == 2 ? (int)(threadIdx.x & 127) : (int)threadIdx.x;
    const int half = TPS == 2 ? (int)(threadIdx.x >> 7) : 0;
    const int64_t xyz = (int64_t)xt * SPB + lane;
    const bool valid = xyz < S3;
    int32_t co[4] = {0, 0, 0, 0};
    if (valid) {
        const int32_t q = (int32_t)xyz;
        co[0] = q % g.L[0];
        co[1] = (q / g.L[0]) % g.L[1];
        co[2] = q / (g.L[0] * g.L[1]);
    }
    const int32_t Ls[4] = {g.L[0], g.L[1], g.L[2], g.L[3]};
    const int64_t st[4] = {g.stride[0], g.stride[1], g.stride[2], g.stride[3]};
    const ST *in = a.in + f * fstride<ST>(V);
    const bool tdir = TPS == 1 || half == 1;
    cplx<R> hp[6], gb[6];   // (1 + gamma_t) psi(t), and the backward t term of site t
    if (valid && tdir) {
        const int64_t s0 = xyz + (int64_t)t0 * S3;
        const int64_t sm = t0 == 0 ? s0 + (int64_t)(Lt - 1) * S3 : s0 - S3;
        cplx<R> v[12], u[9];
        ld_sp(in, V, sm, v);
        spin_proj<3, false>(v, hp);
        ld_link(U, Pu, 3, sm, u);
        link_mul<false>(u, hp, gb);
        ld_sp(in, V, s0, v);
        spin_proj<3, false>(v, hp);
    }
    double part[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < T; ++j) {
        const int t = t0 + j;
        const int64_t s = xyz + (int64_t)t * S3;
        cplx<R> acc[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = {R(0), R(0)};
        if (valid) {
            co[3] = t;
            if constexpr (TPS == 1) {
                gather<0, 2, R>(in, U, V, Pu, s, co, Ls, st, acc);
            } else {
                if (half == 0)
                    gather<0, 1, R>(in, U, V, Pu, s, co, Ls, st, acc);
                else
                    gather_dir<2, R>(in, U, V, Pu, s, co[2], Ls[2], st[2], acc);
            }
            if (tdir) {
                const int64_t sp = t == Lt - 1 ? s - (int64_t)(Lt - 1) * S3 : s + S3;
                cplx<R> v[12], u[9], h[6], gg[6];
                ld_sp(in, V, sp, v);
                ld_link(U, Pu, 3, s, u);
                spin_proj<3, true>(v, h);
                link_mul<true>(u, h, gg);
                spin_recon<3, true>(gg, acc);    // (1 - gamma_t) U_t(t) psi(t + 1)
                spin_recon<3, false>(gb, acc);   // (1 + gamma_t) U_t(t - 1)^+ psi(t - 1)
                link_mul<false>(u, hp, gb);      // the backward term of site t + 1
                spin_proj<3, false>(v, hp);      // (1 + gamma_t) psi(t + 1)
            }
        }
        if constexpr (TPS == 2) exchange_halves<true>(acc, half);
        if (valid) stencil_epilogue<ST, EPI, TPS>(a, f, s, half, acc, part);
    }
    store_partials<ST, EPI>(a, f, tile, part);
}

// Launch shape chosen per (precision, epilogue, nf) by timing the variants on
// the context's lattice the first time that shape is used (autotuning).
// Launch variants: 0 / 1 one lane per site, MAP_LEX / MAP_REMAP; 2 / 3 two
// lanes per site, likewise; 4 / 5 MAP_COL with one / two lanes per site; 6 / 7
// the t-marching kernel with one / two lanes per site (Lt a multiple of 8).
// FP16 storage runs one lane per site (variants 0, 1, 4, 6).
static int variant_tps(int v) { return (v == 2 || v == 3 || v == 5 || v == 7) ? 2 : 1; }

unsigned stencil_tiles(const Geom &g, int v)
{
    const int tps = variant_tps(v);
    const int spb = 256 / tps;
    if (v >= 6) return 8u * (unsigned)((g.stride[3] + spb - 1) / spb);
    if (v >= 4) return 8u * (unsigned)g.L[3] * (unsigned)((g.col_sites + spb - 1) / spb);
    return (unsigned)((g.V * tps + 255) / 256);
}

bool stencil_variant_ok(const Geom &g, int prec, int v)
{
    if (v < 0 || v > 7) return false;
    if ((v == 4 || v == 5) && !g.col_ok) return false;
    if (v >= 6 && g.L[3] % 8 != 0) return false;
    if (prec == OVL_HALF) return v == 0 || v == 1 || v == 4 || v == 6;
    return true;
}

int64_t stencil_tiles_max(const Geom &g)
{
    int64_t m = 0;
    for (int v = 0; v < 8; ++v)
        if (stencil_variant_ok(g, OVL_F64, v)) m = std::max<int64_t>(m, stencil_tiles(g, v));
    return m;
}

template <typename ST, typename GT, int EPI, int TPS, int MAP>
static void launch_variant(Context &c, const StencilArgs<ST> &a, const GT *U, int nf, const PendingEvent *pe)
{
    const int v = MAP == MAP_COL ? (TPS == 2 ? 5 : 4) : (TPS == 2 ? 2 : 0) + (MAP == MAP_REMAP ? 1 : 0);
    dim3 grid(stencil_tiles(c.g, v), nf);
    launch_k(c, pe, k_stencil<ST, GT, EPI, TPS, MAP>, grid, dim3(256), 0, a, U);
}

template <typename ST, typename GT, int EPI, int TPS>
static void launch_tmarch(Context &c, const StencilArgs<ST> &a, const GT *U, int nf, const PendingEvent *pe)
{
    dim3 grid(stencil_tiles(c.g, TPS == 2 ? 7 : 6), nf);
    launch_k(c, pe, k_stencil_tm<ST, GT, EPI, TPS>, grid, dim3(256), 0, a, U);
}

template <typename ST, typename GT, int EPI>
static void launch_by_id(Context &c, int id, const StencilArgs<ST> &a, const GT *U, int nf,
                         const PendingEvent *pe = nullptr)
{
    if constexpr (std::is_same<ST, h8>::value) {   // FP16 storage: one lane per site only
        if (id == 0)
            launch_variant<ST, GT, EPI, 1, MAP_LEX>(c, a, U, nf, pe);
        else if (id == 1)
            launch_variant<ST, GT, EPI, 1, MAP_REMAP>(c, a, U, nf, pe);
        else if (id == 4)
            launch_variant<ST, GT, EPI, 1, MAP_COL>(c, a, U, nf, pe);
        else
            launch_tmarch<ST, GT, EPI, 1>(c, a, U, nf, pe);
    } else {
        switch (id) {
        case 0: launch_variant<ST, GT, EPI, 1, MAP_LEX>(c, a, U, nf, pe); break;
        case 1: launch_variant<ST, GT, EPI, 1, MAP_REMAP>(c, a, U, nf, pe); break;
        case 2: launch_variant<ST, GT, EPI, 2, MAP_LEX>(c, a, U, nf, pe); break;
        case 3: launch_variant<ST, GT, EPI, 2, MAP_REMAP>(c, a, U, nf, pe); break;
        case 4: launch_variant<ST, GT, EPI, 1, MAP_COL>(c, a, U, nf, pe); break;
        case 5: launch_variant<ST, GT, EPI, 2, MAP_COL>(c, a, U, nf, pe); break;
        case 6: launch_tmarch<ST, GT, EPI, 1>(c, a, U, nf, pe); break;
        default: launch_tmarch<ST, GT, EPI, 2>(c, a, U, nf, pe); break;
        }
    }
}

static constexpr int N_VARIANTS = 8;

template <typename ST, typename GT, int EPI>
static int tuned_variant(Context &c, const StencilArgs<ST> &a, const GT *U, int nf, int prec)
{
    const int key = (prec * 8 + EPI) * 64 + (nf < 63 ? nf : 63);
    auto it = c.tuned.find(key);
    if (it != c.tuned.end()) return it->second;
    if (c.autotune == 0) return c.tuned[key] = 1;
    // time every variant on scratch output
    StencilArgs<ST> t = a;
    t.stop = nullptr;
    t.out = (ST *)c.buf("tune_out", field_bytes(c.g, prec) * nf);
    t.partial = (double *)c.buf("tune_part", sizeof(double) * 3 * (size_t)nf * stencil_tiles_max(c.g));
    hipEvent_t e0 = c.event(), e1 = c.event();
    int best = 0;
    float best_ms = 1e30f;
    for (int v = 0; v < N_VARIANTS; ++v) {
        if (!stencil_variant_ok(c.g, prec, v)) continue;
        launch_by_id<ST, GT, EPI>(c, v, t, U, nf);   // warm-up
        OVL_HIP(hipEventRecord(e0, c.stream));
        for (int r = 0; r < 5; ++r) launch_by_id<ST, GT, EPI>(c, v, t, U, nf);
        OVL_HIP(hipEventRecord(e1, c.stream));
        OVL_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        OVL_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best_ms) {
            best_ms = ms;
            best = v;
        }
    }
    OVL_HIP(hipGetLastError());
    return c.tuned[key] = best;
}

template <typename ST, typename GT, int EPI>
static void launch_stencil_t(Context &c, const StencilArgs<ST> &a, const GT *U, int nf, int prec,
                             bool profile)
{
    const int v = tuned_variant<ST, GT, EPI>(c, a, U, nf, prec);
    PendingEvent pe;
    // launches inside the multi-shift CG (a.stop set) may skip converged
    // fields; their driver books the bytes of the work actually done
    const double bytes = a.stop ? 0.0 : stencil_bytes(c.g, prec, EPI) * nf;
    const bool prof = profile && c.prof;
    if (prof) c.prof_begin(pe, KERN_STENCIL, prec, bytes);
    launch_by_id<ST, GT, EPI>(c, v, a, U, nf, prof ? &pe : nullptr);
    OVL_HIP(hipGetLastError());
    if (prof) c.prof_end(pe);
}

void stencil(Context &c, int epi, int prec, const void *in, void *out, int nf, double rho,
             double sigma, const void *aux, double *partial, const int *stop, int it, const void *aux2,
             const int *itb)
{
    OVL_REQUIRE(c.have_gauge, OVL_ERR_STATE, "no gauge field loaded");
    if (prec == OVL_F64) {
        StencilArgs<double2> a{c.g, (const double2 *)in, (double2 *)out, (const double2 *)aux,
                               (const double2 *)aux2, 4.0 - rho, sigma, partial, stop, it, itb};
        switch (epi) {
        case EPI_HOP: launch_stencil_t<double2, double2, EPI_HOP>(c, a, c.U64, nf, prec, true); break;
        case EPI_K: launch_stencil_t<double2, double2, EPI_K>(c, a, c.U64, nf, prec, true); break;
        case EPI_K2DOT: launch_stencil_t<double2, double2, EPI_K2DOT>(c, a, c.U64, nf, prec, true); break;
        case EPI_KPLUS: launch_stencil_t<double2, double2, EPI_KPLUS>(c, a, c.U64, nf, prec, true); break;
        }
    } else if (prec == OVL_F32) {
        StencilArgs<float4> a{c.g, (const float4 *)in, (float4 *)out, (const float4 *)aux,
                              (const float4 *)aux2, 4.0 - rho, sigma, partial, stop, it, itb};
        switch (epi) {
        case EPI_HOP: launch_stencil_t<float4, float2, EPI_HOP>(c, a, c.U32, nf, prec, true); break;
        case EPI_K: launch_stencil_t<float4, float2, EPI_K>(c, a, c.U32, nf, prec, true); break;
        case EPI_K2DOT: launch_stencil_t<float4, float2, EPI_K2DOT>(c, a, c.U32, nf, prec, true); break;
        case EPI_KPLUS: launch_stencil_t<float4, float2, EPI_KPLUS>(c, a, c.U32, nf, prec, true); break;
        }
    } else {
        StencilArgs<h8> a{c.g, (const h8 *)in, (h8 *)out, (const h8 *)aux, (const h8 *)aux2, 4.0 - rho,
                          sigma, partial, stop, it, itb};
        const __half2 *U = (const __half2 *)c.U16;
        switch (epi) {
        case EPI_HOP: launch_stencil_t<h8, __half2, EPI_HOP>(c, a, U, nf, prec, true); break;
        case EPI_K: launch_stencil_t<h8, __half2, EPI_K>(c, a, U, nf, prec, true); break;
        case EPI_K2DOT: launch_stencil_t<h8, __half2, EPI_K2DOT>(c, a, U, nf, prec, true); break;
        case EPI_KPLUS: launch_stencil_t<h8, __half2, EPI_KPLUS>(c, a, U, nf, prec, true); break;
        }
    }
}

// w = K t + s0 p with (p, w) partials per tile; returns the number of tiles.
int stencil_k2_dot(Context &c, int prec, const void *t, void *w, int nf, double rho, double s0, const void *p,
                   const void *r, double *partial, const int *stop, int it, const int *itb)
{
    stencil(c, EPI_K2DOT, prec, t, w, nf, rho, s0, p, partial, stop, it, r, itb);
    const int key = (prec * 8 + EPI_K2DOT) * 64 + (nf < 63 ? nf : 63);
    const int v = c.tuned.count(key) ? c.tuned[key] : 1;
    return (int)stencil_tiles(c.g, v);
}

int stencil_variant(Context &c, int epi, int prec, int nf)
{
    const int key = (prec * 8 + epi) * 64 + (nf < 63 ? nf : 63);
    const auto it = c.tuned.find(key);
    return it == c.tuned.end() ? -1 : it->second;
}

void launch_hop(Context &c, const void *in, void *out, int nf, int prec)
{
    stencil(c, EPI_HOP, prec, in, out, nf, 0.0, 0.0, nullptr, nullptr);
}

void launch_K(Context &c, double rho, const void *in, void *out, int nf, int prec)
{
    stencil(c, EPI_K, prec, in, out, nf, rho, 0.0, nullptr, nullptr);
}

// Algorithmic HBM bytes of one stencil launch per field (perfect neighbour
// reuse, no index table): read in + links, write out, plus the extra own-site
// reads of the epilogues that take more inputs.
double stencil_bytes(const Geom &g, int prec, int epi)
{
    const double S = (double)field_bytes(g, prec);
    const double G = (double)g.V * 36 * (prec == OVL_F64 ? 16 : prec == OVL_F32 ? 8 : 4);
    double b = 2 * S + G;
    if (epi == EPI_KPLUS) b += S;
    if (epi == EPI_K2DOT) b += 2 * S;   // p and r
    return b;
}

}  // namespace ovl
