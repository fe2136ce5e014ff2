// Wilson hopping stencil H and kernel K = gamma_5 [(4 - rho) - H/2]
// (paper Sec. 1, eq. 2) on gfx950, plus layout conversions.
//
// The basic scheme: one lane per lattice site, 256 threads (four wave64) per
// block, one right-hand side per grid row.  A lane gathers the eight
// neighbour spinors, spin-projects them to half spinors (6 complex),
// multiplies by the link (or its adjoint) and reconstructs the lower spin
// components, so a direction costs one spinor load, one link load and
// 2 x 3 x 3 complex multiply-adds per half spinor.  Neighbour indices are
// computed arithmetically (no index table).  Spinor and link planes are
// site-major, so consecutive lanes issue consecutive 16-byte loads.  The
// launch variants below change who does what (two lanes per site, XCD-aware
// block orders, lanes walking time columns, LDS-shared spatial tiles); an
// autotuner picks one per precision, epilogue and field count.
#include <algorithm>
#include <cmath>
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
                             float2 *__restrict__ U32, __half2 *__restrict__ U16, float2 *__restrict__ U32r,
                             __half2 *__restrict__ U16r, int64_t V, int64_t Pu)
{
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= V) return;
    // two-row forms (the planes ld_link reads for f2r12 / h2r12): entries
    // 0..3 in the Q planes, 4 and 5 in the R plane
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double2 u = canon[s * 36 + mu * 9 + k];
            const float2 f = make_float2((float)u.x, (float)u.y);
            if (k < 4) {
                U32r[2 * ((mu * 2 + k / 2) * Pu + s) + k % 2] = f;
                U16r[4 * (mu * Pu + s) + k] = __floats2half2_rn((float)u.x, (float)u.y);
            } else {
                U32r[2 * (8 * Pu + mu * Pu + s) + (k - 4)] = f;
                U16r[4 * 4 * Pu + 2 * (mu * Pu + s) + (k - 4)] = __floats2half2_rn((float)u.x, (float)u.y);
            }
        }
    // FP32: float4 Q[4][4][Pu] then float2 R[4][Pu]; FP16: uint4 Q[4][2][Pu]
    // then uint32 R[4][Pu] (the layouts ld_link reads)
    float *Q32 = reinterpret_cast<float *>(U32);
    float2 *R32 = reinterpret_cast<float2 *>(U32 + 32 * Pu);
    __half2 *Q16 = U16;
    __half2 *R16 = U16 + 32 * Pu;
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const double2 u = canon[s * 36 + mu * 9 + k];
            U64[(mu * 9 + k) * Pu + s] = u;
            const float2 f = make_float2((float)u.x, (float)u.y);
            const __half2 h = __floats2half2_rn((float)u.x, (float)u.y);
            if (k < 8) {
                float *q = Q32 + 4 * ((mu * 4 + k / 2) * Pu + s) + 2 * (k % 2);
                q[0] = f.x;
                q[1] = f.y;
                Q16[4 * ((mu * 2 + k / 4) * Pu + s) + k % 4] = h;
            } else {
                R32[mu * Pu + s] = f;
                R16[mu * Pu + s] = h;
            }
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

void pack_spinor(Context &c, const double *canon, void *packed, int nf, int prec, double2 *tmp)
{
    const Geom &g = c.g;
    dim3 grid(site_blocks(g), nf);
    if (prec != OVL_F64 && tmp == nullptr) tmp = (double2 *)c.buf("pack_tmp", field_bytes(g, OVL_F64) * nf);
    if (prec == OVL_F64) {
        k_pack_f64<<<grid, 256, 0, c.stream>>>((const double2 *)canon, (double2 *)packed, g.V);
    } else if (prec == OVL_F32) {
        k_pack_f64<<<grid, 256, 0, c.stream>>>((const double2 *)canon, tmp, g.V);
        k_f64_to_f32<<<grid, 256, 0, c.stream>>>(tmp, (float4 *)packed, g.V);
    } else {
        k_pack_f64<<<grid, 256, 0, c.stream>>>((const double2 *)canon, tmp, g.V);
        k_f64_to_h8<<<grid, 256, 0, c.stream>>>(tmp, (h8 *)packed, g.V);
    }
    OVL_HIP(hipGetLastError());
}

void unpack_spinor(Context &c, const void *packed, double *canon, int nf, int prec, double2 *tmp)
{
    const Geom &g = c.g;
    dim3 grid(site_blocks(g), nf);
    if (prec != OVL_F64 && tmp == nullptr) tmp = (double2 *)c.buf("pack_tmp", field_bytes(g, OVL_F64) * nf);
    if (prec == OVL_F64) {
        k_unpack_f64<<<grid, 256, 0, c.stream>>>((const double2 *)packed, (double2 *)canon, g.V);
    } else if (prec == OVL_F32) {
        k_f32_to_f64<<<grid, 256, 0, c.stream>>>((const float4 *)packed, tmp, g.V);
        k_unpack_f64<<<grid, 256, 0, c.stream>>>(tmp, (double2 *)canon, g.V);
    } else {
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

// Per block: the largest |u_2b - conj(u_0 x u_1)_b| over the links of its
// sites (FP64), the test for the two-row form.
__global__ __launch_bounds__(256) void k_su3_dev(const double2 *__restrict__ canon, int64_t V,
                                                 double *__restrict__ part)
{
    __shared__ double red[256];
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double m = 0.0;
    if (s < V)
        for (int mu = 0; mu < 4; ++mu) {
            cplx<double> u[9];
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const double2 t = canon[s * 36 + mu * 9 + k];
                u[k] = {t.x, t.y};
            }
            cplx<double> w[9] = {u[0], u[1], u[2], u[3], u[4], u[5], u[6], u[7], u[8]};
            su3_third_row(w);
#pragma unroll
            for (int k = 6; k < 9; ++k) m = fmax(m, fmax(fabs(w[k].re - u[k].re), fabs(w[k].im - u[k].im)));
        }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Links whose third rows agree with the two-row rebuild to this bound use
// the two-row form in FP32 and FP16 (about the rounding of FP32 storage).
static constexpr double TWO_ROW_TOL = 0x1p-23;

void pack_gauge(Context &c, const double *canon)
{
    const Geom &g = c.g;
    if (!c.U64) {
        OVL_HIP(hipMalloc(&c.U64, (size_t)g.Pu * 36 * sizeof(double2)));
        OVL_HIP(hipMalloc(&c.U32, (size_t)g.Pu * 36 * sizeof(float2)));
        OVL_HIP(hipMalloc(&c.U16, (size_t)g.Pu * 36 * sizeof(__half2)));
        OVL_HIP(hipMalloc(&c.U32r, (size_t)g.Pu * 24 * sizeof(float2)));
        OVL_HIP(hipMalloc(&c.U16r, (size_t)g.Pu * 24 * sizeof(__half2)));
        c.bytes_held += (int64_t)g.Pu * (36 * (16 + 8 + 4) + 24 * (8 + 4));
    }
    k_pack_gauge<<<site_blocks(g), 256, 0, c.stream>>>((const double2 *)canon, c.U64, c.U32, (__half2 *)c.U16,
                                                       (float2 *)c.U32r, (__half2 *)c.U16r, g.V, g.Pu);
    OVL_HIP(hipGetLastError());
    const int nb = (int)site_blocks(g);
    double *part = (double *)c.buf("su3_dev", sizeof(double) * nb);
    k_su3_dev<<<nb, 256, 0, c.stream>>>((const double2 *)canon, g.V, part);
    OVL_HIP(hipGetLastError());
    std::vector<double> h(nb);
    OVL_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * nb, hipMemcpyDeviceToHost, c.stream));
    OVL_HIP(hipStreamSynchronize(c.stream));
    double m = 0.0;
    for (double v : h) m = std::max(m, std::isnan(v) ? INFINITY : v);
    c.su3_dev = m;
    c.have_gauge = true;
    update_link_form(c);
}

void update_link_form(Context &c)
{
    c.g.two_row = (c.two_row_opt && c.have_gauge && c.su3_dev >= 0.0 && c.su3_dev <= TWO_ROW_TOL) ? 1 : 0;
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
    const int64_t fwd = (c == Lm - 1) ? s - (int64_t)(Lm - 1) * st : s + st;
    const int64_t bwd = (c == 0) ? s + (int64_t)(Lm - 1) * st : s - st;
    if constexpr (std::is_same<ST, h8>::value) {   // FP16 storage: on the packed halves
        hv2 w[12], u[9];
        float sc;
        ld_sp_h(in, V, fwd, w, sc);
        ld_link_h(U, Pu, MU, s, u);
        hop_term_h<MU, true>(w, sc, u, acc);
        ld_sp_h(in, V, bwd, w, sc);
        ld_link_h(U, Pu, MU, bwd, u);
        hop_term_h<MU, false>(w, sc, u, acc);
    } else {
        cplx<R> psi[12];
        cplx<R> u[9];
        ld_sp(in, V, fwd, psi);
        ld_link(U, Pu, MU, s, u);
        hop_term<MU, true>(psi, u, acc);
        ld_sp(in, V, bwd, psi);
        ld_link(U, Pu, MU, bwd, u);
        hop_term<MU, false>(psi, u, acc);
    }
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
    } else if constexpr (std::is_same<ST, h8>::value) {   // FP16 storage: on the packed halves
        hv2 w[12], u[9];
        float sc;
#pragma unroll 1
        for (int mu = MU0; mu <= MU1; ++mu) {
            const int32_t c = co[mu], Lm = Ls[mu];
            const int64_t fwd = (c == Lm - 1) ? s - (int64_t)(Lm - 1) * st[mu] : s + st[mu];
            const int64_t bwd = (c == 0) ? s + (int64_t)(Lm - 1) * st[mu] : s - st[mu];
            ld_sp_h(in, V, fwd, w, sc);
            ld_link_h(U, Pu, mu, s, u);
            switch (mu) {
            case 0: hop_term_h<0, true>(w, sc, u, acc); break;
            case 1: hop_term_h<1, true>(w, sc, u, acc); break;
            case 2: hop_term_h<2, true>(w, sc, u, acc); break;
            default: hop_term_h<3, true>(w, sc, u, acc); break;
            }
            ld_sp_h(in, V, bwd, w, sc);
            ld_link_h(U, Pu, mu, bwd, u);
            switch (mu) {
            case 0: hop_term_h<0, false>(w, sc, u, acc); break;
            case 1: hop_term_h<1, false>(w, sc, u, acc); break;
            case 2: hop_term_h<2, false>(w, sc, u, acc); break;
            default: hop_term_h<3, false>(w, sc, u, acc); break;
            }
        }
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
//  MAP_GRP32 / MAP_GRP64  (for several fields) each XCD owns a contiguous
//             range of tiles and walks it in groups of G = 32 / 64 tiles, all
//             fields of a group one after another, the tiles of a group side
//             by side: the blocks of one tile's fields are G blocks apart on
//             the same XCD, so the group's links (G x 256 sites, 2.4 MB at
//             G = 32 in FP32, G = 64 in FP16) are fetched by the first field
//             and found in that XCD's L2 by the others, and no two blocks in
//             flight ask for the same link lines at once.
// Fields run fastest within a tile (the fields of one tile share its links).
enum { MAP_LEX = 0, MAP_REMAP = 1, MAP_COL = 2, MAP_GRP32 = 3, MAP_GRP64 = 4 };

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
        bool idle = false;
        if constexpr (MAP == MAP_GRP32 || MAP == MAP_GRP64) {
            // X = 8 ceil(T / 8) for T tiles; XCD x owns T_x = q or q + 1
            // consecutive tiles (q = T / 8, the first T % 8 XCDs one more),
            // in groups of G tiles, each group's fields back to back (a last
            // partial group likewise).  An XCD with q tiles has one idle block
            // per field, which writes the (zero) partials of slot T + x - r.
            constexpr unsigned G = MAP == MAP_GRP32 ? 32u : 64u;
            const unsigned X = gridDim.x, Y = gridDim.y;
            const unsigned T = (unsigned)((g.V + SPB - 1) / SPB);
            const unsigned lin = blockIdx.y * X + blockIdx.x;
            const unsigned xcd = lin % 8, k = lin / 8;
            const unsigned q = T / 8, rr = T % 8;
            const unsigned Tx = q + (xcd < rr ? 1u : 0u);
            const unsigned start = xcd * q + (xcd < rr ? xcd : rr);
            if (k >= Tx * Y) {
                idle = true;
                f = k - Tx * Y;
                tile = T + xcd - rr;
            } else {
                const unsigned full = Tx / G;            // whole groups
                unsigned t;
                if (k < full * G * Y) {
                    const unsigned grp = k / (G * Y), r = k % (G * Y);
                    f = r / G;
                    t = grp * G + r % G;
                } else {
                    const unsigned last = Tx - full * G, r = k - full * G * Y;
                    f = r / last;
                    t = full * G + r % last;
                }
                tile = start + t;
            }
        } else {
            tile_of_block<MAP == MAP_REMAP>(tile, f);
        }
        s = idle ? g.V : (int64_t)tile * SPB + lane;
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
// OWN: the site's own input spinor is passed in own (one lane per site)
// instead of being read again.
template <typename ST, int EPI, int TPS, bool OWN = false, typename R>
__device__ __forceinline__ void stencil_epilogue(const StencilArgs<ST> &a, unsigned f, int64_t s, int half,
                                                 const cplx<R> *acc, double part[3], const cplx<R> *own = nullptr)
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
        if constexpr (OWN) {
            static_assert(TPS == 1, "own spinor with one lane per site");
#pragma unroll
            for (int c = 0; c < NC; ++c) x[c] = own[c];
        } else {
            if constexpr (TPS == 1) ld_sp(in, V, s, x); else ld_sp_half(in, V, s, half, x);
        }
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
                // a site's sums in the arithmetic precision, the tile's in FP64
                R d0 = 0, d1 = 0, d2 = 0;
#pragma unroll
                for (int c = 0; c < NC; ++c) {
                    const R wr = ws[c].re, wi = ws[c].im;
                    d0 += x[c].re * wr + x[c].im * wi;
                    d1 += rv[c].re * wr + rv[c].im * wi;
                    d2 += wr * wr + wi * wi;
                }
                part[0] += (double)d0;
                part[1] += (double)d1;
                part[2] += (double)d2;
            } else {
#pragma unroll
                for (int c = 0; c < NC; ++c) o[c] = o[c] + x[c];
            }
        }
        if constexpr (TPS == 1) st_sp(out, V, s, o); else st_sp_half(out, V, s, half, o);
    }
}

// The epilogue for FP16 storage with two lanes per site: the lanes of a site
// sit in different waves (threadIdx.x and threadIdx.x ^ 128) and must store
// with one scale, the larger of their halves' maxima, exchanged through LDS.
// Every thread of the block calls it (valid: the lane has a site).
template <int EPI>
__device__ __forceinline__ void stencil_epilogue_pair_h8(const StencilArgs<h8> &a, unsigned f, int64_t s, int half,
                                                         const cplx<float> *acc, double part[3], bool valid)
{
    __shared__ float mx[256];
    const int64_t V = a.g.V;
    const h8 *in = a.in + f * fstride<h8>(V);
    h8 *out = a.out + f * fstride<h8>(V);
    cplx<float> o[6], x[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) o[c] = acc[c];
    if (valid && EPI != EPI_HOP) {
        ld_sp_half(in, V, s, half, x);
        const float m = (float)a.diag;
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const cplx<float> d = m * x[c] - 0.5f * o[c];
            o[c] = half == 0 ? d : -d;   // gamma_5: spins 2, 3 are components 6..11
        }
        if constexpr (EPI == EPI_K2DOT || EPI == EPI_KPLUS) {
            ld_sp_half(a.aux + f * fstride<h8>(V), V, s, half, x);
            const float sg = EPI == EPI_K2DOT ? (float)a.sigma : 1.f;
#pragma unroll
            for (int c = 0; c < 6; ++c) o[c] = o[c] + sg * x[c];
        }
    }
    const float ml = valid ? half_max(o) : 0.f;
    mx[threadIdx.x] = ml;
    __syncthreads();
    const float m = fmaxf(ml, mx[threadIdx.x ^ 128]);
    if (!valid) return;
    if constexpr (EPI == EPI_K2DOT) {
        // partials (p, w), Re (r, w), (w, w) on w as stored
        cplx<float> ws[6], rv[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) ws[c] = o[c];
        as_stored_scaled(ws, m);
        ld_sp_half(a.aux2 + f * fstride<h8>(V), V, s, half, rv);
        float d0 = 0.f, d1 = 0.f, d2 = 0.f;   // a site's sums in FP32, the tile's in FP64
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const float wr = ws[c].re, wi = ws[c].im;
            d0 += x[c].re * wr + x[c].im * wi;
            d1 += rv[c].re * wr + rv[c].im * wi;
            d2 += wr * wr + wi * wi;
        }
        part[0] += (double)d0;
        part[1] += (double)d1;
        part[2] += (double)d2;
    }
    st_sp_half_scaled(out, V, s, half, o, m);
}

// K2DOT: one partial of each dot per (field, tile).  Every thread of the block
// must call it.
template <typename ST, int EPI>
__device__ __forceinline__ void store_partials(const StencilArgs<ST> &a, unsigned f, unsigned tile,
                                               const double part[3])
{
    if constexpr (EPI == EPI_K2DOT) {
        // the three block sums in one LDS pass, each with block_sum's tree
        __shared__ double l3[3][4];
        double v[3] = {part[0], part[1], part[2]};
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        __syncthreads();
        if (lane == 0)
#pragma unroll
            for (int k = 0; k < 3; ++k) l3[k][wave] = v[k];
        __syncthreads();
        if (threadIdx.x == 0) {
            double t[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                t[k] = 0.0;
#pragma unroll
                for (int w = 0; w < 4; ++w) t[k] += l3[k][w];
            }
            const double t0 = t[0], t1 = t[1], t2 = t[2];
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
    if constexpr (TPS == 2 && std::is_same<ST, h8>::value)
        stencil_epilogue_pair_h8<EPI>(a, f, s, half, acc, part, valid);
    else if (valid)
        stencil_epilogue<ST, EPI, TPS>(a, f, s, half, acc, part);
    store_partials<ST, EPI>(a, f, tile, part);
}

// Several fields at once with their links read once per group of fields
// (FP16 storage): one lane per site of a 256-site tile loads the site's eight
// links, U_mu(x) and U_mu(x - mu), into registers as packed halves (the
// two-row form rebuilt once) and then walks the MF_GROUP fields of its block
// (grid y), so a launch over nf fields fetches each link nf / MF_GROUP times
// instead of nf times (and the launch has nf / MF_GROUP times more blocks
// than with every field in one block).  Blocks go to the eight XCDs
// round-robin, and the groups run one after another (grid y).  Without COL,
// tiles are lexicographic runs of 256 sites, each XCD owning a contiguous
// eighth of them.  With COL, each XCD owns one of the eight xyz columns
// (Geom::cb, as MAP_COL) and walks it through t a column slice at a time, so
// that the spinors a slice fetches for its t + 1 hops are still in that
// XCD's L2 when the next two slices use them (a column slice of a group of
// four FP16 fields is under 1 MB on 24^3 x 48).
static constexpr int MF_GROUP = 4;   // fields per block of the multi-field stencil

template <typename GT, int EPI, bool COL>
__global__ __launch_bounds__(256) void k_stencil_mf(StencilArgs<h8> a, const GT *__restrict__ U, int nf)
{
    const Geom &g = a.g;
    const int64_t V = g.V, Pu = g.Pu;
    unsigned tile;
    int64_t s;
    bool valid;
    if constexpr (COL) {
        // grid x = 8 Lt tps (tps tiles per column slice): column x % 8, then
        // slice t and the tile within it
        const unsigned per_col = gridDim.x / 8, col = blockIdx.x % 8, rest = blockIdx.x / 8;
        const unsigned tps = per_col / (unsigned)g.L[3];
        const int32_t t = (int32_t)(rest / tps);
        const int32_t local = (int32_t)(rest % tps) * 256 + (int32_t)threadIdx.x;
        tile = col * per_col + rest;
        valid = local < g.col_sites;
        const int32_t l = valid ? local : 0;
        const int32_t cx = (int32_t)col % g.cn[0], cy = ((int32_t)col / g.cn[0]) % g.cn[1],
                      cz = (int32_t)col / (g.cn[0] * g.cn[1]);
        const int32_t x0 = cx * g.cb[0] + l % g.cb[0], x1 = cy * g.cb[1] + (l / g.cb[0]) % g.cb[1],
                      x2 = cz * g.cb[2] + l / (g.cb[0] * g.cb[1]);
        s = x0 + (int64_t)g.L[0] * (x1 + (int64_t)g.L[1] * (x2 + (int64_t)g.L[2] * t));
    } else {
        const unsigned T = (unsigned)((V + 255) / 256), per = gridDim.x / 8;
        tile = (blockIdx.x % 8) * per + blockIdx.x / 8;
        s = (int64_t)tile * 256 + threadIdx.x;
        valid = tile < T && s < V;
    }
    hv2 u[8][9];        // U_mu(x) in u[mu], U_mu(x - mu) in u[4 + mu]
    int64_t nb[8];      // x + mu in nb[mu], x - mu in nb[4 + mu]
    if (valid) {
        int64_t r = s;
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) {
            const int32_t c = (int32_t)(r % g.L[mu]), Lm = g.L[mu];
            r /= g.L[mu];
            const int64_t st = g.stride[mu];
            nb[mu] = (c == Lm - 1) ? s - (int64_t)(Lm - 1) * st : s + st;
            nb[4 + mu] = (c == 0) ? s + (int64_t)(Lm - 1) * st : s - st;
            ld_link_h(U, Pu, mu, s, u[mu]);
            ld_link_h(U, Pu, mu, nb[4 + mu], u[4 + mu]);
        }
    }
    const int it = a.itb ? *a.itb + a.it : a.it;
    const int f0 = (int)blockIdx.y * MF_GROUP, f1 = f0 + MF_GROUP < nf ? f0 + MF_GROUP : nf;
#pragma unroll 1
    for (int f = f0; f < f1; ++f) {
        if (a.stop != nullptr && it >= a.stop[f]) continue;   // field converged (the same for the whole block)
        double part[3] = {0.0, 0.0, 0.0};
        if (valid) {
            const h8 *in = a.in + f * fstride<h8>(V);
            cplx<float> acc[12];
#pragma unroll
            for (int c = 0; c < 12; ++c) acc[c] = {0.f, 0.f};
            hv2 w[12];
            float sc;
            ld_sp_h(in, V, nb[0], w, sc);
            hop_term_h<0, true>(w, sc, u[0], acc);
            ld_sp_h(in, V, nb[4], w, sc);
            hop_term_h<0, false>(w, sc, u[4], acc);
            ld_sp_h(in, V, nb[1], w, sc);
            hop_term_h<1, true>(w, sc, u[1], acc);
            ld_sp_h(in, V, nb[5], w, sc);
            hop_term_h<1, false>(w, sc, u[5], acc);
            ld_sp_h(in, V, nb[2], w, sc);
            hop_term_h<2, true>(w, sc, u[2], acc);
            ld_sp_h(in, V, nb[6], w, sc);
            hop_term_h<2, false>(w, sc, u[6], acc);
            ld_sp_h(in, V, nb[3], w, sc);
            hop_term_h<3, true>(w, sc, u[3], acc);
            ld_sp_h(in, V, nb[7], w, sc);
            hop_term_h<3, false>(w, sc, u[7], acc);
            stencil_epilogue<h8, EPI, 1>(a, f, s, 0, acc, part);
        }
        store_partials<h8, EPI>(a, f, tile, part);
    }
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
        if constexpr (TPS == 2 && std::is_same<ST, h8>::value)
            stencil_epilogue_pair_h8<EPI>(a, f, s, half, acc, part, valid);
        else if (valid)
            stencil_epilogue<ST, EPI, TPS>(a, f, s, half, acc, part);
    }
    store_partials<ST, EPI>(a, f, tile, part);
}

// ----------------------------------------------------- LDS-tiled time march
// A block owns a spatial tile of b0 x b1 x b2 = 256 sites (one lane each) and
// walks T consecutive time slices.  At every slice each lane copies its own
// stored spinor psi(y) into LDS (same plane layout as in memory, 256-site
// planes); after a barrier a lane reads each x, y, z neighbour through one
// generic pointer that points into the LDS tile when the neighbour is inside
// it and into memory on a tile face or across a periodic wrap (no divergent
// branches), so inside the tile every spinor is read from memory once per
// slice instead of seven times.  Links are read from memory.  The time hops
// are carried in registers as in the column march (psi(t + 1) becomes the next
// slice's own spinor; U_t(t)^+ (1 + gamma_t) psi(t) is the next slice's
// backward term), and the epilogue takes the own spinor from registers.  Math
// in FP32 (FP32 and FP16 storage).
struct TileShape {
    int32_t b[3];   // tile extent per spatial direction (b0 b1 b2 = 256)
    int32_t n[3];   // tiles per direction (the last one may be partial)
    int32_t T;      // time slices per block
    int32_t nch;    // time chunks, Lt / T
};
static constexpr int LDS_SITES = 256;

// A site's spinor as stored.
template <typename ST> struct SpRaw;
template <> struct SpRaw<float4> {
    float4 q[6];
};
template <> struct SpRaw<h8> {
    uint4 q[3];
    float sc;
};

// Planes at base[k * stride] (memory: stride V; LDS tile: stride 256); for
// FP16 storage the scale at *sc.
__device__ __forceinline__ void ld_raw(const float4 *base, const float *, int64_t stride, SpRaw<float4> &r)
{
#pragma unroll
    for (int k = 0; k < 6; ++k) r.q[k] = base[k * stride];
}
__device__ __forceinline__ void ld_raw(const h8 *base, const float *sc, int64_t stride, SpRaw<h8> &r)
{
#pragma unroll
    for (int k = 0; k < 3; ++k) r.q[k] = base[k * stride].v;
    r.sc = *sc;
}
__device__ __forceinline__ void st_raw(float4 *base, float *, int64_t stride, const SpRaw<float4> &r)
{
#pragma unroll
    for (int k = 0; k < 6; ++k) base[k * stride] = r.q[k];
}
__device__ __forceinline__ void st_raw(h8 *base, float *sc, int64_t stride, const SpRaw<h8> &r)
{
#pragma unroll
    for (int k = 0; k < 3; ++k) base[k * stride].v = r.q[k];
    *sc = r.sc;
}
// the values ld_sp returns for the same stored spinor
__device__ __forceinline__ void unpack(const SpRaw<float4> &r, cplx<float> v[12])
{
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        v[2 * k] = {r.q[k].x, r.q[k].y};
        v[2 * k + 1] = {r.q[k].z, r.q[k].w};
    }
}
__device__ __forceinline__ void unpack(const SpRaw<h8> &r, cplx<float> v[12])
{
    const float sc = r.sc;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const uint4 t = r.q[k];
        const float2 a = h2f2(t.x), b = h2f2(t.y), c = h2f2(t.z), d = h2f2(t.w);
        v[4 * k] = {a.x * sc, a.y * sc};
        v[4 * k + 1] = {b.x * sc, b.y * sc};
        v[4 * k + 2] = {c.x * sc, c.y * sc};
        v[4 * k + 3] = {d.x * sc, d.y * sc};
    }
}
// scale plane of a field in memory (FP16 storage; unused otherwise)
__device__ __forceinline__ const float *scale_plane(const float4 *, int64_t) { return nullptr; }
__device__ __forceinline__ const float *scale_plane(const h8 *p, int64_t V)
{
    return reinterpret_cast<const float *>(p + 3 * V);
}
__device__ __forceinline__ void ld_raw_site(const float4 *in, const float *, int64_t V, int64_t s, SpRaw<float4> &r)
{
    ld_raw(in + s, nullptr, V, r);
}
__device__ __forceinline__ void ld_raw_site(const h8 *in, const float *sc, int64_t V, int64_t s, SpRaw<h8> &r)
{
    ld_raw(in + s, sc + s, V, r);
}

// Neighbour spinor of lane tid: in the LDS tile (lane tid + d) when inside,
// at site ns in memory otherwise.
template <typename ST>
__device__ __forceinline__ void ld_nbr(const ST *in, const float *sc, int64_t V, int64_t ns, bool inside, const ST *Lsp,
                                       const float *Lsc, int lane, cplx<float> v[12])
{
    const ST *b = inside ? Lsp + lane : in + ns;
    const float *q = inside ? Lsc + lane : (sc ? sc + ns : nullptr);
    SpRaw<ST> r;
    ld_raw(b, q, inside ? (int64_t)LDS_SITES : V, r);
    unpack(r, v);
}

// A link as stored (the planes ld_link reads), for staging in LDS: FP32 as
// four float4 and one float2, FP16 as two uint4 and one uint32.
template <typename GT>
struct LinkRaw;
template <>
struct LinkRaw<float2> {
    float4 q[4];
    float2 r;
};
template <>
struct LinkRaw<__half2> {
    uint4 q[2];
    uint32_t r;
};
__device__ __forceinline__ void ld_link_raw(const float2 *__restrict__ U, int64_t P, int mu, int64_t s,
                                            LinkRaw<float2> &l)
{
    const float4 *Q = reinterpret_cast<const float4 *>(U);
    const float2 *R = reinterpret_cast<const float2 *>(Q + 16 * P);
#pragma unroll
    for (int k = 0; k < 4; ++k) l.q[k] = Q[(mu * 4 + k) * P + s];
    l.r = R[mu * P + s];
}
__device__ __forceinline__ void ld_link_raw(const __half2 *__restrict__ U, int64_t P, int mu, int64_t s,
                                            LinkRaw<__half2> &l)
{
    const uint4 *Q = reinterpret_cast<const uint4 *>(U);
    const uint32_t *R = reinterpret_cast<const uint32_t *>(Q + 8 * P);
#pragma unroll
    for (int k = 0; k < 2; ++k) l.q[k] = Q[(mu * 2 + k) * P + s];
    l.r = R[mu * P + s];
}
template <>
struct LinkRaw<f2r12> {
    float4 q[2];
    float4 r;
};
template <>
struct LinkRaw<h2r12> {
    uint4 q[1];
    uint2 r;
};
__device__ __forceinline__ void ld_link_raw(const f2r12 *__restrict__ U, int64_t P, int mu, int64_t s,
                                            LinkRaw<f2r12> &l)
{
    const float4 *Q = reinterpret_cast<const float4 *>(U);
#pragma unroll
    for (int k = 0; k < 2; ++k) l.q[k] = Q[(mu * 2 + k) * P + s];
    l.r = Q[8 * P + mu * P + s];
}
__device__ __forceinline__ void ld_link_raw(const h2r12 *__restrict__ U, int64_t P, int mu, int64_t s,
                                            LinkRaw<h2r12> &l)
{
    const uint4 *Q = reinterpret_cast<const uint4 *>(U);
    l.q[0] = Q[mu * P + s];
    l.r = reinterpret_cast<const uint2 *>(Q + 4 * P)[mu * P + s];
}
__device__ __forceinline__ void unpack_link(const LinkRaw<f2r12> &l, cplx<float> u[9])
{
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        u[2 * k] = {l.q[k].x, l.q[k].y};
        u[2 * k + 1] = {l.q[k].z, l.q[k].w};
    }
    u[4] = {l.r.x, l.r.y};
    u[5] = {l.r.z, l.r.w};
    su3_third_row(u);
}
__device__ __forceinline__ void unpack_link(const LinkRaw<h2r12> &l, cplx<float> u[9])
{
    const uint4 q = l.q[0];
    const float2 a = h2f2(q.x), b = h2f2(q.y), c = h2f2(q.z), d = h2f2(q.w);
    u[0] = {a.x, a.y};
    u[1] = {b.x, b.y};
    u[2] = {c.x, c.y};
    u[3] = {d.x, d.y};
    const float2 e = h2f2(l.r.x), f = h2f2(l.r.y);
    u[4] = {e.x, e.y};
    u[5] = {f.x, f.y};
    su3_third_row(u);
}
// the values ld_link returns for the same stored link
__device__ __forceinline__ void unpack_link(const LinkRaw<float2> &l, cplx<float> u[9])
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        u[2 * k] = {l.q[k].x, l.q[k].y};
        u[2 * k + 1] = {l.q[k].z, l.q[k].w};
    }
    u[8] = {l.r.x, l.r.y};
}
__device__ __forceinline__ void unpack_link(const LinkRaw<__half2> &l, cplx<float> u[9])
{
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const uint4 q = l.q[k];
        const float2 a = h2f2(q.x), b = h2f2(q.y), c = h2f2(q.z), d = h2f2(q.w);
        u[4 * k] = {a.x, a.y};
        u[4 * k + 1] = {b.x, b.y};
        u[4 * k + 2] = {c.x, c.y};
        u[4 * k + 3] = {d.x, d.y};
    }
    const float2 r = h2f2(l.r);
    u[8] = {r.x, r.y};
}
// The forward links of NLD spatial directions for the tile's sites at the
// current slice, plane by plane (lane-consecutive words, no bank conflicts):
// FP16 stages x, y, z (27 KB), FP32 x, y (36 KB beside the 24 KB of spinors).
template <typename GT, int NLD>
struct LinkLds {
    using QT = typename std::remove_reference<decltype(LinkRaw<GT>{}.q[0])>::type;
    using RT = decltype(LinkRaw<GT>{}.r);
    static constexpr int NQ = sizeof(LinkRaw<GT>{}.q) / sizeof(QT);
    QT q[NLD][NQ][LDS_SITES];
    RT r[NLD][LDS_SITES];
    __device__ __forceinline__ void put(int mu, int lane, const LinkRaw<GT> &l)
    {
#pragma unroll
        for (int k = 0; k < NQ; ++k) q[mu][k][lane] = l.q[k];
        r[mu][lane] = l.r;
    }
    __device__ __forceinline__ void get(int mu, int lane, cplx<float> u[9]) const
    {
        LinkRaw<GT> l;
#pragma unroll
        for (int k = 0; k < NQ; ++k) l.q[k] = q[mu][k][lane];
        l.r = r[mu][lane];
        unpack_link(l, u);
    }
};

// A link through one generic pointer pair: planes q[k * qs] and the last
// entry *r, in LDS (qs = LDS_SITES) or in memory (qs = the plane stride).
template <typename GT>
__device__ __forceinline__ void ld_link_at(const typename LinkLds<GT, 1>::QT *q, int64_t qs,
                                           const typename LinkLds<GT, 1>::RT *r, cplx<float> u[9])
{
    LinkRaw<GT> l;
#pragma unroll
    for (int k = 0; k < LinkLds<GT, 1>::NQ; ++k) l.q[k] = q[k * qs];
    l.r = *r;
    unpack_link(l, u);
}

// One spatial direction of the LDS-tiled stencil.  With Lu (links staged in
// LDS for this direction) the own forward link and, for a neighbour inside the
// tile, the backward neighbour's forward link U_mu(x - mu) come from LDS; the
// choice is a pointer, not a branch (as for the neighbour spinors).
template <int MU, bool USEL, typename ST, typename GT, typename LL>
__device__ __forceinline__ void tile_dir(const ST *in, const float *sc, const GT *__restrict__ U, int64_t V,
                                         int64_t Pu, int64_t s, int32_t c, int32_t Lm, int64_t st, int tid, int lstep,
                                         bool fin, bool bin, const ST *Lsp, const float *Lsc, const LL *Lu,
                                         cplx<float> acc[12])
{
    cplx<float> v[12], u[9];
    const int64_t fwd = (c == Lm - 1) ? s - (int64_t)(Lm - 1) * st : s + st;
    const int64_t bwd = (c == 0) ? s + (int64_t)(Lm - 1) * st : s - st;
    ld_nbr(in, sc, V, fwd, fin, Lsp, Lsc, tid + lstep, v);
    if constexpr (USEL)
        ld_link_at<GT>(&Lu->q[MU][0][tid], LDS_SITES, &Lu->r[MU][tid], u);
    else
        ld_link(U, Pu, MU, s, u);
    hop_term<MU, true>(v, u, acc);
    ld_nbr(in, sc, V, bwd, bin, Lsp, Lsc, tid - lstep, v);
    if constexpr (USEL) {
        using QT = typename LinkLds<GT, 1>::QT;
        using RT = typename LinkLds<GT, 1>::RT;
        constexpr int NQ = LinkLds<GT, 1>::NQ;
        const QT *Qg = reinterpret_cast<const QT *>(U);
        const RT *Rg = reinterpret_cast<const RT *>(Qg + 4 * NQ * Pu);
        const QT *q = bin ? &Lu->q[MU][0][tid - lstep] : Qg + (int64_t)MU * NQ * Pu + bwd;
        const RT *r = bin ? &Lu->r[MU][tid - lstep] : Rg + (int64_t)MU * Pu + bwd;
        ld_link_at<GT>(q, bin ? (int64_t)LDS_SITES : Pu, r, u);
    } else {
        ld_link(U, Pu, MU, bwd, u);
    }
    hop_term<MU, false>(v, u, acc);
}

template <typename ST, typename GT, int EPI, bool LINKS>
__device__ __forceinline__ void stencil_lds_body(const StencilArgs<ST> &a, const GT *__restrict__ U,
                                                 const TileShape &ts)
{
    __shared__ ST Lsp[Planes<ST>::n * LDS_SITES];   // the tile's stored spinors at the current slice
    __shared__ float Lsc[LDS_SITES];                 // their scales (FP16 storage; unused otherwise)
    // spatial directions with staged links: three where a link takes at most
    // 48 bytes (FP16, both FP32 two-row and FP16 two-row), else two
    constexpr int NLD = sizeof(LinkRaw<GT>) <= 48 ? 3 : 2;
    using LL = LinkLds<GT, NLD>;
    __shared__ typename std::conditional<LINKS, LL, char>::type Lu_store;
    LL *Lu = LINKS ? reinterpret_cast<LL *>(&Lu_store) : nullptr;
    const Geom &g = a.g;
    const unsigned X = gridDim.x, Y = gridDim.y;
    const unsigned lin = blockIdx.y * X + blockIdx.x;
    const unsigned ntl = (unsigned)(ts.n[0] * ts.n[1] * ts.n[2]);
    unsigned chunk, f, tl;
    if (ts.nch % 8 == 0) {   // XCD x (blocks go to the XCDs round-robin) owns nch / 8 consecutive chunks
        const unsigned x = lin % 8, k = lin / 8, per = (unsigned)ts.nch / 8;
        f = k % Y;
        const unsigned r = k / Y;
        chunk = x * per + r / ntl;
        tl = r % ntl;
    } else {
        f = lin % Y;
        const unsigned r = lin / Y;
        chunk = r / ntl;
        tl = r % ntl;
    }
    const unsigned tile = chunk * ntl + tl;
    const int it = a.itb ? *a.itb + a.it : a.it;
    if (a.stop != nullptr && it >= a.stop[f]) return;   // whole block: field converged
    const int tid = (int)threadIdx.x;
    const int b0 = ts.b[0], b1 = ts.b[1];
    const int l0 = tid % b0, l1 = (tid / b0) % b1, l2 = tid / (b0 * b1);
    int32_t co[3];
    co[0] = (int32_t)(tl % (unsigned)ts.n[0]) * b0 + l0;
    co[1] = (int32_t)((tl / (unsigned)ts.n[0]) % (unsigned)ts.n[1]) * b1 + l1;
    co[2] = (int32_t)(tl / (unsigned)(ts.n[0] * ts.n[1])) * ts.b[2] + l2;
    const bool valid = co[0] < g.L[0] && co[1] < g.L[1] && co[2] < g.L[2];
    const int64_t V = g.V, S3 = g.stride[3], Pu = g.Pu;
    const int64_t xyz = valid ? co[0] + (int64_t)g.L[0] * (co[1] + (int64_t)g.L[1] * co[2]) : 0;
    // neighbour inside the tile and no periodic wrap (a valid lane's in-tile
    // neighbours are valid)
    const bool f0 = l0 + 1 < b0 && co[0] + 1 < g.L[0], f1 = l1 + 1 < b1 && co[1] + 1 < g.L[1],
               f2 = l2 + 1 < ts.b[2] && co[2] + 1 < g.L[2];
    const bool k0 = l0 > 0, k1 = l1 > 0, k2 = l2 > 0;
    const ST *in = a.in + f * fstride<ST>(V);
    const float *sc = scale_plane(in, V);
    const int Lt = g.L[3], T = ts.T, t0 = (int)chunk * T;
    SpRaw<ST> cur;     // psi(t) as stored
    cplx<float> gb[6];  // backward t term of site t
    if (valid) {
        const int64_t s0 = xyz + (int64_t)t0 * S3;
        const int64_t sm = t0 == 0 ? s0 + (int64_t)(Lt - 1) * S3 : s0 - S3;
        cplx<float> v[12], u[9], h[6];
        ld_sp(in, V, sm, v);
        ld_link(U, Pu, 3, sm, u);
        spin_proj<3, false>(v, h);
        link_mul<false>(u, h, gb);
        ld_raw_site(in, sc, V, s0, cur);
    }
    double part[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < T; ++j) {
        const int t = t0 + j;
        const int64_t s = xyz + (int64_t)t * S3;
        if (valid) st_raw(Lsp + tid, Lsc + tid, LDS_SITES, cur);
        if constexpr (LINKS) {
            if (valid)
#pragma unroll
                for (int mu = 0; mu < NLD; ++mu) {
                    LinkRaw<GT> l;
                    ld_link_raw(U, Pu, mu, s, l);
                    Lu->put(mu, tid, l);
                    asm volatile("" ::: "memory");   // one direction's link in registers at a time
                }
        }
        __syncthreads();
        if (valid) {
            cplx<float> acc[12];
#pragma unroll
            for (int c = 0; c < 12; ++c) acc[c] = {0.f, 0.f};
            tile_dir<0, LINKS>(in, sc, U, V, Pu, s, co[0], g.L[0], g.stride[0], tid, 1, f0, k0, Lsp, Lsc, Lu, acc);
            tile_dir<1, LINKS>(in, sc, U, V, Pu, s, co[1], g.L[1], g.stride[1], tid, b0, f1, k1, Lsp, Lsc, Lu, acc);
            tile_dir<2, LINKS && (NLD > 2)>(in, sc, U, V, Pu, s, co[2], g.L[2], g.stride[2], tid, b0 * b1, f2, k2,
                                            Lsp, Lsc, Lu, acc);
            const int64_t sp = t == Lt - 1 ? s - (int64_t)(Lt - 1) * S3 : s + S3;
            SpRaw<ST> nr;
            ld_raw_site(in, sc, V, sp, nr);
            cplx<float> v[12], ut[9], h[6], gg[6];
            ld_link(U, Pu, 3, s, ut);
            unpack(nr, v);
            spin_proj<3, true>(v, h);
            link_mul<true>(ut, h, gg);
            spin_recon<3, true>(gg, acc);    // (1 - gamma_t) U_t(t) psi(t + 1)
            spin_recon<3, false>(gb, acc);   // (1 + gamma_t) U_t(t - 1)^+ psi(t - 1)
            unpack(cur, v);
            spin_proj<3, false>(v, h);
            link_mul<false>(ut, h, gb);      // the backward term of site t + 1
            stencil_epilogue<ST, EPI, 1, true>(a, f, s, 0, acc, part, v);
            cur = nr;
        }
        if (j + 1 < T) __syncthreads();     // LDS is rewritten by the next slice
    }
    store_partials<ST, EPI>(a, f, tile, part);
}

template <typename ST, typename GT, int EPI, bool LINKS>
__global__ __launch_bounds__(256) void k_stencil_lds(StencilArgs<ST> a, const GT *__restrict__ U, TileShape ts)
{
    stencil_lds_body<ST, GT, EPI, LINKS>(a, U, ts);
}
// with the links staged: registers held to two waves per SIMD (the LDS of
// two blocks fits a compute unit)
template <typename ST, typename GT, int EPI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_stencil_ldsl(
    StencilArgs<ST> a, const GT *__restrict__ U, TileShape ts)
{
    stencil_lds_body<ST, GT, EPI, true>(a, U, ts);
}

// Launch shape chosen per (precision, epilogue, nf) by timing the variants on
// the context's lattice the first time that shape is used (autotuning).
// Launch variants: 0 / 1 one lane per site, MAP_LEX / MAP_REMAP; 2 / 3 two
// lanes per site, likewise; 4 / 5 MAP_COL with one / two lanes per site; 6 / 7
// the t-marching kernel with one / two lanes per site (Lt a multiple of 8).
// With FP16 storage the two lanes of a site share its scale through LDS.  8 .. 11 the
// LDS-tiled march with T = 1, 2, 4, 8 time slices per block (Lt a multiple of
// T; FP32 and FP16 storage).  12 .. 15 the grouped XCD order MAP_GRP32 /
// MAP_GRP64 with one / two lanes per site (12: G 32, one lane; 13: G 32, two;
// 14: G 64, one; 15: G 64, two).  16 .. 19 the LDS-tiled march (T = 1, 2, 4,
// 8) with the tile's forward spatial links also staged in LDS, so that the
// backward hop of a site inside the tile reads its neighbour's link there.
// 20 (FP16 storage) one lane per site walking a group of four fields with the
// site's links held in registers (k_stencil_mf); 21 the same in the XCD
// column order of 4 / 5.
static constexpr int N_VARIANTS = OVL_STENCIL_VARIANTS;
static bool variant_lds(int v) { return (v >= 8 && v < 12) || (v >= 16 && v < 20); }
static int variant_tps(int v) { return (v == 2 || v == 3 || v == 5 || v == 7 || v == 13 || v == 15) ? 2 : 1; }

// Tile of the LDS-tiled march: the 256-site box with the fewest padded sites,
// then the fewest face sites (each face lane fetches a neighbour from memory).
static TileShape tile_shape(const Geom &g, int v)
{
    static const int cand[][3] = {{8, 8, 4}, {8, 4, 8}, {4, 8, 8}, {16, 4, 4}, {4, 16, 4}, {4, 4, 16},
                                  {16, 8, 2}, {8, 16, 2}, {16, 16, 1}, {32, 8, 1}, {32, 4, 2}, {2, 8, 16}};
    TileShape ts{};
    double best = 1e300;
    for (const auto &b : cand) {
        int64_t padded = 1;
        double face = 0.0;
        for (int m = 0; m < 3; ++m) {
            padded *= (int64_t)((g.L[m] + b[m] - 1) / b[m]) * b[m];
            face += 1.0 / b[m];
        }
        const double score = (double)padded * (1.0 + 0.5 * face);
        if (score < best) {
            best = score;
            for (int m = 0; m < 3; ++m) {
                ts.b[m] = b[m];
                ts.n[m] = (g.L[m] + b[m] - 1) / b[m];
            }
        }
    }
    ts.T = 1 << (v >= 16 ? v - 16 : v - 8);
    ts.nch = g.L[3] / ts.T;
    return ts;
}

unsigned stencil_tiles(const Geom &g, int v)
{
    const int tps = variant_tps(v);
    const int spb = 256 / tps;
    if ((v >= 12 && v < 16) || v == 20)
        return 8u * (unsigned)(((g.V + spb - 1) / spb + 7) / 8);   // 8 XCDs x their largest share
    if (variant_lds(v)) {
        const TileShape ts = tile_shape(g, v);
        return (unsigned)(ts.n[0] * ts.n[1] * ts.n[2] * ts.nch);
    }
    if (v == 21) return 8u * (unsigned)g.L[3] * (unsigned)((g.col_sites + 255) / 256);
    if (v >= 6) return 8u * (unsigned)((g.stride[3] + spb - 1) / spb);
    if (v >= 4) return 8u * (unsigned)g.L[3] * (unsigned)((g.col_sites + spb - 1) / spb);
    return (unsigned)((g.V * tps + 255) / 256);
}

bool stencil_variant_ok(const Geom &g, int prec, int v)
{
    if (v < 0 || v >= N_VARIANTS) return false;
    if ((v == 4 || v == 5) && !g.col_ok) return false;
    if ((v == 6 || v == 7) && g.L[3] % 8 != 0) return false;
    if (variant_lds(v)) return prec != OVL_F64 && g.L[3] % (1 << (v >= 16 ? v - 16 : v - 8)) == 0;
    if (v == 20) return prec == OVL_HALF;
    if (v == 21) return prec == OVL_HALF && g.col_ok;
    return true;
}

int64_t stencil_tiles_max(const Geom &g)
{
    int64_t m = 0;
    for (int v = 0; v < N_VARIANTS; ++v)
        if (stencil_variant_ok(g, OVL_F64, v) || stencil_variant_ok(g, OVL_F32, v) ||
            stencil_variant_ok(g, OVL_HALF, v))
            m = std::max<int64_t>(m, stencil_tiles(g, v));
    return m;
}

template <typename ST, typename GT, int EPI, int TPS, int MAP>
static void launch_variant(Context &c, const StencilArgs<ST> &a, const GT *U, int nf, const PendingEvent *pe)
{
    const int v = MAP == MAP_COL     ? (TPS == 2 ? 5 : 4)
                  : MAP == MAP_GRP32 ? (TPS == 2 ? 13 : 12)
                  : MAP == MAP_GRP64 ? (TPS == 2 ? 15 : 14)
                                     : (TPS == 2 ? 2 : 0) + (MAP == MAP_REMAP ? 1 : 0);
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
static void launch_lds(Context &c, int v, const StencilArgs<ST> &a, const GT *U, int nf, const PendingEvent *pe)
{
    const TileShape ts = tile_shape(c.g, v);
    dim3 grid(stencil_tiles(c.g, v), nf);
    if (v >= 16)
        launch_k(c, pe, k_stencil_ldsl<ST, GT, EPI>, grid, dim3(256), 0, a, U, ts);
    else
        launch_k(c, pe, k_stencil_lds<ST, GT, EPI, false>, grid, dim3(256), 0, a, U, ts);
}

template <typename ST, typename GT, int EPI>
static void launch_by_id(Context &c, int id, const StencilArgs<ST> &a, const GT *U, int nf,
                         const PendingEvent *pe = nullptr)
{
    if constexpr (!std::is_same<ST, double2>::value) {   // FP32 math only
        if (variant_lds(id)) {
            launch_lds<ST, GT, EPI>(c, id, a, U, nf, pe);
            return;
        }
    }
    {
        switch (id) {
        case 0: launch_variant<ST, GT, EPI, 1, MAP_LEX>(c, a, U, nf, pe); break;
        case 1: launch_variant<ST, GT, EPI, 1, MAP_REMAP>(c, a, U, nf, pe); break;
        case 2: launch_variant<ST, GT, EPI, 2, MAP_LEX>(c, a, U, nf, pe); break;
        case 3: launch_variant<ST, GT, EPI, 2, MAP_REMAP>(c, a, U, nf, pe); break;
        case 4: launch_variant<ST, GT, EPI, 1, MAP_COL>(c, a, U, nf, pe); break;
        case 5: launch_variant<ST, GT, EPI, 2, MAP_COL>(c, a, U, nf, pe); break;
        case 6: launch_tmarch<ST, GT, EPI, 1>(c, a, U, nf, pe); break;
        case 12: launch_variant<ST, GT, EPI, 1, MAP_GRP32>(c, a, U, nf, pe); break;
        case 13: launch_variant<ST, GT, EPI, 2, MAP_GRP32>(c, a, U, nf, pe); break;
        case 14: launch_variant<ST, GT, EPI, 1, MAP_GRP64>(c, a, U, nf, pe); break;
        case 15: launch_variant<ST, GT, EPI, 2, MAP_GRP64>(c, a, U, nf, pe); break;
        case 20:
        case 21:
            if constexpr (std::is_same<ST, h8>::value) {
                const dim3 grid(stencil_tiles(c.g, id), (nf + MF_GROUP - 1) / MF_GROUP);
                if (id == 20)
                    launch_k(c, pe, k_stencil_mf<GT, EPI, false>, grid, dim3(256), 0, a, U, nf);
                else
                    launch_k(c, pe, k_stencil_mf<GT, EPI, true>, grid, dim3(256), 0, a, U, nf);
            } else {
                throw Error{OVL_ERR_ARG, "stencil variants 20 and 21 are for FP16 storage"};
            }
            break;
        default: launch_tmarch<ST, GT, EPI, 2>(c, a, U, nf, pe); break;
        }
    }
}

template <typename ST, typename GT, int EPI>
static int tuned_variant(Context &c, const StencilArgs<ST> &a, const GT *U, int nf, int prec)
{
    const int key = (prec * 8 + EPI) * 64 + (nf < 63 ? nf : 63);
    auto it = c.tuned.find(key);
    if (it != c.tuned.end()) return it->second;
    if (c.no_alloc) return 1;   // timing would need workspace and events: fixed shape, not recorded
    if (c.autotune == 0) return c.tuned[key] = 1;
    // time every variant on scratch output
    StencilArgs<ST> t = a;
    t.stop = nullptr;
    t.out = (ST *)c.buf("tune_out", field_bytes(c.g, prec) * nf);
    t.partial = (double *)c.buf("tune_part", sizeof(double) * 3 * (size_t)nf * stencil_tiles_max(c.g));
    hipEvent_t e0 = c.event(), e1 = c.event();
    // three rounds over the variants (interleaved, so that clock drift hits
    // them alike), five launches each; a variant counts with its best round
    std::vector<float> ms_best(N_VARIANTS, 1e30f);
    for (int v = 0; v < N_VARIANTS; ++v)
        if (stencil_variant_ok(c.g, prec, v)) launch_by_id<ST, GT, EPI>(c, v, t, U, nf);   // warm-up
    for (int round = 0; round < 3; ++round)
        for (int v = 0; v < N_VARIANTS; ++v) {
            if (!stencil_variant_ok(c.g, prec, v)) continue;
            OVL_HIP(hipEventRecord(e0, c.stream));
            for (int r = 0; r < 5; ++r) launch_by_id<ST, GT, EPI>(c, v, t, U, nf);
            OVL_HIP(hipEventRecord(e1, c.stream));
            OVL_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            OVL_HIP(hipEventElapsedTime(&ms, e0, e1));
            ms_best[v] = std::min(ms_best[v], ms);
        }
    int best = 0;
    for (int v = 1; v < N_VARIANTS; ++v)
        if (ms_best[v] < ms_best[best]) best = v;
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
    // nf fields in one launch share one read of the links
    const double G = stencil_link_bytes(c.g, prec);
    const double bytes = a.stop ? 0.0 : (stencil_bytes(c.g, prec, EPI) - G) * nf + G;
    const bool prof = profile && c.prof && !c.no_alloc;
    if (prof) c.prof_begin(pe, KERN_STENCIL, prec, bytes);
    launch_by_id<ST, GT, EPI>(c, v, a, U, nf, prof ? &pe : nullptr);
    OVL_HIP(hipGetLastError());
    if (prof) c.prof_end(pe);
}

template <typename ST, typename GT>
static void stencil_epi(Context &c, int epi, const StencilArgs<ST> &a, const GT *U, int nf, int prec)
{
    switch (epi) {
    case EPI_HOP: launch_stencil_t<ST, GT, EPI_HOP>(c, a, U, nf, prec, true); break;
    case EPI_K: launch_stencil_t<ST, GT, EPI_K>(c, a, U, nf, prec, true); break;
    case EPI_K2DOT: launch_stencil_t<ST, GT, EPI_K2DOT>(c, a, U, nf, prec, true); break;
    case EPI_KPLUS: launch_stencil_t<ST, GT, EPI_KPLUS>(c, a, U, nf, prec, true); break;
    default: throw Error{OVL_ERR_ARG, "stencil: epilogue"};
    }
}

void stencil(Context &c, int epi, int prec, const void *in, void *out, int nf, double rho,
             double sigma, const void *aux, double *partial, const int *stop, int it, const void *aux2,
             const int *itb)
{
    OVL_REQUIRE(c.have_gauge, OVL_ERR_STATE, "no gauge field loaded");
    if (prec == OVL_F64) {
        StencilArgs<double2> a{c.g, (const double2 *)in, (double2 *)out, (const double2 *)aux,
                               (const double2 *)aux2, 4.0 - rho, sigma, partial, stop, it, itb};
        stencil_epi(c, epi, a, c.U64, nf, prec);
    } else if (prec == OVL_F32) {
        StencilArgs<float4> a{c.g, (const float4 *)in, (float4 *)out, (const float4 *)aux,
                              (const float4 *)aux2, 4.0 - rho, sigma, partial, stop, it, itb};
        if (c.g.two_row)
            stencil_epi(c, epi, a, (const f2r12 *)c.U32r, nf, prec);
        else
            stencil_epi(c, epi, a, (const float2 *)c.U32, nf, prec);
    } else {
        StencilArgs<h8> a{c.g, (const h8 *)in, (h8 *)out, (const h8 *)aux, (const h8 *)aux2, 4.0 - rho,
                          sigma, partial, stop, it, itb};
        if (c.g.two_row)
            stencil_epi(c, epi, a, (const h2r12 *)c.U16r, nf, prec);
        else
            stencil_epi(c, epi, a, (const __half2 *)c.U16, nf, prec);
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
double stencil_link_bytes(const Geom &g, int prec)
{
    const int entries = (prec != OVL_F64 && g.two_row) ? 24 : 36;   // complex entries per site
    return (double)g.V * entries * (prec == OVL_F64 ? 16 : prec == OVL_F32 ? 8 : 4);
}

double stencil_bytes(const Geom &g, int prec, int epi)
{
    const double S = (double)field_bytes(g, prec);
    const double G = stencil_link_bytes(g, prec);
    double b = 2 * S + G;
    if (epi == EPI_KPLUS) b += S;
    if (epi == EPI_K2DOT) b += 2 * S;   // p and r
    return b;
}

}  // namespace ovl
