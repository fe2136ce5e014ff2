// Device-side field access in the internal (packed) layouts.
//
// Spinor fields are site-major structure-of-arrays planes so that a wavefront
// of 64 consecutive sites reads each plane with one coalesced 16-byte load
// per lane:
//   FP64: double2 [12][V]   (plane c = spin*3 + colour holds one complex)
//   FP32: float4  [6][V]    (plane k holds complex components 2k, 2k+1)
//   HALF: uint4   [3][V]    (plane k holds 4 complex FP16 values, 4k..4k+3)
//         + float scale[V]  (the site's largest |real component|)
// Gauge fields (P = the padded plane stride, Geom::Pu):
//   FP64: double2 [4][9][P]   (one plane per complex entry and direction)
//   FP32: float4 [4][4][P] (entries 0..7 in pairs) + float2 [4][P] (entry 8)
//   HALF: uint4 [4][2][P] (entries 0..7 as __half2, four per uint4)
//         + uint32 [4][P] (entry 8)
#pragma once
#include <hip/hip_fp16.h>
#include <type_traits>

#include "common.h"

namespace ovl {

// ------------------------------------------------------------------ spinors
__device__ __forceinline__ void ld_sp(const double2 *__restrict__ p, int64_t V, int64_t s,
                                      cplx<double> v[12])
{
#pragma unroll
    for (int c = 0; c < 12; ++c) {
        double2 t = p[c * V + s];
        v[c] = {t.x, t.y};
    }
}
__device__ __forceinline__ void st_sp(double2 *__restrict__ p, int64_t V, int64_t s,
                                      const cplx<double> v[12])
{
#pragma unroll
    for (int c = 0; c < 12; ++c) p[c * V + s] = make_double2(v[c].re, v[c].im);
}
__device__ __forceinline__ void ld_sp(const float4 *__restrict__ p, int64_t V, int64_t s,
                                      cplx<float> v[12])
{
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        float4 t = p[k * V + s];
        v[2 * k] = {t.x, t.y};
        v[2 * k + 1] = {t.z, t.w};
    }
}
__device__ __forceinline__ void st_sp(float4 *__restrict__ p, int64_t V, int64_t s,
                                      const cplx<float> v[12])
{
#pragma unroll
    for (int k = 0; k < 6; ++k)
        p[k * V + s] = make_float4(v[2 * k].re, v[2 * k].im, v[2 * k + 1].re, v[2 * k + 1].im);
}

// Half of a spinor: spins 2h, 2h+1 (complex components 6h .. 6h+5).
__device__ __forceinline__ void ld_sp_half(const double2 *__restrict__ p, int64_t V, int64_t s, int h,
                                           cplx<double> v[6])
{
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        double2 t = p[(6 * h + c) * V + s];
        v[c] = {t.x, t.y};
    }
}
__device__ __forceinline__ void st_sp_half(double2 *__restrict__ p, int64_t V, int64_t s, int h,
                                           const cplx<double> v[6])
{
#pragma unroll
    for (int c = 0; c < 6; ++c) p[(6 * h + c) * V + s] = make_double2(v[c].re, v[c].im);
}
__device__ __forceinline__ void ld_sp_half(const float4 *__restrict__ p, int64_t V, int64_t s, int h,
                                           cplx<float> v[6])
{
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float4 t = p[(3 * h + k) * V + s];
        v[2 * k] = {t.x, t.y};
        v[2 * k + 1] = {t.z, t.w};
    }
}
__device__ __forceinline__ void st_sp_half(float4 *__restrict__ p, int64_t V, int64_t s, int h,
                                           const cplx<float> v[6])
{
#pragma unroll
    for (int k = 0; k < 3; ++k)
        p[(3 * h + k) * V + s] = make_float4(v[2 * k].re, v[2 * k].im, v[2 * k + 1].re, v[2 * k + 1].im);
}

// FP16 spinor storage: one h8 = 8 FP16 values = 4 complex numbers.  A field
// is [3][V] h8 planes followed by one FP32 scale per site (V floats, packed
// four per h8 slot): the site's 24 reals are stored divided by their largest
// magnitude (so every stored value is in [-1, 1]).
struct h8 {
    uint4 v;
};

// The values a spinor takes once stored: identity for FP64 / FP32 storage; for
// FP16 storage the per-site scaling and rounding of st_sp(h8).
__device__ __forceinline__ void as_stored(const double2 *, cplx<double> *, int) {}
__device__ __forceinline__ void as_stored(const float4 *, cplx<float> *, int) {}

// Number of storage elements of one field per site (planes).
template <typename ST> struct Planes;
template <> struct Planes<double2> { static constexpr int n = 12; using R = double; };
template <> struct Planes<float4> { static constexpr int n = 6; using R = float; };
template <> struct Planes<h8> { static constexpr int n = 3; using R = float; };

// Elements of ST between consecutive fields.
template <typename ST> __host__ __device__ __forceinline__ int64_t fstride(int64_t V)
{
    return (int64_t)Planes<ST>::n * V;
}
template <> __host__ __device__ __forceinline__ int64_t fstride<h8>(int64_t V) { return 3 * V + V / 4; }

__device__ __forceinline__ float2 h2f2(uint32_t w)
{
    __half2 h = *reinterpret_cast<__half2 *>(&w);
    return __half22float2(h);
}
__device__ __forceinline__ uint32_t f22h2(float a, float b)
{
    __half2 h = __floats2half2_rn(a, b);
    return *reinterpret_cast<uint32_t *>(&h);
}

// 1 / m for an FP16-stored site whose largest |real component| is m.  A
// site with m below the smallest normal float is stored as zero (m set to 0):
// 1 / m would overflow to infinity there (such values occur at the edge of the
// support of Krylov vectors grown from a point source).
__device__ __forceinline__ float h8_inv_scale(float &m)
{
    if (!(m >= 0x1p-126f)) {
        m = 0.f;
        return 0.f;
    }
    return 1.f / m;
}

__device__ __forceinline__ void as_stored(const h8 *, cplx<float> *v, int n)
{
    float m = 0.f;
    for (int c = 0; c < n; ++c) m = fmaxf(m, fmaxf(fabsf(v[c].re), fabsf(v[c].im)));
    const float inv = h8_inv_scale(m);
    for (int c = 0; c < n; ++c) {
        const float2 q = h2f2(f22h2(v[c].re * inv, v[c].im * inv));
        v[c] = {q.x * m, q.y * m};
    }
}

__device__ __forceinline__ void ld_sp(const h8 *__restrict__ p, int64_t V, int64_t s, cplx<float> v[12])
{
    const float sc = reinterpret_cast<const float *>(p + 3 * V)[s];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const uint4 t = p[k * V + s].v;
        const float2 a = h2f2(t.x), b = h2f2(t.y), c = h2f2(t.z), d = h2f2(t.w);
        v[4 * k] = {a.x * sc, a.y * sc};
        v[4 * k + 1] = {b.x * sc, b.y * sc};
        v[4 * k + 2] = {c.x * sc, c.y * sc};
        v[4 * k + 3] = {d.x * sc, d.y * sc};
    }
}
__device__ __forceinline__ void st_sp(h8 *__restrict__ p, int64_t V, int64_t s, const cplx<float> v[12])
{
    float m = 0.f;
#pragma unroll
    for (int c = 0; c < 12; ++c) m = fmaxf(m, fmaxf(fabsf(v[c].re), fabsf(v[c].im)));
    const float inv = h8_inv_scale(m);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        uint4 t;
        t.x = f22h2(v[4 * k].re * inv, v[4 * k].im * inv);
        t.y = f22h2(v[4 * k + 1].re * inv, v[4 * k + 1].im * inv);
        t.z = f22h2(v[4 * k + 2].re * inv, v[4 * k + 2].im * inv);
        t.w = f22h2(v[4 * k + 3].re * inv, v[4 * k + 3].im * inv);
        p[k * V + s].v = t;
    }
    reinterpret_cast<float *>(p + 3 * V)[s] = m;
}

// One site's spinor as stored, for loads issued well before their values are
// needed (sp_values then gives what ld_sp would have).
template <typename ST> struct SpStored;
template <> struct SpStored<double2> { double2 q[12]; };
template <> struct SpStored<float4> { float4 q[6]; };
template <> struct SpStored<h8> { uint4 q[3]; float sc; };

template <typename ST>
__device__ __forceinline__ void ld_sp_stored(const ST *__restrict__ p, int64_t V, int64_t s, SpStored<ST> &r)
{
    if constexpr (std::is_same<ST, h8>::value) {
#pragma unroll
        for (int k = 0; k < 3; ++k) r.q[k] = p[k * V + s].v;
        r.sc = reinterpret_cast<const float *>(p + 3 * V)[s];
    } else {
#pragma unroll
        for (int k = 0; k < Planes<ST>::n; ++k) r.q[k] = p[k * V + s];
    }
}
__device__ __forceinline__ void sp_values(const SpStored<double2> &r, cplx<double> v[12])
{
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = {r.q[c].x, r.q[c].y};
}
__device__ __forceinline__ void sp_values(const SpStored<float4> &r, cplx<float> v[12])
{
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        v[2 * k] = {r.q[k].x, r.q[k].y};
        v[2 * k + 1] = {r.q[k].z, r.q[k].w};
    }
}
__device__ __forceinline__ void sp_values(const SpStored<h8> &r, cplx<float> v[12])
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

// Half of an FP16-stored spinor (two lanes per site): half 0 holds complex
// components 0..5 (plane 0 and the low half of plane 1), half 1 components
// 6..11 (the high half of plane 1 and plane 2).  The site's scale is shared,
// so the store takes it (the larger of both halves' maxima) as an argument;
// half 0 writes it.
__device__ __forceinline__ void ld_sp_half(const h8 *__restrict__ p, int64_t V, int64_t s, int h,
                                           cplx<float> v[6])
{
    const float sc = reinterpret_cast<const float *>(p + 3 * V)[s];
    const uint2 mid = reinterpret_cast<const uint2 *>(p + V + s)[h];
    const uint4 q = p[(h == 0 ? 0 : 2) * V + s].v;
    const uint32_t w[6] = {h == 0 ? q.x : mid.x, h == 0 ? q.y : mid.y, h == 0 ? q.z : q.x,
                           h == 0 ? q.w : q.y, h == 0 ? mid.x : q.z, h == 0 ? mid.y : q.w};
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const float2 a = h2f2(w[c]);
        v[c] = {a.x * sc, a.y * sc};
    }
}
__device__ __forceinline__ float half_max(const cplx<float> v[6])
{
    float m = 0.f;
#pragma unroll
    for (int c = 0; c < 6; ++c) m = fmaxf(m, fmaxf(fabsf(v[c].re), fabsf(v[c].im)));
    return m;
}
// the values st_sp_half_scaled stores, with the site scale m
__device__ __forceinline__ void as_stored_scaled(cplx<float> v[6], float m)
{
    const float inv = h8_inv_scale(m);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const float2 q = h2f2(f22h2(v[c].re * inv, v[c].im * inv));
        v[c] = {q.x * m, q.y * m};
    }
}
__device__ __forceinline__ void st_sp_half_scaled(h8 *__restrict__ p, int64_t V, int64_t s, int h,
                                                  const cplx<float> v[6], float m)
{
    const float inv = h8_inv_scale(m);
    uint32_t w[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) w[c] = f22h2(v[c].re * inv, v[c].im * inv);
    if (h == 0) {
        p[s].v = make_uint4(w[0], w[1], w[2], w[3]);
        reinterpret_cast<uint2 *>(p + V + s)[0] = make_uint2(w[4], w[5]);
        reinterpret_cast<float *>(p + 3 * V)[s] = m;
    } else {
        reinterpret_cast<uint2 *>(p + V + s)[1] = make_uint2(w[0], w[1]);
        p[2 * V + s].v = make_uint4(w[2], w[3], w[4], w[5]);
    }
}

// ------------------------------------------------------------------ links
// Link planes [mu][9][P], P the padded plane stride (Geom::Pu).
__device__ __forceinline__ void ld_link(const double2 *__restrict__ U, int64_t P, int mu,
                                        int64_t s, cplx<double> u[9])
{
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        double2 t = U[(mu * 9 + k) * P + s];
        u[k] = {t.x, t.y};
    }
}
// FP32 links: the eight entries 0..7 of a link as four float4 planes per
// direction, Q [4 mu][4][P], followed by entry 8 as float2 planes R [4 mu][P]
// (five loads per link instead of nine).
__device__ __forceinline__ void ld_link(const float2 *__restrict__ U, int64_t P, int mu,
                                        int64_t s, cplx<float> u[9])
{
    const float4 *Q = reinterpret_cast<const float4 *>(U);
    const float2 *R = reinterpret_cast<const float2 *>(Q + 16 * P);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float4 q = Q[(mu * 4 + k) * P + s];
        u[2 * k] = {q.x, q.y};
        u[2 * k + 1] = {q.z, q.w};
    }
    const float2 r = R[mu * P + s];
    u[8] = {r.x, r.y};
}

// FP16 links: one __half2 per complex entry (entries of a unitary matrix have
// modulus <= 1, so no scale is needed); entries 0..7 as two uint4 planes per
// direction, Q [4 mu][2][P], followed by entry 8 as uint32 planes R [4 mu][P]
// (three loads per link).
__device__ __forceinline__ void ld_link(const __half2 *__restrict__ U, int64_t P, int mu,
                                        int64_t s, cplx<float> u[9])
{
    const uint4 *Q = reinterpret_cast<const uint4 *>(U);
    const uint32_t *R = reinterpret_cast<const uint32_t *>(Q + 8 * P);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const uint4 q = Q[(mu * 2 + k) * P + s];
        const float2 a = h2f2(q.x), b = h2f2(q.y), c = h2f2(q.z), d = h2f2(q.w);
        u[4 * k] = {a.x, a.y};
        u[4 * k + 1] = {b.x, b.y};
        u[4 * k + 2] = {c.x, c.y};
        u[4 * k + 3] = {d.x, d.y};
    }
    const float2 r = h2f2(R[mu * P + s]);
    u[8] = {r.x, r.y};
}

// Two-row links.  For a link in SU(3) the third row is the complex conjugate
// of the cross product of the first two, so the FP32 and FP16 stencils can
// read 12 reals per link and rebuild the rest; the context keeps this form
// beside the full one and uses it when every loaded link passes an SU(3)
// test.  The tag types (the size of one stored complex entry) select the
// loaders below; their planes: FP32 entries 0..3 as two float4 planes per
// direction, Q [4 mu][2][P], then entries 4, 5 as one float4 plane R [4 mu][P]
// (three loads per link); FP16 entries 0..3 as one uint4 plane Q [4 mu][1][P],
// then entries 4, 5 as one uint2 plane R [4 mu][P] (two loads per link).
struct f2r12 {
    float2 v;
};
struct h2r12 {
    __half2 v;
};
template <typename GT>
struct is_two_row {
    static constexpr bool value = std::is_same<GT, f2r12>::value || std::is_same<GT, h2r12>::value;
};

// u[6..8] = conj(u[0..2] x u[3..5]), row-major u[a * 3 + b]
template <typename R>
__device__ __forceinline__ void su3_third_row(cplx<R> u[9])
{
    const cplx<R> c0 = u[1] * u[5] - u[2] * u[4];
    const cplx<R> c1 = u[2] * u[3] - u[0] * u[5];
    const cplx<R> c2 = u[0] * u[4] - u[1] * u[3];
    u[6] = {c0.re, -c0.im};
    u[7] = {c1.re, -c1.im};
    u[8] = {c2.re, -c2.im};
}

__device__ __forceinline__ void ld_link(const f2r12 *__restrict__ U, int64_t P, int mu, int64_t s,
                                        cplx<float> u[9])
{
    const float4 *Q = reinterpret_cast<const float4 *>(U);
    const float4 *R = Q + 8 * P;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const float4 q = Q[(mu * 2 + k) * P + s];
        u[2 * k] = {q.x, q.y};
        u[2 * k + 1] = {q.z, q.w};
    }
    const float4 r = R[mu * P + s];
    u[4] = {r.x, r.y};
    u[5] = {r.z, r.w};
    su3_third_row(u);
}

__device__ __forceinline__ void ld_link(const h2r12 *__restrict__ U, int64_t P, int mu, int64_t s,
                                        cplx<float> u[9])
{
    const uint4 *Q = reinterpret_cast<const uint4 *>(U);
    const uint2 *R = reinterpret_cast<const uint2 *>(Q + 4 * P);
    const uint4 q = Q[mu * P + s];
    const float2 a = h2f2(q.x), b = h2f2(q.y), c = h2f2(q.z), d = h2f2(q.w);
    u[0] = {a.x, a.y};
    u[1] = {b.x, b.y};
    u[2] = {c.x, c.y};
    u[3] = {d.x, d.y};
    const uint2 r = R[mu * P + s];
    const float2 e = h2f2(r.x), f = h2f2(r.y);
    u[4] = {e.x, e.y};
    u[5] = {f.x, f.y};
    su3_third_row(u);
}

// ------------------------------------------------------------------ spin algebra
// Chiral basis: gamma_mu = [[0, A_mu], [B_mu, 0]] in 2x2 spin blocks with
// A_k = -i s_k, B_k = i s_k = -A_k (k = x, y, z), A_t = B_t = 1, A B = 1.
// (1 -+ gamma_mu) psi: upper = h = psi_u -+ A psi_d, lower = -+ B h.
// apply_A: w = A_mu v for a 2-spinor (v0, v1) of colour vectors, component-wise.
template <int MU, typename R>
__device__ __forceinline__ void apply_A(const cplx<R> &v0, const cplx<R> &v1, cplx<R> &w0,
                                        cplx<R> &w1)
{
    if constexpr (MU == 0) {          // -i s_x: (-i v1, -i v0)
        w0 = times_mi(v1);
        w1 = times_mi(v0);
    } else if constexpr (MU == 1) {   // -i s_y: (-v1, v0)
        w0 = -v1;
        w1 = v0;
    } else if constexpr (MU == 2) {   // -i s_z: (-i v0, i v1)
        w0 = times_mi(v0);
        w1 = times_i(v1);
    } else {                          // 1
        w0 = v0;
        w1 = v1;
    }
}

// The three parts of a hop, FWD = true: (1 - gamma_mu) U_mu(x) psi(x + mu);
// FWD = false: (1 + gamma_mu) U_mu(x - mu)^+ psi(x - mu).
// spin_proj: h = upper half of (1 -+ gamma_mu) psi = psi_up -+ A psi_down
template <int MU, bool FWD, typename R>
__device__ __forceinline__ void spin_proj(const cplx<R> psi[12], cplx<R> h[6])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        cplx<R> a0, a1;
        apply_A<MU>(psi[6 + c], psi[9 + c], a0, a1);
        if constexpr (FWD) {
            h[c] = psi[c] - a0;
            h[3 + c] = psi[3 + c] - a1;
        } else {
            h[c] = psi[c] + a0;
            h[3 + c] = psi[3 + c] + a1;
        }
    }
}

// link_mul: g = W h (FWD) or W^+ h, per spin of the half spinor
template <bool FWD, typename R>
__device__ __forceinline__ void link_mul(const cplx<R> u[9], const cplx<R> h[6], cplx<R> g[6])
{
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cplx<R> t;
            if constexpr (FWD) {
                t = u[a * 3 + 0] * h[sp * 3 + 0];
                t = t + u[a * 3 + 1] * h[sp * 3 + 1];
                t = t + u[a * 3 + 2] * h[sp * 3 + 2];
            } else {
                t = cmul_conj(u[0 * 3 + a], h[sp * 3 + 0]);
                t = t + cmul_conj(u[1 * 3 + a], h[sp * 3 + 1]);
                t = t + cmul_conj(u[2 * 3 + a], h[sp * 3 + 2]);
            }
            g[sp * 3 + a] = t;
        }
}

// spin_recon: acc += the full spinor whose upper half is g (lower half
// -B g for FWD, B g otherwise)
template <int MU, bool FWD, typename R>
__device__ __forceinline__ void spin_recon(const cplx<R> g[6], cplx<R> acc[12])
{
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        acc[c] = acc[c] + g[c];
        acc[3 + c] = acc[3 + c] + g[3 + c];
        if constexpr (MU == 3) {
            if constexpr (FWD) {          // lower = -g
                acc[6 + c] = acc[6 + c] - g[c];
                acc[9 + c] = acc[9 + c] - g[3 + c];
            } else {                      // lower = +g
                acc[6 + c] = acc[6 + c] + g[c];
                acc[9 + c] = acc[9 + c] + g[3 + c];
            }
        } else {
            cplx<R> a0, a1;
            apply_A<MU>(g[c], g[3 + c], a0, a1);
            if constexpr (FWD) {          // lower = -B g = A g
                acc[6 + c] = acc[6 + c] + a0;
                acc[9 + c] = acc[9 + c] + a1;
            } else {                      // lower = B g = -A g
                acc[6 + c] = acc[6 + c] - a0;
                acc[9 + c] = acc[9 + c] - a1;
            }
        }
    }
}

// acc += (1 - gamma_mu) W psi_fwd   (FWD = true,  W = U_mu(x))
// acc += (1 + gamma_mu) W^+ psi_bwd (FWD = false, W = U_mu(x - mu))
template <int MU, bool FWD, typename R>
__device__ __forceinline__ void hop_term(const cplx<R> psi[12], const cplx<R> u[9], cplx<R> acc[12])
{
    cplx<R> h[6], g[6];
    spin_proj<MU, FWD>(psi, h);
    link_mul<FWD>(u, h, g);
    spin_recon<MU, FWD>(g, acc);
}

// ------------------------------------------------------------------ FP16 hops on packed halves
// With FP16 storage the hop runs on the stored halves: the spin projection as
// packed FP16 adds (a site's components are at most 1 in modulus after its
// scale, so the projection is at most 2), the link product as two-term FP16
// dot products accumulated in FP32 (each half product is exact in FP32), the
// neighbour's scale applied to the product, the spin reconstruction and the
// sum over directions in FP32.  This halves the vector instructions of a hop
// against converting everything to FP32 first.
typedef _Float16 hv2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ hv2 as_hv2(uint32_t w) { return __builtin_bit_cast(hv2, w); }

// d = w.x h.x + w.y h.y + c with the half products exact in FP32
// (v_dot2_f32_f16; through the builtin, so that the compiler schedules it).
__device__ __forceinline__ float dot2(hv2 w, hv2 h, float c) { return __builtin_amdgcn_fdot2(w, h, c, false); }

// an FP16-stored site: its 12 components as packed halves, and its scale
__device__ __forceinline__ void ld_sp_h(const h8 *__restrict__ p, int64_t V, int64_t s, hv2 w[12], float &sc)
{
    sc = reinterpret_cast<const float *>(p + 3 * V)[s];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const uint4 t = p[k * V + s].v;
        w[4 * k] = as_hv2(t.x);
        w[4 * k + 1] = as_hv2(t.y);
        w[4 * k + 2] = as_hv2(t.z);
        w[4 * k + 3] = as_hv2(t.w);
    }
}

// FP16 links as packed halves (the planes of ld_link)
__device__ __forceinline__ void ld_link_h(const __half2 *__restrict__ U, int64_t P, int mu, int64_t s, hv2 u[9])
{
    const uint4 *Q = reinterpret_cast<const uint4 *>(U);
    const uint32_t *R = reinterpret_cast<const uint32_t *>(Q + 8 * P);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const uint4 q = Q[(mu * 2 + k) * P + s];
        u[4 * k] = as_hv2(q.x);
        u[4 * k + 1] = as_hv2(q.y);
        u[4 * k + 2] = as_hv2(q.z);
        u[4 * k + 3] = as_hv2(q.w);
    }
    u[8] = as_hv2(R[mu * P + s]);
}
// conj(x y - z w) for complex halves, rounded to half
__device__ __forceinline__ hv2 conj_cross_h(hv2 x, hv2 y, hv2 z, hv2 w)
{
    const float re = dot2(z, (hv2){-w.x, w.y}, dot2(x, (hv2){y.x, -y.y}, 0.f));
    const float im = dot2(z, -w.yx, dot2(x, y.yx, 0.f));
    return (hv2){(_Float16)re, (_Float16)(-im)};
}
__device__ __forceinline__ void ld_link_h(const h2r12 *__restrict__ U, int64_t P, int mu, int64_t s, hv2 u[9])
{
    const uint4 *Q = reinterpret_cast<const uint4 *>(U);
    const uint2 *R = reinterpret_cast<const uint2 *>(Q + 4 * P);
    const uint4 q = Q[mu * P + s];
    u[0] = as_hv2(q.x);
    u[1] = as_hv2(q.y);
    u[2] = as_hv2(q.z);
    u[3] = as_hv2(q.w);
    const uint2 r = R[mu * P + s];
    u[4] = as_hv2(r.x);
    u[5] = as_hv2(r.y);
    u[6] = conj_cross_h(u[1], u[5], u[2], u[4]);
    u[7] = conj_cross_h(u[2], u[3], u[0], u[5]);
    u[8] = conj_cross_h(u[0], u[4], u[1], u[3]);
}

template <int MU>
__device__ __forceinline__ void apply_A_h(hv2 v0, hv2 v1, hv2 &w0, hv2 &w1)
{
    if constexpr (MU == 0) {          // -i s_x: (-i v1, -i v0)
        w0 = (hv2){v1.y, -v1.x};
        w1 = (hv2){v0.y, -v0.x};
    } else if constexpr (MU == 1) {   // -i s_y: (-v1, v0)
        w0 = -v1;
        w1 = v0;
    } else if constexpr (MU == 2) {   // -i s_z: (-i v0, i v1)
        w0 = (hv2){v0.y, -v0.x};
        w1 = (hv2){-v1.y, v1.x};
    } else {                          // 1
        w0 = v0;
        w1 = v1;
    }
}

// hop_term on packed halves: psi the neighbour's stored components and sc its
// scale, u the link (W = U_mu(x) for FWD, U_mu(x - mu) otherwise)
template <int MU, bool FWD>
__device__ __forceinline__ void hop_term_h(const hv2 psi[12], float sc, const hv2 u[9], cplx<float> acc[12])
{
    // With h = psi_up -+ A psi_down (the upper half of (1 -+ gamma_mu) psi):
    // W h = sum_b W_ab h_b: re = dot2(W_ab, (h.x, -h.y)), im = dot2(W_ab, (h.y, h.x));
    // W^+ h = sum_b conj(W_ba) h_b: re = dot2(W_ba, h), im = dot2(W_ba, (h.y, -h.x)).
    // Each operand form is one packed add of psi_up and A psi_down, written
    // out from the two (not from h) so that the swaps and signs become its
    // source modifiers.
    hv2 pr[6], pi[6];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            hv2 a0, a1;
            apply_A_h<MU>(psi[6 + c], psi[9 + c], a0, a1);
            const hv2 up = psi[3 * k + c], ad = k == 0 ? a0 : a1;
            if constexpr (FWD) {   // h = up - ad
                pr[3 * k + c] = (hv2){up.x, -up.y} - (hv2){ad.x, -ad.y};
                pi[3 * k + c] = (hv2){up.y, up.x} - (hv2){ad.y, ad.x};
            } else {               // h = up + ad
                pr[3 * k + c] = up + ad;
                pi[3 * k + c] = (hv2){up.y, -up.x} + (hv2){ad.y, -ad.x};
            }
        }
    cplx<float> g[6];   // W h (FWD) or W^+ h, times the neighbour's scale
#pragma unroll
    for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            float re = 0.f, im = 0.f;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const hv2 W = FWD ? u[a * 3 + b] : u[b * 3 + a];
                re = dot2(W, pr[sp * 3 + b], re);
                im = dot2(W, pi[sp * 3 + b], im);
            }
            g[sp * 3 + a] = {sc * re, sc * im};
        }
    spin_recon<MU, FWD>(g, acc);
}

// ------------------------------------------------------------------ block -> tile mapping
// Work-groups are handed to the eight XCDs round-robin by linear id.  With
// REMAP, each XCD receives a contiguous range of logical ids, so neighbouring
// site tiles (and the fields of one tile, which share its links) run on the
// same XCD and meet in its L2.  Logical id -> (site tile, field), field
// fastest.
template <bool REMAP>
__device__ __forceinline__ void tile_of_block(unsigned &tile, unsigned &field)
{
    const unsigned X = gridDim.x, Y = gridDim.y, B = X * Y;
    const unsigned lin = blockIdx.y * X + blockIdx.x;
    unsigned lid = lin;
    if constexpr (REMAP) {
        const unsigned q = B / 8, r = B % 8, x = lin % 8, k = lin / 8;
        lid = x * q + (x < r ? x : r) + k;
    }
    tile = lid / Y;
    field = lid % Y;
}

// ------------------------------------------------------------------ reductions
// Sum over a 64-lane wavefront, then over the block through LDS.  Every
// thread of the block must call it; the result is valid in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *lds)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) r += lds[w];
    }
    return r;
}

}  // namespace ovl
