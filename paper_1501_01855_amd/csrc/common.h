// Internal declarations of the overlap library (gfx950 / HIP).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/ovl.h"

namespace ovl {

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);

struct Error {
    ovl_status code;
    std::string msg;
};

#define OVL_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            throw ::ovl::Error{OVL_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

#define OVL_REQUIRE(cond, code, msg)                                                    \
    do {                                                                                \
        if (!(cond)) throw ::ovl::Error{code, msg};                                     \
    } while (0)

// ---------------------------------------------------------------- complex
template <typename R>
struct cplx {
    R re, im;
};

template <typename R>
__host__ __device__ inline cplx<R> cmk(R a, R b) { return cplx<R>{a, b}; }
template <typename R>
__host__ __device__ inline cplx<R> operator+(cplx<R> a, cplx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__host__ __device__ inline cplx<R> operator-(cplx<R> a, cplx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__host__ __device__ inline cplx<R> operator-(cplx<R> a) { return {-a.re, -a.im}; }
template <typename R>
__host__ __device__ inline cplx<R> operator*(cplx<R> a, cplx<R> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__host__ __device__ inline cplx<R> operator*(R s, cplx<R> a) { return {s * a.re, s * a.im}; }
// conj(a) * b
template <typename R>
__host__ __device__ inline cplx<R> cmul_conj(cplx<R> a, cplx<R> b)
{
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// i * a, -i * a
template <typename R>
__host__ __device__ inline cplx<R> times_i(cplx<R> a) { return {-a.im, a.re}; }
template <typename R>
__host__ __device__ inline cplx<R> times_mi(cplx<R> a) { return {a.im, -a.re}; }

// ---------------------------------------------------------------- geometry
// Column blocking of the x, y, z extents for the XCD-aware stencil launch:
// the xyz volume is cut into 8 columns of cb[0] x cb[1] x cb[2] sites
// (cn[m] columns along m), each column running through all of t.  col_ok is
// false when no split into 8 columns divides the extents.
// Link planes ([mu][9][Pu]) are Pu = V + LINK_PAD sites apart, not V: with a
// power-of-two V the 36 planes of a site would otherwise sit a power of two
// apart and compete for the same L2 sets and memory channels.
constexpr int64_t LINK_PAD = 544;   // 17 x 32 sites: an odd number of 128 B lines for 8 B entries

struct Geom {
    int32_t L[4];
    int64_t stride[4];
    int64_t V;
    int64_t Pu;          // link plane stride (sites)
    int32_t cb[3], cn[3];
    int32_t col_sites;   // cb[0] cb[1] cb[2]
    int32_t col_ok;
    int32_t two_row;     // FP32 / FP16 stencils read the two-row links (set when the links are loaded)
};

inline Geom make_geom(const int32_t d[4])
{
    Geom g;
    int64_t s = 1;
    for (int m = 0; m < 4; ++m) {
        g.L[m] = d[m];
        g.stride[m] = s;
        s *= d[m];
    }
    g.V = s;
    g.Pu = s + LINK_PAD;
    g.two_row = 0;
    // the split into 8 = cx cy cz columns with the smallest halo: a cut face
    // along m re-reads 2 / cb[m] of the column's sites, a cut along x whole
    // 128-byte lines (8 sites) per row end, so x rows stay whole if possible
    g.col_ok = 0;
    double best = 1e30;
    for (int cx = 1; cx <= 8; cx *= 2)
        for (int cy = 1; cx * cy <= 8; cy *= 2) {
            const int cz = 8 / (cx * cy);
            const int c[3] = {cx, cy, cz};
            bool ok = true;
            int b[3];
            for (int m = 0; m < 3; ++m) {
                ok = ok && d[m] % c[m] == 0;
                b[m] = ok ? d[m] / c[m] : 0;
            }
            if (!ok || b[0] < 4) continue;
            double cost = 0.0;
            for (int m = 0; m < 3; ++m)
                if (c[m] > 1) cost += (m == 0 ? 16.0 : 2.0) / b[m];
            cost -= 1e-6 * b[2];   // ties: deeper columns in z
            if (cost < best) {
                best = cost;
                g.col_ok = 1;
                for (int m = 0; m < 3; ++m) {
                    g.cb[m] = b[m];
                    g.cn[m] = c[m];
                }
            }
        }
    if (!g.col_ok)
        for (int m = 0; m < 3; ++m) g.cb[m] = g.cn[m] = 1;
    g.col_sites = g.cb[0] * g.cb[1] * g.cb[2];
    return g;
}

// ---------------------------------------------------------------- device buffers
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

// Half-precision spinor storage: 12 complex FP16 values per site in three
// 16-byte planes plus one FP32 scale per site (max-abs of the site's reals).
struct HalfSpinorPtr {
    uint4 *data;   // [3][V]
    float *scale;  // [V]
};

enum Kern { KERN_STENCIL = 0, KERN_SHIFT = 1, KERN_COUNT = 2 };

struct ProfileSlot {
    int64_t launches = 0;
    double ms = 0.0;
    double bytes = 0.0;
};

struct Context;  // defined in context.hip

}  // namespace ovl
