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
struct Geom {
    int32_t L[4];
    int64_t stride[4];
    int64_t V;
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
