// Seeded generation of gauge fields and sources on the GPU.
//
// The recipe (Philox4x32-10 counters, 53-bit uniforms, Box-Muller with
// series for ln, sin and cos, U = exp(i eps sum_a g_a T^a) by a degree-14
// Taylor polynomial of X/16 squared four times) is written as a fixed
// sequence of IEEE operations, and this file is compiled without
// floating-point contraction, so the fields are bit-identical to the host
// reference generator that uses the same recipe.
#include "context.h"
#include "ops.h"

namespace ovl {

namespace gen {

constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
constexpr uint32_t TAG_GAUGE = 0x47415547u, TAG_GAUSS = 0x53524347u, TAG_Z2 = 0x5A32534Eu;
constexpr double LN2 = 0.6931471805599453;
constexpr double PI_4 = 0.7853981633974483;
constexpr double INV_SQRT3 = 0.5773502691896258;

struct W4 {
    uint32_t w[4];
};

__device__ W4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t seed)
{
    uint32_t k0 = (uint32_t)(seed & 0xFFFFFFFFu), k1 = (uint32_t)(seed >> 32);
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(M0, c0), lo0 = M0 * c0;
        const uint32_t hi1 = __umulhi(M1, c2), lo1 = M1 * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
        if (r < 9) {
            k0 += W0;
            k1 += W1;
        }
    }
    return W4{{c0, c1, c2, c3}};
}

__device__ double uniform53(uint32_t w0, uint32_t w1)
{
    const double a = (double)(w0 >> 5), b = (double)(w1 >> 6);
    return (a * 67108864.0 + b) * (1.0 / 9007199254740992.0);
}

__device__ double log_unit(double u)
{
    int ei;
    double m = frexp(u, &ei);
    double e = (double)ei;
    if (m < 0.7071067811865476) {
        m = m * 2.0;
        e = (double)(ei - 1);
    }
    const double z = (m - 1.0) / (m + 1.0);
    const double z2 = z * z;
    double s = 1.0 / 25.0;
#pragma unroll
    for (int k = 11; k >= 0; --k) s = (1.0 / (2 * k + 1)) + z2 * s;
    return e * LN2 + (2.0 * z) * s;
}

__device__ double sin_poly(double t)
{
    const double t2 = t * t;
    double s = 1.0;
#pragma unroll
    for (int k = 10; k >= 1; --k) s = 1.0 - (t2 * (1.0 / ((2 * k) * (2 * k + 1)))) * s;
    return t * s;
}

__device__ double cos_poly(double t)
{
    const double t2 = t * t;
    double s = 1.0;
#pragma unroll
    for (int k = 10; k >= 1; --k) s = 1.0 - (t2 * (1.0 / ((2 * k - 1) * (2 * k)))) * s;
    return s;
}

__device__ void sincos_2pi(double u, double &s, double &c)
{
    const double v = u * 8.0;
    const double kf = floor(v);
    const double f = v - kf;
    const int k = (int)kf;
    const bool odd = (k & 1) != 0;
    const double t = (odd ? 1.0 - f : f) * PI_4;
    const double st = sin_poly(t), ct = cos_poly(t);
    const double sa = odd ? ct : st, ca = odd ? st : ct;
    switch (k >> 1) {
    case 0: s = sa; c = ca; break;
    case 1: s = ca; c = -sa; break;
    case 2: s = -sa; c = -ca; break;
    default: s = -ca; c = sa; break;
    }
}

__device__ void normal_pair(uint32_t index, uint32_t draw, uint32_t tag, uint64_t seed, double &za, double &zb)
{
    const W4 w = philox(index, draw, tag, 0u, seed);
    const double ua = uniform53(w.w[0], w.w[1]), ub = uniform53(w.w[2], w.w[3]);
    const double r = sqrt(-2.0 * log_unit(1.0 - ua));
    double s, c;
    sincos_2pi(ub, s, c);
    za = r * c;
    zb = r * s;
}

// C = A B for 3x3 complex matrices (separate re / im), summation k = 0, 1, 2.
__device__ void cmatmul3(const double ar[9], const double ai[9], const double br[9], const double bi[9],
                         double cr[9], double ci[9])
{
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double sr = ar[i * 3] * br[j] - ai[i * 3] * bi[j];
            double si = ar[i * 3] * bi[j] + ai[i * 3] * br[j];
#pragma unroll
            for (int k = 1; k < 3; ++k) {
                sr = sr + (ar[i * 3 + k] * br[k * 3 + j] - ai[i * 3 + k] * bi[k * 3 + j]);
                si = si + (ar[i * 3 + k] * bi[k * 3 + j] + ai[i * 3 + k] * br[k * 3 + j]);
            }
            cr[i * 3 + j] = sr;
            ci[i * 3 + j] = si;
        }
}

__global__ void k_gauge(double2 *__restrict__ U, int64_t nlink, uint64_t seed, double eps)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nlink) return;
    double g[8];
    for (int d = 0; d < 4; ++d) normal_pair((uint32_t)i, (uint32_t)d, TAG_GAUGE, seed, g[2 * d], g[2 * d + 1]);
    const double h = 0.5 * eps;
    double a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = g[k] * h;
    double Ar[9], Ai[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        Ar[k] = 0.0;
        Ai[k] = 0.0;
    }
    Ar[0] = a[2] + a[7] * INV_SQRT3;
    Ar[4] = (0.0 - a[2]) + a[7] * INV_SQRT3;
    Ar[8] = a[7] * (-2.0 * INV_SQRT3);
    Ar[1] = a[0];
    Ai[1] = 0.0 - a[1];
    Ar[3] = a[0];
    Ai[3] = a[1];
    Ar[2] = a[3];
    Ai[2] = 0.0 - a[4];
    Ar[6] = a[3];
    Ai[6] = a[4];
    Ar[5] = a[5];
    Ai[5] = 0.0 - a[6];
    Ar[7] = a[5];
    Ai[7] = a[6];
    // X = i A, scaled by 1/16
    double xr[9], xi[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        xr[k] = (0.0 - Ai[k]) * (1.0 / 16.0);
        xi[k] = Ar[k] * (1.0 / 16.0);
    }
    double pr[9], pi[9], tr[9], ti[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        pr[k] = (k % 4 == 0) ? 1.0 : 0.0;
        pi[k] = 0.0;
    }
    constexpr double INV[15] = {0.0,       1.0 / 1,  1.0 / 2,  1.0 / 3,  1.0 / 4,
                                1.0 / 5,   1.0 / 6,  1.0 / 7,  1.0 / 8,  1.0 / 9,
                                1.0 / 10,  1.0 / 11, 1.0 / 12, 1.0 / 13, 1.0 / 14};
    for (int k = 14; k >= 1; --k) {
        cmatmul3(xr, xi, pr, pi, tr, ti);
        const double inv = INV[k];
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            pr[e] = ((e % 4 == 0) ? 1.0 : 0.0) + tr[e] * inv;
            pi[e] = ti[e] * inv;
        }
    }
    for (int q = 0; q < 4; ++q) {
        cmatmul3(pr, pi, pr, pi, tr, ti);
#pragma unroll
        for (int e = 0; e < 9; ++e) {
            pr[e] = tr[e];
            pi[e] = ti[e];
        }
    }
#pragma unroll
    for (int e = 0; e < 9; ++e) U[i * 9 + e] = make_double2(pr[e], pi[e]);
}

__global__ void k_source(double2 *__restrict__ out, int64_t n, int kind, uint64_t seed, int64_t hot)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double re = 0.0, im = 0.0;
    if (kind == OVL_SRC_POINT) {
        re = (i == hot) ? 1.0 : 0.0;
    } else if (kind == OVL_SRC_GAUSS) {
        normal_pair((uint32_t)i, 0u, TAG_GAUSS, seed, re, im);
    } else {
        const W4 w = philox((uint32_t)i, 0u, TAG_Z2, 0u, seed);
        re = 1.0 - 2.0 * (double)(w.w[0] & 1u);
        im = 1.0 - 2.0 * (double)(w.w[1] & 1u);
    }
    out[i] = make_double2(re, im);
}

}  // namespace gen

void gauge_generate(Context &c, uint64_t seed, double eps, double *canon_out)
{
    const int64_t nlink = 4 * c.g.V;
    double2 *U = canon_out ? (double2 *)canon_out : (double2 *)c.buf("gen_U", (size_t)nlink * 9 * sizeof(double2));
    gen::k_gauge<<<(unsigned)((nlink + 127) / 128), 128, 0, c.stream>>>(U, nlink, seed, eps);
    OVL_HIP(hipGetLastError());
    pack_gauge(c, (const double *)U);
}

void source_generate(Context &c, int kind, uint64_t seed, int64_t site, int spin, int colour, double *canon_out)
{
    const int64_t n = 12 * c.g.V;
    const int64_t hot = site * 12 + spin * 3 + colour;
    gen::k_source<<<(unsigned)((n + 255) / 256), 256, 0, c.stream>>>((double2 *)canon_out, n, kind, seed, hot);
    OVL_HIP(hipGetLastError());
}

}  // namespace ovl
