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
                             float2 *__restrict__ U32, int64_t V)
{
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (s >= V) return;
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const double2 u = canon[s * 36 + mu * 9 + k];
            U64[(mu * 9 + k) * V + s] = u;
            U32[(mu * 9 + k) * V + s] = make_float2((float)u.x, (float)u.y);
        }
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
        throw Error{OVL_ERR_UNSUPPORTED, "pack_spinor: precision"};
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
        throw Error{OVL_ERR_UNSUPPORTED, "unpack_spinor: precision"};
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
    } else {
        throw Error{OVL_ERR_UNSUPPORTED, "convert_spinor: precision pair"};
    }
    OVL_HIP(hipGetLastError());
}

void pack_gauge(Context &c, const double *canon)
{
    const Geom &g = c.g;
    if (!c.U64) {
        OVL_HIP(hipMalloc(&c.U64, (size_t)g.V * 36 * sizeof(double2)));
        OVL_HIP(hipMalloc(&c.U32, (size_t)g.V * 36 * sizeof(float2)));
        c.bytes_held += (int64_t)g.V * 36 * (16 + 8);
    }
    k_pack_gauge<<<site_blocks(g), 256, 0, c.stream>>>((const double2 *)canon, c.U64, c.U32, g.V);
    OVL_HIP(hipGetLastError());
    c.have_gauge = true;
}

// ------------------------------------------------------------- stencil kernel
template <typename ST, typename GT, int EPI>
__global__ __launch_bounds__(256) void k_stencil(StencilArgs<ST> a, const GT *__restrict__ U)
{
    using R = typename Planes<ST>::R;
    constexpr int NP = Planes<ST>::n;
    if (a.stop != nullptr && a.it >= a.stop[blockIdx.y]) return;
    const int64_t V = a.g.V;
    const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int f = blockIdx.y;
    const bool valid = s < V;
    const ST *in = a.in + (int64_t)f * NP * V;
    double part = 0.0;
    if (valid) {
        const int32_t L0 = a.g.L[0], L1 = a.g.L[1], L2 = a.g.L[2], L3 = a.g.L[3];
        const int32_t si = (int32_t)s;
        int32_t co[4];
        co[0] = si % L0;
        int32_t rem = si / L0;
        co[1] = rem % L1;
        rem /= L1;
        co[2] = rem % L2;
        co[3] = rem / L2;
        const int32_t Ls[4] = {L0, L1, L2, L3};
        cplx<R> acc[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = {R(0), R(0)};
        cplx<R> psi[12];
        cplx<R> u[9];
#pragma unroll 1
        for (int mu = 0; mu < 4; ++mu) {
            const int64_t st = a.g.stride[mu];
            const int32_t c = co[mu], Lm = Ls[mu];
            const int64_t fwd = (c == Lm - 1) ? s - (int64_t)(Lm - 1) * st : s + st;
            const int64_t bwd = (c == 0) ? s + (int64_t)(Lm - 1) * st : s - st;
            ld_sp(in, V, fwd, psi);
            ld_link(U, V, mu, s, u);
            switch (mu) {
            case 0: hop_term<0, true>(psi, u, acc); break;
            case 1: hop_term<1, true>(psi, u, acc); break;
            case 2: hop_term<2, true>(psi, u, acc); break;
            default: hop_term<3, true>(psi, u, acc); break;
            }
            ld_sp(in, V, bwd, psi);
            ld_link(U, V, mu, bwd, u);
            switch (mu) {
            case 0: hop_term<0, false>(psi, u, acc); break;
            case 1: hop_term<1, false>(psi, u, acc); break;
            case 2: hop_term<2, false>(psi, u, acc); break;
            default: hop_term<3, false>(psi, u, acc); break;
            }
        }
        ST *out = a.out + (int64_t)f * NP * V;
        if constexpr (EPI == EPI_HOP) {
            st_sp(out, V, s, acc);
        } else {
            // D_W psi = (4 - rho) psi - H psi / 2, then gamma_5 (negate spins 2, 3)
            ld_sp(in, V, s, psi);
            const R m = (R)a.diag, h = (R)0.5;
#pragma unroll
            for (int c = 0; c < 12; ++c) {
                cplx<R> d = m * psi[c] - h * acc[c];
                acc[c] = (c < 6) ? d : -d;
            }
            if constexpr (EPI == EPI_K2DOT) {
                // w = K t + sigma p ; partial (p, w)
                ld_sp(a.aux + (int64_t)f * NP * V, V, s, psi);
                const R sg = (R)a.sigma;
                double d = 0.0;
#pragma unroll
                for (int c = 0; c < 12; ++c) {
                    acc[c] = acc[c] + sg * psi[c];
                    d += (double)psi[c].re * (double)acc[c].re + (double)psi[c].im * (double)acc[c].im;
                }
                part = d;
            } else if constexpr (EPI == EPI_KPLUS) {
                ld_sp(a.aux + (int64_t)f * NP * V, V, s, psi);
#pragma unroll
                for (int c = 0; c < 12; ++c) acc[c] = acc[c] + psi[c];
            }
            st_sp(out, V, s, acc);
        }
    }
    if constexpr (EPI == EPI_K2DOT) {
        __shared__ double lds[4];
        const double t = block_sum<256>(part, lds);
        if (threadIdx.x == 0) a.partial[(int64_t)f * gridDim.x + blockIdx.x] = t;
    }
}

template <typename ST, typename GT, int EPI>
static void launch_stencil_t(Context &c, const StencilArgs<ST> &a, const GT *U, int nf, int prec,
                             bool profile)
{
    dim3 grid(site_blocks(c.g), nf);
    PendingEvent pe;
    const double bytes = stencil_bytes(c.g, prec, EPI) * nf;
    if (profile) c.prof_begin(pe, KERN_STENCIL, prec, bytes);
    k_stencil<ST, GT, EPI><<<grid, 256, 0, c.stream>>>(a, U);
    OVL_HIP(hipGetLastError());
    if (profile) c.prof_end(pe);
}

void stencil(Context &c, int epi, int prec, const void *in, void *out, int nf, double rho,
             double sigma, const void *aux, double *partial, const int *stop, int it)
{
    OVL_REQUIRE(c.have_gauge, OVL_ERR_STATE, "no gauge field loaded");
    if (prec == OVL_F64) {
        StencilArgs<double2> a{c.g, (const double2 *)in, (double2 *)out, (const double2 *)aux,
                               4.0 - rho, sigma, partial, stop, it};
        switch (epi) {
        case EPI_HOP: launch_stencil_t<double2, double2, EPI_HOP>(c, a, c.U64, nf, prec, true); break;
        case EPI_K: launch_stencil_t<double2, double2, EPI_K>(c, a, c.U64, nf, prec, true); break;
        case EPI_K2DOT: launch_stencil_t<double2, double2, EPI_K2DOT>(c, a, c.U64, nf, prec, true); break;
        case EPI_KPLUS: launch_stencil_t<double2, double2, EPI_KPLUS>(c, a, c.U64, nf, prec, true); break;
        }
    } else if (prec == OVL_F32) {
        StencilArgs<float4> a{c.g, (const float4 *)in, (float4 *)out, (const float4 *)aux,
                              4.0 - rho, sigma, partial, stop, it};
        switch (epi) {
        case EPI_HOP: launch_stencil_t<float4, float2, EPI_HOP>(c, a, c.U32, nf, prec, true); break;
        case EPI_K: launch_stencil_t<float4, float2, EPI_K>(c, a, c.U32, nf, prec, true); break;
        case EPI_K2DOT: launch_stencil_t<float4, float2, EPI_K2DOT>(c, a, c.U32, nf, prec, true); break;
        case EPI_KPLUS: launch_stencil_t<float4, float2, EPI_KPLUS>(c, a, c.U32, nf, prec, true); break;
        }
    } else {
        throw Error{OVL_ERR_UNSUPPORTED, "stencil: precision"};
    }
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
// reads of the epilogues that take a second input.
double stencil_bytes(const Geom &g, int prec, int epi)
{
    const double S = (double)field_bytes(g, prec);
    const double G = (double)g.V * 36 * (prec == OVL_F64 ? 16 : prec == OVL_F32 ? 8 : 4);
    double b = 2 * S + G;
    if (epi == EPI_K2DOT || epi == EPI_KPLUS) b += S;
    return b;
}

}  // namespace ovl
