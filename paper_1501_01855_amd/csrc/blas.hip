// BLAS-1 on packed FP64 spinor fields (12 V complex numbers per field):
// dots, norms and vector updates for SUMR (Alg. 2), GMRESR (Alg. 3) and the
// eigenspace code.  Reductions: per-thread sums over a fixed grid-stride
// pattern, wave64 shuffles, one partial per block, then one block sums the
// partials in a fixed order, so results are run-to-run reproducible.
#include <algorithm>

#include "context.h"
#include "fields.h"
#include "kernels.h"

namespace ovl {

static constexpr int RB = 512;   // reduction blocks per field

__global__ __launch_bounds__(256) void k_dot(const double2 *__restrict__ x, const double2 *__restrict__ y,
                                             int64_t n, double *partial)
{
    const int f = blockIdx.y;
    const double2 *xf = x + (int64_t)f * n, *yf = y + (int64_t)f * n;
    double re = 0.0, im = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double2 a = xf[i], b = yf[i];
        re += a.x * b.x + a.y * b.y;
        im += a.x * b.y - a.y * b.x;
    }
    __shared__ double lds[4];
    const double tr = block_sum<256>(re, lds);
    const double ti = block_sum<256>(im, lds);
    if (threadIdx.x == 0) {
        partial[((int64_t)f * 2 + 0) * gridDim.x + blockIdx.x] = tr;
        partial[((int64_t)f * 2 + 1) * gridDim.x + blockIdx.x] = ti;
    }
}

// out may be host memory: the store is fenced at system scope, so it has
// completed when the kernel has.
__global__ __launch_bounds__(256) void k_sum_rows(const double *partial, int nblk, double *out)
{
    __shared__ double lds[4];
    double v = 0.0;
    const double *p = partial + (int64_t)blockIdx.x * nblk;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) v += p[i];
    const double t = block_sum<256>(v, lds);
    if (threadIdx.x == 0) {
        out[blockIdx.x] = t;
        __threadfence_system();
    }
}

void sum_partials(Context &c, const double *partial, int nblk, int rows, double *out)
{
    k_sum_rows<<<rows, 256, 0, c.stream>>>(partial, nblk, out);
    OVL_HIP(hipGetLastError());
}

const double *sum_partials_host(Context &c, const double *partial, int nblk, int rows)
{
    double *dev = nullptr;
    const double *h = c.host_results(rows, &dev);
    k_sum_rows<<<rows, 256, 0, c.stream>>>(partial, nblk, dev);   // into host memory: no copy command
    OVL_HIP(hipGetLastError());
    if (!c.sync_ev) OVL_HIP(hipEventCreate(&c.sync_ev));
    OVL_HIP(hipEventRecord(c.sync_ev, c.stream));
    c.spin_wait(c.sync_ev);
    return h;
}

void dot_f64(Context &c, const double2 *x, const double2 *y, int nf, std::vector<cplx<double>> &out)
{
    const int64_t n = 12 * c.g.V;
    double *part = (double *)c.buf("blas_part", sizeof(double) * RB * 2 * nf);
    k_dot<<<dim3(RB, nf), 256, 0, c.stream>>>(x, y, n, part);
    OVL_HIP(hipGetLastError());
    const double *h = sum_partials_host(c, part, RB, 2 * nf);
    out.resize(nf);
    for (int f = 0; f < nf; ++f) out[f] = {h[2 * f], h[2 * f + 1]};
}

void norm2_f64(Context &c, const double2 *x, int nf, std::vector<double> &out)
{
    std::vector<cplx<double>> d;
    dot_f64(c, x, x, nf, d);
    out.resize(nf);
    for (int f = 0; f < nf; ++f) out[f] = d[f].re;
}

struct Coef {
    double re, im;
};

static constexpr int MAXNF = 16;

struct AxpbyCoef {
    Coef a[MAXNF], b[MAXNF];
};

__global__ __launch_bounds__(256) void k_axpby(AxpbyCoef k, const double2 *__restrict__ x,
                                               double2 *__restrict__ y, int64_t n)
{
    const int f = blockIdx.y;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const cplx<double> af = {k.a[f].re, k.a[f].im}, bf = {k.b[f].re, k.b[f].im};
    if (af.re == 0.0 && af.im == 0.0 && bf.re == 1.0 && bf.im == 0.0) return;   // field left as is
    const double2 xv = x[(int64_t)f * n + i];
    cplx<double> r = af * cplx<double>{xv.x, xv.y};
    if (bf.re != 0.0 || bf.im != 0.0) {   // b = 0: y is not read (it may be uninitialised)
        const double2 yv = y[(int64_t)f * n + i];
        r = r + bf * cplx<double>{yv.x, yv.y};
    }
    y[(int64_t)f * n + i] = make_double2(r.re, r.im);
}

void axpby_f64(Context &c, const cplx<double> *a, const double2 *x, const cplx<double> *b, double2 *y, int nf)
{
    OVL_REQUIRE(nf >= 1 && nf <= MAXNF, OVL_ERR_ARG, "too many fields in one update");
    const int64_t n = 12 * c.g.V;
    AxpbyCoef k{};
    for (int f = 0; f < nf; ++f) {
        k.a[f] = {a[f].re, a[f].im};
        k.b[f] = {b[f].re, b[f].im};
    }
    k_axpby<<<dim3((unsigned)((n + 255) / 256), nf), 256, 0, c.stream>>>(k, x, y, n);
    OVL_HIP(hipGetLastError());
}

__global__ __launch_bounds__(256) void k_gamma5(double2 *__restrict__ y, int64_t V)
{
    const int f = blockIdx.y;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= 6 * V) return;
    double2 *p = y + (int64_t)f * 12 * V + 6 * V;   // planes of spins 2, 3
    const double2 v = p[i];
    p[i] = make_double2(-v.x, -v.y);
}

void gamma5_f64(Context &c, double2 *y, int nf)
{
    const int64_t V = c.g.V;
    k_gamma5<<<dim3((unsigned)((6 * V + 255) / 256), nf), 256, 0, c.stream>>>(y, V);
    OVL_HIP(hipGetLastError());
}

void copy_fields(Context &c, const void *src, void *dst, int nf, int prec)
{
    OVL_HIP(hipMemcpyAsync(dst, src, field_bytes(c.g, prec) * nf, hipMemcpyDeviceToDevice, c.stream));
}

__global__ void k_zero(uint4 *p, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = make_uint4(0, 0, 0, 0);
}

void zero_fields(Context &c, void *dst, int nf, int prec)
{
    const int64_t n = (int64_t)(field_bytes(c.g, prec) * nf / 16);
    k_zero<<<(unsigned)((n + 255) / 256), 256, 0, c.stream>>>((uint4 *)dst, n);
    OVL_HIP(hipGetLastError());
}

// out[f][j] = (V_j, x_f)
__global__ __launch_bounds__(256) void k_multidot(const double2 *__restrict__ Vb, int nv,
                                                  const double2 *__restrict__ x, int64_t n, double *partial)
{
    const int f = blockIdx.y;
    const int j = blockIdx.z;
    const double2 *xf = x + (int64_t)f * n, *vj = Vb + (int64_t)j * n;
    double re = 0.0, im = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double2 a = vj[i], b = xf[i];
        re += a.x * b.x + a.y * b.y;
        im += a.x * b.y - a.y * b.x;
    }
    __shared__ double lds[4];
    const double tr = block_sum<256>(re, lds);
    const double ti = block_sum<256>(im, lds);
    if (threadIdx.x == 0) {
        const int64_t row = ((int64_t)f * nv + j) * 2;
        partial[(row + 0) * gridDim.x + blockIdx.x] = tr;
        partial[(row + 1) * gridDim.x + blockIdx.x] = ti;
    }
}

void multidot_f64(Context &c, const double2 *Vb, int nv, const double2 *x, int nf,
                  std::vector<cplx<double>> &out)
{
    out.assign((size_t)nf * nv, {0.0, 0.0});
    if (nv == 0) return;
    const int64_t n = 12 * c.g.V;
    const int nb = 128;
    double *part = (double *)c.buf("mdot_part", sizeof(double) * nb * 2 * nf * nv);
    k_multidot<<<dim3(nb, nf, nv), 256, 0, c.stream>>>(Vb, nv, x, n, part);
    OVL_HIP(hipGetLastError());
    const double *h = sum_partials_host(c, part, nb, 2 * nf * nv);
    for (int i = 0; i < nf * nv; ++i) out[i] = {h[2 * i], h[2 * i + 1]};
}

// x_f += sum_j coef[f*nv + j] V_j
__global__ __launch_bounds__(256) void k_multiaxpy(const double2 *__restrict__ Vb, int nv, const Coef *coef,
                                                   double2 *__restrict__ x, int64_t n)
{
    const int f = blockIdx.y;
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 xv = x[(int64_t)f * n + i];
    cplx<double> acc = {xv.x, xv.y};
    for (int j = 0; j < nv; ++j) {
        const double2 v = Vb[(int64_t)j * n + i];
        acc = acc + cplx<double>{coef[f * nv + j].re, coef[f * nv + j].im} * cplx<double>{v.x, v.y};
    }
    x[(int64_t)f * n + i] = make_double2(acc.re, acc.im);
}

void multiaxpy_f64(Context &c, const double2 *Vb, int nv, const cplx<double> *coef, double2 *x, int nf)
{
    if (nv == 0) return;
    const int64_t n = 12 * c.g.V;
    Coef *d = (Coef *)c.buf("maxpy_coef", sizeof(Coef) * nf * nv);
    std::vector<Coef> h((size_t)nf * nv);   // pageable: the copy is staged before return
    for (int i = 0; i < nf * nv; ++i) h[i] = {coef[i].re, coef[i].im};
    OVL_HIP(hipMemcpyAsync(d, h.data(), sizeof(Coef) * nf * nv, hipMemcpyHostToDevice, c.stream));
    k_multiaxpy<<<dim3((unsigned)((n + 255) / 256), nf), 256, 0, c.stream>>>(Vb, nv, d, x, n);
    OVL_HIP(hipGetLastError());
}

}  // namespace ovl

namespace ovl {

// out = a A + b B + g C over nf whole fields (real coefficients); C may be null.
__global__ __launch_bounds__(256) void k_lincomb3(double a, const double2 *__restrict__ A, double b,
                                                  const double2 *__restrict__ B, double g,
                                                  const double2 *__restrict__ C, double2 *__restrict__ out,
                                                  int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 x = A[i], y = B[i];
    double re = a * x.x + b * y.x, im = a * x.y + b * y.y;
    if (C != nullptr) {
        const double2 z = C[i];
        re += g * z.x;
        im += g * z.y;
    }
    out[i] = make_double2(re, im);
}

void lincomb3_f64(Context &c, double a, const double2 *A, double b, const double2 *B, double g, const double2 *C,
                  double2 *out, int nf)
{
    const int64_t n = 12 * c.g.V * (int64_t)nf;
    k_lincomb3<<<(unsigned)((n + 255) / 256), 256, 0, c.stream>>>(a, A, b, B, g, C, out, n);
    OVL_HIP(hipGetLastError());
}

}  // namespace ovl

namespace ovl {

// ---------------------------------------------------------------- tall-skinny block products
// G[i][j] = sum_n conj(X_i[n]) (g5 Y_j)[n] over whole FP64 fields (n < 12 V),
// optionally with gamma_5 applied to Y (planes 6..11 negated).  Output tiles
// of 32 x 32, each thread 2 x 2 entries; rows streamed through LDS in chunks
// of 64; the row range is split over blockIdx.z and the split partials are
// summed in a fixed order by a second kernel.
static constexpr int GT = 32, GR = 64;

__global__ __launch_bounds__(256) void k_gram(const double2 *__restrict__ X, int nx, const double2 *__restrict__ Y,
                                              int ny, int64_t n, int64_t V, int g5, int64_t rows_per_split,
                                              double2 *__restrict__ part)
{
    __shared__ double2 xs[GT][GR + 1];
    __shared__ double2 ys[GT][GR + 1];
    const int i0 = blockIdx.x * GT, j0 = blockIdx.y * GT;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int64_t r0 = (int64_t)blockIdx.z * rows_per_split;
    const int64_t r1 = r0 + rows_per_split < n ? r0 + rows_per_split : n;
    cplx<double> acc[2][2] = {{{0, 0}, {0, 0}}, {{0, 0}, {0, 0}}};
    for (int64_t rb = r0; rb < r1; rb += GR) {
        // load 32 vectors x 64 rows of X and Y (8 elements per thread each)
        for (int e = threadIdx.x; e < GT * GR; e += 256) {
            const int v = e / GR, rr = e % GR;
            const int64_t row = rb + rr;
            double2 xv = make_double2(0.0, 0.0), yv = make_double2(0.0, 0.0);
            if (row < r1) {
                if (i0 + v < nx) xv = X[(int64_t)(i0 + v) * n + row];
                if (j0 + v < ny) {
                    yv = Y[(int64_t)(j0 + v) * n + row];
                    if (g5 && row >= 6 * V) yv = make_double2(-yv.x, -yv.y);
                }
            }
            xs[v][rr] = xv;
            ys[v][rr] = yv;
        }
        __syncthreads();
#pragma unroll 4
        for (int rr = 0; rr < GR; ++rr) {
            const double2 a0 = xs[2 * ty][rr], a1 = xs[2 * ty + 1][rr];
            const double2 b0 = ys[2 * tx][rr], b1 = ys[2 * tx + 1][rr];
            acc[0][0] = acc[0][0] + cmul_conj(cplx<double>{a0.x, a0.y}, cplx<double>{b0.x, b0.y});
            acc[0][1] = acc[0][1] + cmul_conj(cplx<double>{a0.x, a0.y}, cplx<double>{b1.x, b1.y});
            acc[1][0] = acc[1][0] + cmul_conj(cplx<double>{a1.x, a1.y}, cplx<double>{b0.x, b0.y});
            acc[1][1] = acc[1][1] + cmul_conj(cplx<double>{a1.x, a1.y}, cplx<double>{b1.x, b1.y});
        }
        __syncthreads();
    }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            const int i = i0 + 2 * ty + a, j = j0 + 2 * tx + b;
            if (i < nx && j < ny)
                part[((int64_t)blockIdx.z * nx + i) * ny + j] = make_double2(acc[a][b].re, acc[a][b].im);
        }
}

__global__ void k_gram_sum(const double2 *__restrict__ part, int nsplit, int64_t nxy, double2 *__restrict__ out)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= nxy) return;
    double re = 0.0, im = 0.0;
    for (int z = 0; z < nsplit; ++z) {
        const double2 v = part[(int64_t)z * nxy + e];
        re += v.x;
        im += v.y;
    }
    out[e] = make_double2(re, im);
}

void gram_f64(Context &c, const double2 *X, int nx, const double2 *Y, int ny, bool g5,
              std::vector<cplx<double>> &G)
{
    G.assign((size_t)nx * ny, {0.0, 0.0});
    if (nx == 0 || ny == 0) return;
    const int64_t V = c.g.V, n = 12 * V;
    const int tiles = ((nx + GT - 1) / GT) * ((ny + GT - 1) / GT);
    int nsplit = std::max(1, 1024 / tiles);
    int64_t rps = (n + nsplit - 1) / nsplit;
    rps = ((rps + GR - 1) / GR) * GR;
    nsplit = (int)((n + rps - 1) / rps);
    double2 *part = (double2 *)c.buf("gram_part", sizeof(double2) * (size_t)nsplit * nx * ny);
    double2 *res = (double2 *)c.buf("gram_res", sizeof(double2) * (size_t)nx * ny);
    dim3 grid((nx + GT - 1) / GT, (ny + GT - 1) / GT, nsplit);
    k_gram<<<grid, 256, 0, c.stream>>>(X, nx, Y, ny, n, V, g5 ? 1 : 0, rps, part);
    const int64_t nxy = (int64_t)nx * ny;
    k_gram_sum<<<(unsigned)((nxy + 255) / 256), 256, 0, c.stream>>>(part, nsplit, nxy, res);
    OVL_HIP(hipGetLastError());
    std::vector<double2> h((size_t)nxy);
    OVL_HIP(hipMemcpyAsync(h.data(), res, sizeof(double2) * nxy, hipMemcpyDeviceToHost, c.stream));
    OVL_HIP(hipStreamSynchronize(c.stream));
    for (int64_t e = 0; e < nxy; ++e) G[e] = {h[e].x, h[e].y};
}

// Z_k = beta Z_k + sum_j W[j][k] Y_j  (k < nz, j < ny), whole FP64 fields.
// One row per thread, 16 outputs per grid row; W staged in LDS.
static constexpr int RK = 16;

__global__ __launch_bounds__(256) void k_rotate(const double2 *__restrict__ Y, int ny, const double2 *__restrict__ W,
                                                int nz, double2 *__restrict__ Z, int64_t n, double beta)
{
    extern __shared__ double2 ws[];   // [ny][RK]
    const int k0 = blockIdx.y * RK;
    for (int e = threadIdx.x; e < ny * RK; e += 256) {
        const int j = e / RK, k = e % RK;
        ws[e] = (k0 + k < nz) ? W[(int64_t)j * nz + k0 + k] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (row >= n) return;
    cplx<double> acc[RK];
#pragma unroll
    for (int k = 0; k < RK; ++k) acc[k] = {0.0, 0.0};
    for (int j = 0; j < ny; ++j) {
        const double2 yv = Y[(int64_t)j * n + row];
        const cplx<double> y{yv.x, yv.y};
#pragma unroll
        for (int k = 0; k < RK; ++k) {
            const double2 w = ws[j * RK + k];
            acc[k] = acc[k] + cplx<double>{w.x, w.y} * y;
        }
    }
#pragma unroll
    for (int k = 0; k < RK; ++k) {
        if (k0 + k >= nz) break;
        double2 *z = Z + (int64_t)(k0 + k) * n + row;
        cplx<double> v = acc[k];
        if (beta != 0.0) {
            const double2 o = *z;
            v = v + beta * cplx<double>{o.x, o.y};
        }
        *z = make_double2(v.re, v.im);
    }
}

void rotate_f64(Context &c, const double2 *Y, int ny, const std::vector<cplx<double>> &W, int nz, double2 *Z,
                double beta)
{
    if (nz == 0) return;
    OVL_REQUIRE(ny >= 1 && ny <= 512, OVL_ERR_ARG, "rotate: too many input fields");
    const int64_t n = 12 * c.g.V;
    double2 *wd = (double2 *)c.buf("rot_w", sizeof(double2) * (size_t)ny * nz);
    std::vector<double2> h((size_t)ny * nz);
    for (size_t e = 0; e < h.size(); ++e) h[e] = make_double2(W[e].re, W[e].im);
    OVL_HIP(hipMemcpyAsync(wd, h.data(), sizeof(double2) * h.size(), hipMemcpyHostToDevice, c.stream));
    dim3 grid((unsigned)((n + 255) / 256), (nz + RK - 1) / RK);
    k_rotate<<<grid, 256, sizeof(double2) * ny * RK, c.stream>>>(Y, ny, wd, nz, Z, n, beta);
    OVL_HIP(hipGetLastError());
}

}  // namespace ovl
