// Host-side launchers of the device kernels, shared by the drivers.
#pragma once
#include "context.h"

namespace ovl {

enum Epilogue {
    EPI_HOP = 0,    // out = H in
    EPI_K = 1,      // out = K in
    EPI_K2DOT = 2,  // out = K in + sigma aux; per tile (aux, out), Re (aux2, out), (out, out)
    EPI_KPLUS = 3   // out = K in + aux
};

template <typename ST>
struct StencilArgs {
    Geom g;
    const ST *in;
    ST *out;
    const ST *aux;
    const ST *aux2;  // second own-site input (EPI_K2DOT)
    double diag;     // 4 - rho
    double sigma;
    double *partial; // [nf][3][gridDim.x] (EPI_K2DOT)
    const int *stop; // per-field: skip when it >= stop[f] (nullable)
    int it;          // iteration, or its offset from *itb when itb is set
    const int *itb = nullptr;   // device iteration base (graph replays)
};

// w = K t + s0 p with the partials (p, w), Re (r, w) and (w, w) of every tile
// in partial[f][q][tile] (computed on w as stored); returns the number of
// tiles of the launch (it depends on the launch variant).
// itb (nullable): the iteration is *itb + it, read on the device (so that a
// recorded graph can be replayed for later iterations).
int stencil_k2_dot(Context &c, int prec, const void *t, void *w, int nf, double rho, double s0, const void *p,
                   const void *r, double *partial, const int *stop, int it, const int *itb = nullptr);

void stencil(Context &c, int epi, int prec, const void *in, void *out, int nf, double rho,
             double sigma, const void *aux, double *partial, const int *stop = nullptr, int it = 0,
             const void *aux2 = nullptr, const int *itb = nullptr);
// algorithmic bytes of one field's stencil (spinors and links), and of the
// links alone (read once by a launch over several fields)
double stencil_bytes(const Geom &g, int prec, int epi);
double stencil_link_bytes(const Geom &g, int prec);
// FP32 / FP16 stencils on the two-row links iff the option allows it and the
// loaded links passed the SU(3) test
void update_link_form(Context &c);
// the launch variant for (prec, epi, nf), autotuned on first use
int stencil_variant(Context &c, int epi, int prec, int nf);
// tiles (blocks per field) of stencil launch variant v; the largest over variants
unsigned stencil_tiles(const Geom &g, int v);
int64_t stencil_tiles_max(const Geom &g);
bool stencil_variant_ok(const Geom &g, int prec, int v);

// ---------------------------------------------------------------- BLAS-1 (packed FP64 fields)
// All take nf fields; scalars are per field (host arrays of nf complex / real).
// dots[f] = (x_f, y_f) complex, computed with a fixed reduction order.
void dot_f64(Context &c, const double2 *x, const double2 *y, int nf, std::vector<cplx<double>> &out);
void norm2_f64(Context &c, const double2 *x, int nf, std::vector<double> &out);
// y_f = a_f x_f + b_f y_f (y not read when b_f = 0; field untouched when a_f = 0, b_f = 1)
void axpby_f64(Context &c, const cplx<double> *a, const double2 *x, const cplx<double> *b, double2 *y, int nf);
// out[row] = sum_i partial[row][i], i < nblk (fixed order)
void sum_partials(Context &c, const double *partial, int nblk, int rows, double *out);
// the same sums written into host memory; waits for them and returns them
// (valid until the next call)
const double *sum_partials_host(Context &c, const double *partial, int nblk, int rows);
// out = a A + b B + g C over nf whole fields (real coefficients; C nullable)
void lincomb3_f64(Context &c, double a, const double2 *A, double b, const double2 *B, double g, const double2 *C,
                  double2 *out, int nf);
// y_f = gamma_5 y_f
void gamma5_f64(Context &c, double2 *y, int nf);
// dst = src
void copy_fields(Context &c, const void *src, void *dst, int nf, int prec);
void zero_fields(Context &c, void *dst, int nf, int prec);

// multi-dot: out[f][j] = (V_j, x_f) for j < nv (V: nv packed FP64 fields)
void multidot_f64(Context &c, const double2 *Vb, int nv, const double2 *x, int nf,
                  std::vector<cplx<double>> &out);
// x_f += sum_j coef[f][j] V_j
void multiaxpy_f64(Context &c, const double2 *Vb, int nv, const cplx<double> *coef, double2 *x, int nf);

// Tall-skinny block products on whole FP64 fields:
// G[i][j] = (X_i, g5^s Y_j) (nx x ny, row-major, host), s = g5 ? 1 : 0
void gram_f64(Context &c, const double2 *X, int nx, const double2 *Y, int ny, bool g5,
              std::vector<cplx<double>> &G);
// Z_k = beta Z_k + sum_j W[j][k] Y_j, W is ny x nz row-major (host); Z may not alias Y
void rotate_f64(Context &c, const double2 *Y, int ny, const std::vector<cplx<double>> &W, int nz, double2 *Z,
                double beta);

}  // namespace ovl
