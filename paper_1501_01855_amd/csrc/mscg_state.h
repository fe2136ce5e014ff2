// Device-resident state of the multi-shift CG, one record per field, double
// buffered by iteration parity: the kernels of iteration it read S[it & 1];
// block 0 of the last kernel of the iteration writes S[(it + 1) & 1].  The
// iteration's scalars (alpha, beta, zeta_l', ...) are recomputed by every
// block from the per-tile partial sums of the previous kernels, in a fixed
// order, so every block sees identical values without grid-wide
// synchronisation or atomics.
#pragma once
#include "common.h"
#include "fields.h"

namespace ovl {

constexpr int NZMAX = OVL_MAX_NZ;

struct MscgScal {
    double rr, alpha_old, beta_old, b2;
    int iters, breakdown, act_total, pad;
    double zeta[NZMAX], zeta_old[NZMAX];
    int act[NZMAX];
};

struct MscgConst {
    int nz, base, maxiter, pad;
    double s0;
    double sigma[NZMAX], omega[NZMAX], tol2[NZMAX];
};

// The block's sum of the per-thread values v (fixed order), returned to every
// thread.
__device__ inline double block_bcast_sum(double v, double *lds)
{
    const double t = block_sum<256>(v, lds);
    __shared__ double bcast;
    if (threadIdx.x == 0) bcast = t;
    __syncthreads();
    const double r = bcast;
    __syncthreads();
    return r;
}

// Four block sums at once (256 threads), each with the same reduction tree as
// block_bcast_sum (so the same values), returned to every thread; one pair of
// barriers instead of four.
__device__ inline void block_bcast_sum4(double v[4], double out[4])
{
    __shared__ double l4[4][4];   // [value][wave]
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < 4; ++k) l4[k][wave] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double r = 0.0;
#pragma unroll
        for (int w = 0; w < 4; ++w) r += l4[k][w];
        out[k] = r;
    }
}

// Sum of p[0..n) by the whole block in a fixed order; the result is returned
// to every thread.
__device__ inline double block_allsum(const double *p, int n, double *lds)
{
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += p[i];
    return block_bcast_sum(v, lds);
}

}  // namespace ovl
