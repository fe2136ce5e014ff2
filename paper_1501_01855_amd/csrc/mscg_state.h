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

// Sum of p[0..n) by the whole block in a fixed order; the result is returned
// to every thread.
__device__ inline double block_allsum(const double *p, int n, double *lds)
{
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += p[i];
    return block_bcast_sum(v, lds);
}

}  // namespace ovl
