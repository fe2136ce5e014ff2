// Streaming ceiling of the memory system, for rooflines (not part of the
// method): a copy and a read-only pass over whole buffers, 16-byte loads and
// stores, a grid sized to the chip with each thread walking the buffer in
// steps of the whole grid, four loads in flight per thread.
#include "context.h"

namespace ovl {

__global__ __launch_bounds__(256) void k_stream_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                     int64_t n)
{
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (; i + 3 * step < n; i += 4 * step) {
        const uint4 a = src[i], b = src[i + step], c = src[i + 2 * step], d = src[i + 3 * step];
        dst[i] = a;
        dst[i + step] = b;
        dst[i + 2 * step] = c;
        dst[i + 3 * step] = d;
    }
    for (; i < n; i += step) dst[i] = src[i];
}

// Reads every word; each block writes one word (the XOR of what it read) so
// that the loads cannot be dropped.
__global__ __launch_bounds__(256) void k_stream_read(const uint4 *__restrict__ src, int64_t n,
                                                     unsigned *__restrict__ out)
{
    __shared__ unsigned red[256];
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    unsigned x = 0;
    for (; i + 3 * step < n; i += 4 * step) {
        const uint4 a = src[i], b = src[i + step], c = src[i + 2 * step], d = src[i + 3 * step];
        x ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w ^ c.x ^ c.y ^ c.z ^ c.w ^ d.x ^ d.y ^ d.z ^ d.w;
    }
    for (; i < n; i += step) {
        const uint4 a = src[i];
        x ^= a.x ^ a.y ^ a.z ^ a.w;
    }
    red[threadIdx.x] = x;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] ^= red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// Average milliseconds per launch over reps launches (after one untimed),
// timed by events on the context's stream.  kind 0: copy src -> dst; kind 1:
// read src (dst receives one word per block, at least 64 KiB).
double stream_bench(Context &c, int kind, const void *src, void *dst, int64_t bytes, int reps)
{
    const int64_t n = bytes / 16;
    const unsigned blocks = (unsigned)c.num_cu * 16;
    auto launch = [&] {
        if (kind == 0)
            k_stream_copy<<<blocks, 256, 0, c.stream>>>((const uint4 *)src, (uint4 *)dst, n);
        else
            k_stream_read<<<blocks, 256, 0, c.stream>>>((const uint4 *)src, n, (unsigned *)dst);
    };
    launch();
    OVL_HIP(hipGetLastError());
    hipEvent_t e0 = c.event(), e1 = c.event();
    OVL_HIP(hipEventRecord(e0, c.stream));
    for (int r = 0; r < reps; ++r) launch();
    OVL_HIP(hipEventRecord(e1, c.stream));
    OVL_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    OVL_HIP(hipEventElapsedTime(&ms, e0, e1));
    return (double)ms / reps;
}

}  // namespace ovl
