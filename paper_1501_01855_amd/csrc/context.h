// The library context: one lattice geometry, its gauge field in every
// precision, the kernel low modes, workspace and profiling state.
#pragma once
#include <map>
#include <tuple>
#include <utility>
#include <string>
#include <vector>

#include <hip/hip_ext.h>

#include "common.h"

namespace ovl {

// A profiled launch: a and b are attached to the kernel's dispatch packet
// (hipExtLaunchKernelGGL), so b - a is the kernel's own execution time, not
// the distance between two markers in the stream.
struct PendingEvent {
    int kern, prec;
    double bytes;
    hipEvent_t a, b;
};

// eigSUMR basis and the deflation data derived from it (eigspace.hip).
struct EigSpace {
    int n = 0, m = 0, k = 0;        // wanted, capacity, held
    double mu = -1.0, delta = 0.1, eps = 1e-4;
    int krecalc = 25;
    bool bound_printed = false;   // eq. (bound) with chi on the square root only (measurement option)
    bool canonical = false;       // Alg. 6 orthonormalises canonically (block collection)
    double2 *V = nullptr, *VD = nullptr;   // [m] packed FP64 fields each
    int ndiag = 0;
    int nsets = 0;   // eigenvector sets kept from earlier eigensolver restarts (0..2)
    std::vector<double> uv_hist, ritz, resid;
    bool defl_ready = false;
    int ndefl = 0;
    double2 *P = nullptr, *DP = nullptr;
    std::vector<double> dn2;
    // spectral preconditioner (Sec. 4): orthonormal vectors S and the factors
    // c / sqrt(m_i) - 1 of their Ritz values m_i of H^2
    bool spec_ready = false;
    bool spec_hold = false;   // keep S fixed (a CG middle solve is running)
    int nspec = 0;
    double2 *S = nullptr;
    std::vector<double> spec_f;
};

struct GraphRec;

struct Context {
    Geom g{};
    hipStream_t stream = nullptr;
    int device = 0;
    int num_cu = 256;
    int upd_per_cu[3][2] = {};   // resident blocks per CU of the multi-shift update kernel [prec][all]

    // gauge field, packed per precision
    double2 *U64 = nullptr;   // [4][9][Pu] (Geom::Pu: padded plane stride)
    float2 *U32 = nullptr;    // 36 Pu float2: float4 [4][4][Pu] + float2 [4][Pu]
    void *U16 = nullptr;      // 36 Pu __half2: uint4 [4][2][Pu] + uint32 [4][Pu]
    void *U32r = nullptr;     // two-row FP32 links: float4 [4][2][Pu] + float4 [4][Pu]
    void *U16r = nullptr;     // two-row FP16 links: uint4 [4][Pu] + uint2 [4][Pu]
    double su3_dev = -1.0;    // largest |third row - conj(row 0 x row 1)| over the loaded links
    bool two_row_opt = true;  // OVL_OPT_TWO_ROW_LINKS
    bool have_gauge = false;

    // kernel low modes: FP64 packed [n][12][V] and eigenvalues
    int n_low = 0;
    double2 *low = nullptr;
    std::vector<double> low_evals;
    // derived from them on first use: the basis in FP32 / FP16 storage (for
    // the sign function in those precisions) and sign(lambda_j) on the device
    void *low_lp[3] = {nullptr, nullptr, nullptr};
    double *low_sgn = nullptr;
    void lowmodes_changed();                  // drop the derived copies
    const void *low_basis(int prec);
    const double *low_signs();

    // multi-shift CG: pinned host staging (constants, accuracies, polled
    // flags), its two poll events and the constants last uploaded
    void *ms_pin = nullptr;
    hipEvent_t ms_ev[2] = {nullptr, nullptr};
    std::vector<char> ms_const_last;

    // named workspace; grows on demand, freed at destroy
    std::map<std::string, DevBuf> pool;
    int64_t bytes_held = 0;

    // host staging (pinned)
    void *pinned = nullptr;
    size_t pinned_bytes = 0;

    // profiling
    bool prof = false;
    std::vector<PendingEvent> pending;
    std::vector<hipEvent_t> event_pool;   // reused by the profiled launches
    std::vector<hipEvent_t> free_events;
    ProfileSlot slots[KERN_COUNT][3];
    int64_t last_mscg_iters = 0;
    int64_t precision_retries = 0;   // sign calls redone one precision up after a breakdown
    std::vector<int64_t> last_field_iters;   // per field, last sign call


    // stencil launch variant per (precision, epilogue, nf), chosen by timing
    std::map<int, int> tuned;
    int autotune = 1;
    // set while an allocation-free entry point runs: no autotuning (a launch
    // shape not yet tuned takes the fixed variant without recording it), no
    // profiling events, no workspace growth
    bool no_alloc = false;

    // sign calls inside the solvers take as few Zolotarev poles as their
    // accuracy allows (coefficients per pole count for the interval zolo_ab)
    bool adaptive_nz = false;
    // the GMRESR outer products to the accuracy Alg. 3 prints (OVL_OPT_OUTER_PRINTED)
    bool outer_printed = false;
    std::map<int, ovl_zolo> zolo_by_n;
    double zolo_ab[2] = {0.0, 0.0};

    EigSpace eig;

    // graphs of multi-shift CG chunks, by launch configuration
    bool use_graphs = false;   // measured slower than direct launches (dependent-dispatch latency dominates)
    GraphRec *rec = nullptr;
    std::map<std::string, hipGraphExec_t> graphs;

    void *buf(const std::string &name, size_t bytes);
    void *host_stage(size_t bytes);
    // small results that kernels write straight into host memory (pinned,
    // mapped, coherent): host address, and the device address of the same
    // memory; valid until the next call (callers synchronise before reading)
    double *host_results(size_t n, double **dev);
    // wait for an event by polling it (lower latency than a blocking wait;
    // the waits here are tens of microseconds)
    void spin_wait(hipEvent_t e);
    hipEvent_t sync_ev = nullptr;   // marks the end of a reduction read back by the host
    double *hres = nullptr, *hres_dev = nullptr;
    size_t hres_n = 0;
    hipEvent_t event();
    // prof_begin creates the events; launch the kernel with them through
    // launch_k(); prof_end queues them for prof_collect().
    void prof_begin(PendingEvent &pe, int kern, int prec, double bytes);
    void prof_end(PendingEvent &pe);
    void prof_collect();
    ~Context();
};

// Bytes of one packed spinor field.
inline size_t field_bytes(const Geom &g, int prec)
{
    return prec == OVL_F64 ? (size_t)g.V * 192 : prec == OVL_F32 ? (size_t)g.V * 96 : (size_t)g.V * 52;
}

// Blocks of 256 threads covering V sites.
inline unsigned site_blocks(const Geom &g, int nt = 256) { return (unsigned)((g.V + nt - 1) / nt); }

// ---- entry points implemented in the .hip files (host side) -------------
// pack / unpack between canonical complex128 [nf][V][12] and packed fields.
// FP32 / FP16 packing goes through an FP64 staging field: tmp (nf FP64 fields)
// if given, else the context's workspace.
void pack_spinor(Context &c, const double *canon, void *packed, int nf, int prec, double2 *tmp = nullptr);
void unpack_spinor(Context &c, const void *packed, double *canon, int nf, int prec, double2 *tmp = nullptr);
void convert_spinor(Context &c, const void *src, int sprec, void *dst, int dprec, int nf);
void pack_gauge(Context &c, const double *canon);

// The library's fixed device scratch array (noalloc.hip): its address on the
// current device, looked up once per device at context creation.  Callers
// that may not allocate work in it.
void noalloc_scratch_init(int device);
void *noalloc_scratch(int device);

// stencil: out = H in / K in; nf fields in packed layout of precision prec
void launch_hop(Context &c, const void *in, void *out, int nf, int prec);
void launch_K(Context &c, double rho, const void *in, void *out, int nf, int prec);

// A graph being built from kernel nodes: while Context::rec is set,
// launch_k() appends each kernel to it (after the previous node) instead of
// launching it.
struct GraphRec {
    hipGraph_t g = nullptr;
    hipGraphNode_t last = nullptr;
};

template <typename Tuple, size_t... I>
inline void arg_ptrs(Tuple &t, void **p, std::index_sequence<I...>)
{
    ((p[I] = (void *)&std::get<I>(t)), ...);
}

// Launch a kernel on the context's stream; with pe (profiling), its events
// time the dispatch itself; while a graph is being recorded, add it as a node.
template <typename... KArgs, typename... Args>
inline void launch_k(Context &c, const PendingEvent *pe, void (*k)(KArgs...), dim3 grid, dim3 block,
                     uint32_t shmem, Args... args)
{
    if (c.rec) {
        std::tuple<KArgs...> vals(static_cast<KArgs>(args)...);
        void *ptrs[sizeof...(KArgs) > 0 ? sizeof...(KArgs) : 1];
        arg_ptrs(vals, ptrs, std::index_sequence_for<KArgs...>{});
        hipKernelNodeParams np{};
        np.func = reinterpret_cast<void *>(k);
        np.gridDim = grid;
        np.blockDim = block;
        np.sharedMemBytes = shmem;
        np.kernelParams = ptrs;
        np.extra = nullptr;
        hipGraphNode_t node;
        OVL_HIP(hipGraphAddKernelNode(&node, c.rec->g, c.rec->last ? &c.rec->last : nullptr, c.rec->last ? 1 : 0,
                                      &np));
        c.rec->last = node;
        return;
    }
    if (pe)
        hipExtLaunchKernelGGL(k, grid, block, shmem, c.stream, pe->a, pe->b, 0, static_cast<KArgs>(args)...);
    else
        hipLaunchKernelGGL(k, grid, block, shmem, c.stream, static_cast<KArgs>(args)...);
}

}  // namespace ovl
