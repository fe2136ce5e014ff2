// Context life cycle, workspace, profiling events.
#include <cstring>

#include <algorithm>

#include <thread>

#include "context.h"
#include "kernels.h"

namespace ovl {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
const char *last_error() { return g_last_error.c_str(); }

void *Context::buf(const std::string &name, size_t bytes)
{
    DevBuf &b = pool[name];
    if (b.bytes < bytes) {
        if (b.p) {
            OVL_HIP(hipStreamSynchronize(stream));
            OVL_HIP(hipFree(b.p));
            bytes_held -= (int64_t)b.bytes;
            b.p = nullptr;
            b.bytes = 0;
        }
        hipError_t e = hipMalloc(&b.p, bytes);
        if (e != hipSuccess) {
            b.p = nullptr;
            throw Error{OVL_ERR_NOMEM, "workspace '" + name + "': hipMalloc of " + std::to_string(bytes) +
                                           " bytes failed"};
        }
        b.bytes = bytes;
        bytes_held += (int64_t)bytes;
    }
    return b.p;
}

double *Context::host_results(size_t n, double **dev)
{
    if (hres_n < n) {
        if (hres) {
            OVL_HIP(hipStreamSynchronize(stream));
            OVL_HIP(hipHostFree(hres));
            hres = nullptr;
        }
        const size_t cap = std::max<size_t>(n, 4096);
        OVL_HIP(hipHostMalloc((void **)&hres, cap * sizeof(double), hipHostMallocMapped | hipHostMallocCoherent));
        OVL_HIP(hipHostGetDevicePointer((void **)&hres_dev, hres, 0));
        hres_n = cap;
    }
    *dev = hres_dev;
    return hres;
}

void Context::spin_wait(hipEvent_t e)
{
    while (true) {
        const hipError_t r = hipEventQuery(e);
        if (r == hipSuccess) return;
        if (r != hipErrorNotReady) OVL_HIP(r);
        std::this_thread::yield();   // several contexts may be polled by threads sharing the cores
    }
}

void *Context::host_stage(size_t bytes)
{
    if (pinned_bytes < bytes) {
        if (pinned) {
            OVL_HIP(hipStreamSynchronize(stream));
            OVL_HIP(hipHostFree(pinned));
            pinned = nullptr;
        }
        OVL_HIP(hipHostMalloc(&pinned, bytes, hipHostMallocDefault));
        pinned_bytes = bytes;
    }
    return pinned;
}

hipEvent_t Context::event()
{
    hipEvent_t e;
    OVL_HIP(hipEventCreate(&e));
    free_events.push_back(e);   // owned by the context; destroyed at exit
    return e;
}

void Context::lowmodes_changed()
{
    OVL_HIP(hipStreamSynchronize(stream));
    for (int p = 1; p < 3; ++p)
        if (low_lp[p]) {
            OVL_HIP(hipFree(low_lp[p]));
            bytes_held -= (int64_t)field_bytes(g, p) * n_low;
            low_lp[p] = nullptr;
        }
    if (low_sgn) {
        OVL_HIP(hipFree(low_sgn));
        low_sgn = nullptr;
    }
}

const void *Context::low_basis(int prec)
{
    if (prec == OVL_F64 || n_low == 0) return low;
    if (!low_lp[prec]) {
        const size_t B = field_bytes(g, prec) * n_low;
        OVL_HIP(hipMalloc(&low_lp[prec], B));
        bytes_held += (int64_t)B;
        convert_spinor(*this, low, OVL_F64, low_lp[prec], prec, n_low);
    }
    return low_lp[prec];
}

const double *Context::low_signs()
{
    if (!low_sgn && n_low > 0) {
        std::vector<double> sg(n_low);
        for (int j = 0; j < n_low; ++j) sg[j] = low_evals[j] >= 0.0 ? 1.0 : -1.0;
        OVL_HIP(hipMalloc(&low_sgn, sizeof(double) * n_low));
        OVL_HIP(hipMemcpyAsync(low_sgn, sg.data(), sizeof(double) * n_low, hipMemcpyHostToDevice, stream));
        OVL_HIP(hipStreamSynchronize(stream));   // sg is released on return
    }
    return low_sgn;
}

void Context::prof_begin(PendingEvent &pe, int kern, int prec, double bytes)
{
    pe.kern = kern;
    pe.prec = prec;
    pe.bytes = bytes;
    if (event_pool.size() < 2) {
        for (int i = 0; i < 64; ++i) {
            hipEvent_t e;
            OVL_HIP(hipEventCreate(&e));
            event_pool.push_back(e);
        }
    }
    pe.a = event_pool.back();
    event_pool.pop_back();
    pe.b = event_pool.back();
    event_pool.pop_back();
}

void Context::prof_end(PendingEvent &pe)
{
    pending.push_back(pe);
    if (pending.size() > 32768) prof_collect();
}

void Context::prof_collect()
{
    if (pending.empty()) return;
    OVL_HIP(hipEventSynchronize(pending.back().b));
    for (auto &pe : pending) {
        float ms = 0.f;
        OVL_HIP(hipEventElapsedTime(&ms, pe.a, pe.b));
        ProfileSlot &s = slots[pe.kern][pe.prec];
        s.launches += 1;
        s.ms += ms;
        s.bytes += pe.bytes;
        event_pool.push_back(pe.a);
        event_pool.push_back(pe.b);
    }
    pending.clear();
}

Context::~Context()
{
    hipStreamSynchronize(stream);
    for (auto &pe : pending) {
        hipEventDestroy(pe.a);
        hipEventDestroy(pe.b);
    }
    for (auto e : event_pool) hipEventDestroy(e);
    for (auto e : free_events) hipEventDestroy(e);
    for (auto &kv : pool)
        if (kv.second.p) hipFree(kv.second.p);
    if (U64) hipFree(U64);
    if (U32) hipFree(U32);
    if (U16) hipFree(U16);
    if (U32r) hipFree(U32r);
    if (U16r) hipFree(U16r);
    if (low) hipFree(low);
    for (int p = 1; p < 3; ++p)
        if (low_lp[p]) hipFree(low_lp[p]);
    if (low_sgn) hipFree(low_sgn);
    if (ms_pin) hipHostFree(ms_pin);
    for (auto e : ms_ev)
        if (e) hipEventDestroy(e);
    if (sync_ev) hipEventDestroy(sync_ev);
    for (auto &kv : graphs) hipGraphExecDestroy(kv.second);
    if (pinned) hipHostFree(pinned);
    if (hres) hipHostFree(hres);
}

}  // namespace ovl
