// The library's fixed device scratch memory, for entry points whose callers
// cannot allocate device memory (code under HIP graph capture, serving loops
// that forbid allocation).  One array per GPU, held until the process ends;
// every call on that GPU shares it, so calls that overlap in time on one GPU
// (two streams, two threads) race on its contents.
//
// In host code the array's name is a host-side stand-in, not a device
// address: its device address is looked up once per device, with that device
// current, at context creation (ovl_create), and only that address is handed
// to kernels.
#include <mutex>
#include <string>

#include "context.h"

namespace ovl {

static __device__ __align__(256) unsigned char scratch[OVL_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_ptr[MAX_DEVICES] = {};
bool g_done[MAX_DEVICES] = {};
hipError_t g_err[MAX_DEVICES] = {};
}  // namespace

void noalloc_scratch_init(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_done[device]) return;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_err[device] = e;
    g_ptr[device] = (e == hipSuccess) ? p : nullptr;
    g_done[device] = true;
    if (e != hipSuccess) (void)hipGetLastError();   // leave no sticky error for the next call
}

void *noalloc_scratch(int device)
{
    OVL_REQUIRE(device >= 0 && device < MAX_DEVICES, OVL_ERR_UNSUPPORTED, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_mu);
    OVL_REQUIRE(g_done[device], OVL_ERR_STATE, "scratch address of this device not looked up (no context created on it)");
    if (!g_ptr[device])
        throw Error{OVL_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(g_err[device])};
    return g_ptr[device];
}

}  // namespace ovl
