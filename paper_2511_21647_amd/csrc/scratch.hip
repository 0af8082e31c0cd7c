// Library-owned device scratch for callers that cannot allocate (code under
// graph capture, serving loops that forbid allocation).  One fixed array per
// device, holding what a caller-supplied workspace holds otherwise; its device
// address is looked up once per device, when the first context is created on
// that device, and kept in a host table.  Every call on a device shares that
// device's array, so calls that overlap on one device race.
#include "common.h"

#include <mutex>

namespace ulm {

static __device__ __align__(256) unsigned char scratch[ULM_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];
}  // namespace

// Called by ulm_create with `device` current.  Idempotent per device.
hipError_t scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
    return hipSuccess;
}

// The device address of `device`'s array, or nullptr if scratch_init has not
// succeeded on it.
void *scratch_ptr(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace ulm
