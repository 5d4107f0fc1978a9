// Static device scratch for callers that cannot allocate (koma_simulate_noalloc).
//
// One file-scope device array holds every buffer such a call needs beyond its
// inputs and outputs: the packed event program and its tables, the phantom
// validation word, the block-start snapshots, the inline and cross-workgroup
// signal partials and, when the final state is exported, the spin state.
// Every GPU the library runs on holds its own copy of the array (at its own
// address) until the process ends. In host code the array's name is only a
// host-side stand-in: the device address comes from hipGetSymbolAddress,
// looked up once per device with that device current (at context creation)
// and kept here; kernels and copies only ever see that address.
//
// The array is shared by every call on a device and keeps the last call's
// contents, so calls that overlap on one device race: the caller orders them
// (one stream, or events). What must start at zero (the validation word) is
// cleared by a kernel of the call itself.
#include <hip/hip_runtime.h>

#include <mutex>

#include "komahip_scratch.h"

namespace koma {

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};
hipError_t g_err[kMaxDevices] = {};
bool g_done[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_attach(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_done[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e == hipSuccess && cur != device) e = hipErrorInvalidDevice;  // the caller sets the device first
        void *p = nullptr;
        if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_err[device] = e;
        g_ptr[device] = e == hipSuccess ? p : nullptr;
        g_done[device] = true;
    }
    *out = g_ptr[device];
    return g_err[device];
}

}  // namespace koma
