// Static device scratch of koma_simulate_noalloc (komahip_scratch.hip),
// shared with the host code. Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace koma {

// Size of the per-device static scratch array (bytes).
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;

// Device address of `device`'s copy of the array, looked up once per device
// (hipGetSymbolAddress, with `device` current) and cached; later calls return
// the cached address and status.
hipError_t noalloc_scratch_attach(int device, void **out);

}  // namespace koma
