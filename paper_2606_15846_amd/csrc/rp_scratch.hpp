// Fixed per-device workspace of the proposer's allocation-free entry point
// (library internal; the array itself lives in rp_scratch.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace navsim {

// Bytes of the workspace on every device the library runs on (held until the
// process ends).
constexpr size_t kRpScratchBytes = (size_t)16 << 20;

// Device address of the workspace on `device`, which must be the current
// device; looked up once per device (hipGetSymbolAddress) and cached.
hipError_t rp_scratch_address(int device, void **out);

}  // namespace navsim
