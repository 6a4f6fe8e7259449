// Static device scratch of the allocation-free zeta entry point (see noalloc.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace px {

// Bytes of the static scratch array that every device loading the library holds.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;

// Device address of that array on `device`, which must be the current device.
// The address is taken once per device (hipGetSymbolAddress) and kept; later
// calls return it without a runtime call.  Thread-safe.
hipError_t static_scratch(int device, void** ptr);

}  // namespace px
