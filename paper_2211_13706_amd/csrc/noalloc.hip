// The scratch of px_zeta_noalloc: a file-scope device array instead of the
// handle's grow-only workspace, so that the entry point calls no allocator.
//
// Each device that loads this code object holds its own copy of the array at
// its own address, kept until the process ends.  In host code the name
// `scratch` is only a host-side stand-in: its device address is taken once per
// device with hipGetSymbolAddress (that device current) and only that address
// is ever passed to kernels or copies.
#include "noalloc.h"

#include <mutex>

static __device__ __align__(256) unsigned char scratch[px::kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};
}  // namespace

namespace px {

hipError_t static_scratch(int device, void** ptr) {
  if (device < 0 || device >= kMaxDevices || !ptr) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[device] = p;
  }
  *ptr = g_ptr[device];
  return hipSuccess;
}

}  // namespace px
