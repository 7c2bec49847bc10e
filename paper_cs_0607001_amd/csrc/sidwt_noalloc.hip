// Library-owned scratch for the entry point that allocates nothing
// (sidwt_correlate_swapped_noalloc): a file-scope device array, one copy per
// GPU the library runs on, held until the process ends.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in
// symbol); it looks up each device's address once with hipGetSymbolAddress,
// with that device current, and hands out that address.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <mutex>

#include "../../include/sidwt.h"

namespace {

constexpr size_t kScratchBytes = (size_t)SIDWT_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

std::mutex scratch_mu;
void *scratch_ptr[kMaxDevices] = {};

}  // namespace

namespace sidwt {

__device__ __align__(256) unsigned char scratch[kScratchBytes];

// The current device's copy of the scratch array (looked up on the first
// call per device).  hipErrorInvalidDevice past kMaxDevices devices.
hipError_t noalloc_scratch(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    scratch_ptr[dev] = p;
  }
  *out = scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace sidwt
