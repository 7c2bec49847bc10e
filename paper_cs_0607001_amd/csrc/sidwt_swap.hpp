// Roles-exchanged correlation (redundant analysis on the received pulse,
// critical on the reference): the weights descriptor shared by the host API
// and the kernels in sidwt_swap.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "sidwt_device.hpp"

namespace sidwt {

// Weights of every plane j (conj is applied in the kernel): j = 0 points at
// the reference (lo 0, len m); j >= 1 at phase 0 of the plan's band-A tree,
// the level-j x-side approximation of the reference, on its linear support
// [lo, lo + len) (element k at a[k - lo]).
struct SwapDesc {
  const float2 *a[kMaxLevels + 1];
  int lo[kMaxLevels + 1];
  int len[kMaxLevels + 1];
};

// LDS of plane j's work item: whole plane (chunk = 0) or one chunk of one
// phase (chunk = 1, long pulses).
size_t swap_lds_bytes(int N, int j, int K, int chunk);
hipError_t launch_swap(int filter, int J, int N, const void *rx, long long n, long long count,
                       long long rx_stride, void *tree, const SwapDesc &wd, size_t lds_bytes,
                       int chunked, void *out, long long out_stride, hipStream_t st);

}  // namespace sidwt
