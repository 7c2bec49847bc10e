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

// Block order of the tree launches (grid = count << j blocks, block x of
// level j -> pulse and child phase p = pp + 2^(j-1) b).  Blocks go to the
// eight XCDs round-robin (x to XCD x mod 8), and the two children b = 0, 1
// of one parent phase read the same parent sequence.  Within every whole
// group of 16 blocks, blocks x and x + 8 (one XCD, dispatched one after the
// other) take the two children of one parent, so the second read finds the
// parent in that XCD's L2; blocks of a trailing partial group keep the
// plain order (b the low bit of the index there too).
__host__ __device__ inline void swap_tree_block(long long x, long long G, int j, long long &pulse,
                                                int &p) {
  const long long q = x < (G & ~15LL) ? ((x & ~15LL) | ((x & 7) << 1) | ((x >> 3) & 1)) : x;
  const int b = (int)(q & 1);
  const long long r = q >> 1;
  const int pp = (int)(r & ((1LL << (j - 1)) - 1));
  pulse = r >> (j - 1);
  p = pp | (b << (j - 1));
}

// LDS of plane j's work item: whole plane (chunk = 0) or one chunk of one
// phase (chunk = 1, long pulses).
size_t swap_lds_bytes(int N, int j, int K, int chunk);
hipError_t launch_swap(int filter, int J, int N, const void *rx, long long n, long long count,
                       long long rx_stride, void *tree, const SwapDesc &wd, size_t lds_bytes,
                       int chunked, void *out, long long out_stride, hipStream_t st);

}  // namespace sidwt
