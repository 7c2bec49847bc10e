// Workgroup-wide y-side lifting of one level (Fig. 7 dataflow) and the
// level-1 loaders of the caller's pulse, shared by the kernels that lift in
// LDS (sidwt_kernels.hip, sidwt_int8.hip).
#pragma once
#include "sidwt_device.hpp"

namespace sidwt {

// ===========================================================================
// y-side lifting of one level across the workgroup (Fig. 7).  Each wave
// takes windows of 64 consecutive pairs; HL/HR edge lanes only feed their
// neighbours (shuffles), the remaining lanes own their pair.  `load(kc, e,
// o)` fetches pair kc (0 <= kc < np) of the level input; `store(k, c, d)`
// receives the owned outputs.
// ===========================================================================
template <int F, int UNROLL, bool WIDE, class Load, class Store>
__device__ __forceinline__ void lift_windows(int np, int k0, int k1, Load load, Store store) {
  using L = YLift<F>;
  using V = typename L::V;
  constexpr int OWN = 64 - L::HL - L::HR;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int nwin = (k1 - k0 + OWN - 1) / OWN;
  for (int w0 = wave * UNROLL; w0 < nwin; w0 += nw * UNROLL) {
    V e[UNROLL], o[UNROLL];
    int kk[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const int k = k0 + (w0 + u) * OWN - L::HL + lane;
      kk[u] = k;
      int kc;
      if constexpr (WIDE) {
        // np >= 64: every needed index is in [-HL, np + HR); the rest only
        // has to stay in bounds
        kc = k < 0 ? k + np : (k >= np ? k - np : k);
        kc = kc < np ? kc : np - 1;
      } else {
        kc = pos_mod(k, np);
      }
      load(kc, e[u], o[u]);
    }
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) L::run(e[u], o[u]);
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      int k = kk[u];
      if (lane >= L::HL && lane < 64 - L::HR && k < k1 && (w0 + u) < nwin) store(k, e[u], o[u]);
    }
  }
}

template <int F, int UNROLL, class Load, class Store>
__device__ __forceinline__ void lift_level_range(int np, int k0, int k1, Load load, Store store) {
  // the wrap is chosen once per level so that the unrolled loads carry no
  // per-load branch (and no integer division when the level is wide)
  if (np >= 64)
    lift_windows<F, UNROLL, true>(np, k0, k1, load, store);
  else
    lift_windows<F, UNROLL, false>(np, k0, k1, load, store);
}

template <int F, int UNROLL, class Load, class Store>
__device__ __forceinline__ void lift_level(int np, Load load, Store store) {
  lift_level_range<F, UNROLL>(np, 0, np, load, store);
}

// Pair kc of a circular sequence of length 2*np held in `src` (LDS or
// global); for the causal D4 form the odd member is u[2k-1].
template <bool ODD_BEFORE, class V>
__device__ __forceinline__ void pair_at(const V *src, int kc, int np, V &e, V &o) {
  e = src[2 * kc];
  o = ODD_BEFORE ? src[kc == 0 ? 2 * np - 1 : 2 * kc - 1] : src[2 * kc + 1];
}

// Level-1 input from the caller's pulse: complex64, or int16 I/Q widened to
// int32.  Samples at index >= n are the zero padding up to N (n <= N < 2^31).
// Branch-free: the load reads a clamped in-bounds index and the zero is
// selected afterwards, so unrolled loads are not split by branches.
__device__ __forceinline__ float2 rx_sample(const float2 *rx, int n, int i) {
  const float2 v = rx[i < n ? i : n - 1];
  return (i < n) ? v : make_float2(0.f, 0.f);
}
// A pulse reached through a batch descriptor: the compiler cannot tell its
// address space and would issue flat loads; these read it as global memory.
typedef float f32x2_global __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 rx_sample_global(const float2 *rx, int n, int i) {
  const __attribute__((address_space(1))) f32x2_global *g =
      (const __attribute__((address_space(1))) f32x2_global *)rx;
  const f32x2_global v = g[i < n ? i : n - 1];
  return (i < n) ? make_float2(v.x, v.y) : make_float2(0.f, 0.f);
}
__device__ __forceinline__ int2 rx_sample(const short2 *rx, int n, int i) {
  const short2 s = rx[i < n ? i : n - 1];
  return (i < n) ? make_int2(s.x, s.y) : make_int2(0, 0);
}

}  // namespace sidwt
