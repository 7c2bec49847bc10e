// Critical lifting of a batch with any factorized filter pair (eq. (16)):
// the steps come at run time from the host factorizer (sidwt_factor.cpp)
// instead of being compiled in, for filter pairs the specialised kernels do
// not carry.  Same output as sidwt_lift_many: per pulse d_1 | ... | d_J | c_J
// (complex64, N elements), I and Q lifted alike (Sec. IV).
//
// One workgroup per pulse; c_l (l < J) in LDS at alternating offsets 0 and
// N/2; each level in 64-lane register windows where a step's taps at offset
// v come from lane + v (ds_bpermute shuffles), so the HL leftmost and HR
// rightmost lanes of a window only feed their neighbours.
#include <atomic>

#include <hip/hip_runtime.h>

#include "sidwt_device.hpp"
#include "sidwt_factor.hpp"

namespace sidwt {

constexpr int kGenericThreads = 512;

// Single-precision copy of a factorization, with the window halos.
struct GenericSteps {
  int n;
  int kind[kMaxLiftSteps];
  int lo[kMaxLiftSteps];
  int len[kMaxLiftSteps];
  float c[kMaxLiftSteps][kMaxLiftTaps];
  float ke, ko;
  int se, so;
  int HL, HR;
};

__device__ __forceinline__ float2 lane_at(float2 v, int src) {
  return make_float2(__shfl(v.x, src), __shfl(v.y, src));
}

__device__ __forceinline__ void stream_store(float2 *p, float2 v) {
  typedef float f2 __attribute__((ext_vector_type(2)));
  __builtin_nontemporal_store(f2{v.x, v.y}, reinterpret_cast<f2 *>(p));
}

// Steps of one window, in place on the lane's pair.  TWO_TAP: the shape of
// the paper's factorizations (every predict step reads e[k], e[k+1], every
// update step o[k-1], o[k], no shifts, at most kSmallSteps steps): one DPP
// neighbour per step.  SMALL: at most kSmallSteps steps of at most
// kSmallTaps taps, loops unrolled with predication so every coefficient sits
// at a fixed kernel-argument offset (loaded once, ahead of the arithmetic);
// otherwise plain loops.
constexpr int kSmallSteps = 8;
constexpr int kSmallTaps = 4;

__device__ __forceinline__ void run_two_tap(const GenericSteps &st, float2 &e, float2 &o) {
#pragma unroll
  for (int s = 0; s < kSmallSteps; ++s) {
    if (s >= st.n) break;
    const float c0 = st.c[s][0], c1 = st.c[s][1];
    if (st.kind[s] == kPredict) {
      const float2 en = lane_next(e);
      o = fma2(c1, en, fma2(c0, e, o));
    } else {
      const float2 op = lane_prev(o);
      e = fma2(c1, o, fma2(c0, op, e));
    }
  }
  e = scale2(st.ke, e);
  o = scale2(st.ko, o);
}

// The two-tap shape with NS alternating steps known at compile time (the
// first a predict step when PRED_FIRST): only the coefficients are read at
// run time.
template <int NS, bool PRED_FIRST>
__device__ __forceinline__ void run_alternating(const GenericSteps &st, float2 &e, float2 &o) {
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const float c0 = st.c[s][0], c1 = st.c[s][1];
    if (((s & 1) == 0) == PRED_FIRST) {
      const float2 en = lane_next(e);
      o = fma2(c1, en, fma2(c0, e, o));
    } else {
      const float2 op = lane_prev(o);
      e = fma2(c1, o, fma2(c0, op, e));
    }
  }
  e = scale2(st.ke, e);
  o = scale2(st.ko, o);
}

template <bool SMALL>
__device__ __forceinline__ void run_steps(const GenericSteps &st, int lane, float2 &e, float2 &o) {
  constexpr int MS = SMALL ? kSmallSteps : kMaxLiftSteps;
  constexpr int MT = SMALL ? kSmallTaps : kMaxLiftTaps;
#pragma unroll
  for (int s = 0; s < MS; ++s) {
    if (s >= st.n) break;
    const bool pred = st.kind[s] == kPredict;
    const float2 src = pred ? e : o;
    float2 acc = make_float2(0.f, 0.f);
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      if (t >= st.len[s]) break;
      const float2 v = lane_at(src, lane + st.lo[s] + t);
      acc.x = fmaf(st.c[s][t], v.x, acc.x);
      acc.y = fmaf(st.c[s][t], v.y, acc.y);
    }
    if (pred)
      o = add2(o, acc);
    else
      e = add2(e, acc);
  }
  const float2 ce = lane_at(e, lane + st.se), co = lane_at(o, lane + st.so);
  e = scale2(st.ke, ce);
  o = scale2(st.ko, co);
}

// 0: loops, 1: unrolled shuffles, 2: two-tap DPP, 3 / 4: two / four
// alternating two-tap steps starting with a predict step, 5 / 6: the same
// starting with an update step
template <int MODE>
__global__ __launch_bounds__(kGenericThreads) void lift_generic(
    GenericSteps st, int J, int N, const float2 *__restrict__ rx_all, long long n,
    long long rx_stride, float2 *__restrict__ pyr_all) {
  constexpr int U = 2;  // windows in flight per wave
  extern __shared__ __align__(16) float2 smem_gen[];
  const long long pulse = blockIdx.x;
  const float2 *rx = rx_all + pulse * rx_stride;
  float2 *pyr = pyr_all + pulse * (long long)N;
  const int ni = (int)n;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int OWN = 64 - st.HL - st.HR;
  for (int l = 1; l <= J; ++l) {
    const int np = N >> l;
    const float2 *cin = smem_gen + (((l - 1) & 1) ? 0 : (N >> 1));  // c_{l-1} (l >= 2)
    float2 *cs = smem_gen + ((l & 1) ? 0 : (N >> 1));              // c_l (l < J)
    float2 *dg = pyr + (N - (N >> (l - 1)));
    float2 *cg = pyr + (N - np);
    const int nwin = (np + OWN - 1) / OWN;
    const bool wide = np >= 64;  // every needed index lies in [-HL, np + HR)
    for (int w0 = wave * U; w0 < nwin; w0 += nw * U) {
      float2 e[U], o[U];
      int kk[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = (w0 + u) * OWN - st.HL + lane;
        kk[u] = k;
        int kc;
        if (wide) {
          kc = k < 0 ? k + np : (k >= np ? k - np : k);
          kc = kc < np ? kc : np - 1;  // windows past the end only stay in bounds
        } else {
          kc = pos_mod(k, np);
        }
        if (l == 1) {
          e[u] = 2 * kc < ni ? rx[2 * kc] : make_float2(0.f, 0.f);
          o[u] = 2 * kc + 1 < ni ? rx[2 * kc + 1] : make_float2(0.f, 0.f);
        } else {
          e[u] = cin[2 * kc];
          o[u] = cin[2 * kc + 1];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if constexpr (MODE == 2)
          run_two_tap(st, e[u], o[u]);
        else if constexpr (MODE == 3)
          run_alternating<2, true>(st, e[u], o[u]);
        else if constexpr (MODE == 4)
          run_alternating<4, true>(st, e[u], o[u]);
        else if constexpr (MODE == 5)
          run_alternating<2, false>(st, e[u], o[u]);
        else if constexpr (MODE == 6)
          run_alternating<4, false>(st, e[u], o[u]);
        else
          run_steps<MODE == 1>(st, lane, e[u], o[u]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = kk[u];
        if (lane >= st.HL && lane < 64 - st.HR && k < np && w0 + u < nwin) {
          stream_store(dg + k, o[u]);
          if (l == J)
            stream_store(cg + k, e[u]);
          else
            cs[k] = e[u];
        }
      }
    }
    __syncthreads();
  }
}

// Halos: a step reading lanes lane + lo .. lane + lo + len - 1 widens the
// invalid edge regions by max(0, -lo) on the left and max(0, lo + len - 1)
// on the right; so do the final shifts.
bool generic_steps(const LiftingDesc &d, GenericSteps *g) {
  g->n = d.n;
  int HL = 0, HR = 0;
  for (int s = 0; s < d.n; ++s) {
    g->kind[s] = d.kind[s];
    g->lo[s] = d.lo[s];
    g->len[s] = d.len[s];
    for (int t = 0; t < kMaxLiftTaps; ++t) g->c[s][t] = t < d.len[s] ? (float)d.c[s][t] : 0.f;
    HL += d.lo[s] < 0 ? -d.lo[s] : 0;
    HR += d.lo[s] + d.len[s] - 1 > 0 ? d.lo[s] + d.len[s] - 1 : 0;
  }
  g->ke = (float)d.ke;
  g->ko = (float)d.ko;
  g->se = d.se;
  g->so = d.so;
  const int smin = d.se < d.so ? d.se : d.so, smax = d.se > d.so ? d.se : d.so;
  HL += smin < 0 ? -smin : 0;
  HR += smax > 0 ? smax : 0;
  g->HL = HL;
  g->HR = HR;
  return HL + HR <= 48;
}

bool generic_steps_fit(const LiftingDesc &d) {
  GenericSteps g;
  return generic_steps(d, &g);
}

size_t generic_lds_bytes(int N) { return (size_t)(N / 2 + N / 4 + 1) * 8; }

template <int MODE>
static hipError_t launch_generic_t(const GenericSteps &g, int J, int N, const void *rx,
                                   long long n, long long count, long long rx_stride, void *pyr,
                                   hipStream_t st) {
  static std::atomic<bool> attr_set{false};  // set once per process (calls may race: both set it)
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)lift_generic<MODE>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(lift_generic<MODE>, dim3((unsigned)count), dim3(kGenericThreads),
                     generic_lds_bytes(N), st, g, J, N, static_cast<const float2 *>(rx), n,
                     rx_stride, static_cast<float2 *>(pyr));
  return hipGetLastError();
}

hipError_t launch_generic(const LiftingDesc &d, int J, int N, const void *rx, long long n,
                          long long count, long long rx_stride, void *pyr, hipStream_t st) {
  GenericSteps g;
  if (!generic_steps(d, &g)) return hipErrorInvalidValue;
  bool small = d.n <= kSmallSteps;
  bool two = small && d.se == 0 && d.so == 0;
  for (int s = 0; s < d.n; ++s) {
    small = small && d.len[s] <= kSmallTaps;
    two = two && d.len[s] == 2 && d.lo[s] == (d.kind[s] == kPredict ? 0 : -1);
  }
  if (two && (d.n == 2 || d.n == 4)) {
    bool alt = true;
    for (int s = 1; s < d.n; ++s) alt = alt && d.kind[s] != d.kind[s - 1];
    if (alt) {
      const bool pf = d.kind[0] == kPredict;
      if (d.n == 2)
        return pf ? launch_generic_t<3>(g, J, N, rx, n, count, rx_stride, pyr, st)
                  : launch_generic_t<5>(g, J, N, rx, n, count, rx_stride, pyr, st);
      return pf ? launch_generic_t<4>(g, J, N, rx, n, count, rx_stride, pyr, st)
                : launch_generic_t<6>(g, J, N, rx, n, count, rx_stride, pyr, st);
    }
  }
  if (two) return launch_generic_t<2>(g, J, N, rx, n, count, rx_stride, pyr, st);
  if (small) return launch_generic_t<1>(g, J, N, rx, n, count, rx_stride, pyr, st);
  return launch_generic_t<0>(g, J, N, rx, n, count, rx_stride, pyr, st);
}

}  // namespace sidwt
