// Coarse-to-fine formation for gfx950: the inverse of the y-side (dual
// analysis) lifting, level by level (eq. (21): the finer approximation is
// synthesized from the coarser approximation and detail by the lifting steps
// undone in reverse order).  Input: the critical pyramid that sidwt_lift_many
// writes, d_1 | d_2 | ... | d_J | c_J (N elements per pulse); output: the
// approximation c_to (N >> to elements; c_0 is the zero-padded pulse).  The
// correlation of a finer plane needs c_l of that level, so a caller that
// correlated the coarse planes first can form the finer ones from the stored
// pyramid without lifting the pulse again (Sec. V).
#include <atomic>

#include <type_traits>

#include "sidwt_device.hpp"

namespace sidwt {

// Workgroup size: 8 waves for the float filters, 4 for the integer filter
// (its pulses are shorter and its levels more numerous per byte; measured
// faster with more, smaller workgroups).
template <int F> struct SynthCfg { static constexpr int kThreads = 512; };
template <> struct SynthCfg<F_LEGALL53_INT> { static constexpr int kThreads = 256; };

// One level of the inverse, in registers: lane k of a 64-lane window holds
// the pair (c_l[k] * kE, d_l[k] * kO) (kE, kO undo the final diagonal
// scaling) and leaves with (c_{l-1}[2k], c_{l-1}[2k+1]).  Neighbour taps come
// from the adjacent lanes; the HL leftmost and HR rightmost lanes of a window
// only feed their neighbours.
template <int F> struct YUnlift;

template <> struct YUnlift<F_LEGALL53> {
  // undo diag(1, 2), then [1 0; -(1+z)/4 1], then [1 (1+z^-1)/2; 0 1]
  static constexpr int HL = 1, HR = 1;
  static constexpr float kE = 1.0f, kO = 0.5f;
  __device__ __forceinline__ static void run(float2 &e, float2 &o) {
    o = fma2(0.25f, add2(e, lane_next(e)), o);
    e = fma2(-0.5f, add2(lane_prev(o), o), e);
  }
};

template <> struct YUnlift<F_CDF97> {
  // undo diag(1/x, x), then the four steps d, g, b, a in reverse order
  static constexpr int HL = 2, HR = 2;
  static constexpr float kE = C97::xi, kO = C97::inv_xi;
  __device__ __forceinline__ static void run(float2 &e, float2 &o) {
    o = fma2(C97::d, add2(e, lane_next(e)), o);
    e = fma2(C97::g, add2(lane_prev(o), o), e);
    o = fma2(C97::b, add2(e, lane_next(e)), o);
    e = fma2(C97::a, add2(lane_prev(o), o), e);
  }
};

template <> struct YUnlift<F_D4> {
  // undo eq. (17) on pairs (u[2k], u[2k-1]): after the load scalings
  // e1 = c / ka and o2 = d / kb, o1[k] = o2[k+1] - e1[k+1] (undoes
  // [1 0; 1 z^-1]); e = e1 - u0 o1[k] - u1 o1[k-1]; u[2k-1] = o1 + sqrt3 e.
  // The odd output is then taken from the next lane (u[2k+1]).
  static constexpr int HL = 1, HR = 2;
  static constexpr float kE = 1.0f / CD4::ka, kO = 1.0f / CD4::kb;
  __device__ __forceinline__ static void run(float2 &e, float2 &o) {
    const float2 t = lane_next(add2(o, scale2(-1.0f, e)));
    e = fma2(-CD4::u1, lane_prev(t), fma2(-CD4::u0, t, e));
    o = lane_next(fma2(CD4::s3, e, t));
  }
};

template <> struct YUnlift<F_LEGALL53_INT> {
  // exact inverse of the reversible steps: o += (e[k] + e[k+1] + 2) >> 2,
  // then e -= (o[k-1] + o[k] + 1) >> 1
  static constexpr int HL = 1, HR = 1;
  static constexpr float kE = 1.0f, kO = 1.0f;  // unused (no scaling)
  __device__ __forceinline__ static void run(int2 &e, int2 &o) {
    const int2 en = lane_next(e);
    o.x += (e.x + en.x + 2) >> 2;
    o.y += (e.y + en.y + 2) >> 2;
    const int2 op = lane_prev(o);
    e.x -= (op.x + o.x + 1) >> 1;
    e.y -= (op.y + o.y + 1) >> 1;
  }
};

template <class V> __device__ __forceinline__ V scaled(float s, V v) { return scale2(s, v); }
template <> __device__ __forceinline__ int2 scaled<int2>(float, int2 v) { return v; }

// Two consecutive elements in one 16-byte store: to LDS, or streamed to HBM
// (written once, never read back by this kernel).
__device__ __forceinline__ void store_pair(float2 *dst, float2 a, float2 b) {
  *reinterpret_cast<float4 *>(dst) = make_float4(a.x, a.y, b.x, b.y);
}
__device__ __forceinline__ void store_pair(int2 *dst, int2 a, int2 b) {
  *reinterpret_cast<int4 *>(dst) = make_int4(a.x, a.y, b.x, b.y);
}
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef int i32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void stream_pair(float2 *dst, float2 a, float2 b) {
  __builtin_nontemporal_store(f32x4_t{a.x, a.y, b.x, b.y}, reinterpret_cast<f32x4_t *>(dst));
}
__device__ __forceinline__ void stream_pair(int2 *dst, int2 a, int2 b) {
  __builtin_nontemporal_store(i32x4_t{a.x, a.y, b.x, b.y}, reinterpret_cast<i32x4_t *>(dst));
}

// One level over the workgroup: each wave takes UNROLL windows of 64 lanes
// at a time (64 - HL - HR owned pairs each, circular indices).
// `load(kc, e, o)` fetches pair kc in [0, L); `store(k, e, o)` receives the
// owned outputs c_{l-1}[2k], c_{l-1}[2k+1].
template <int F, int UNROLL, class Load, class Store>
__device__ __forceinline__ void unlift_level(int L, Load load, Store store) {
  using U = YUnlift<F>;
  using V = typename ElemOf<F>::T;
  constexpr int OWN = 64 - U::HL - U::HR;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int nwin = (L + OWN - 1) / OWN;
  const bool wide = L >= 64;
  for (int w0 = wave * UNROLL; w0 < nwin; w0 += nw * UNROLL) {
    V e[UNROLL], o[UNROLL];
    int kk[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const int k = (w0 + u) * OWN - U::HL + lane;
      kk[u] = k;
      int kc;
      if (wide) {
        // every index a stored output needs lies in [-HL, L + HR); the
        // rest (windows past the end) only has to stay in bounds
        kc = k < 0 ? k + L : (k >= L ? k - L : k);
        kc = kc < L ? kc : L - 1;
      } else {
        kc = pos_mod(k, L);
      }
      load(kc, e[u], o[u]);
    }
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) U::run(e[u], o[u]);
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const int k = kk[u];
      if (lane >= U::HL && lane < 64 - U::HR && k < L && (w0 + u) < nwin) store(k, e[u], o[u]);
    }
  }
}

// One workgroup per pulse.  c_J and every d_l are read from the pyramid in
// HBM; the intermediate approximations c_{J-1} ... c_{to+1} alternate
// between two LDS buffers (P: N >> (to+1) elements, holding c_{to+1},
// c_{to+3}, ...; Q: half that, holding c_{to+2}, c_{to+4}, ...), one barrier
// per level; c_to goes straight to HBM.  Separate load / store lambdas per
// source and destination keep every pointer's address space known to the
// compiler (LDS and global instructions, no flat ones).
template <int F>
__global__ __launch_bounds__(SynthCfg<F>::kThreads) void synth_many(
    int J, int to, int N, const typename ElemOf<F>::T *__restrict__ pyr_all,
    typename ElemOf<F>::T *__restrict__ out_all) {
  using V = typename ElemOf<F>::T;
  using U = YUnlift<F>;
  constexpr int UNROLL = 2;
  extern __shared__ __align__(16) char smem_synth[];
  const int Lmax = N >> (to + 1);
  V *const P = reinterpret_cast<V *>(smem_synth);
  V *const Q = P + Lmax;
  const V *pyr = pyr_all + (long long)blockIdx.x * N;
  V *out = out_all + (long long)blockIdx.x * (N >> to);
  const V *cJ = pyr + (N - (N >> J));
  for (int l = J; l > to; --l) {
    const int L = N >> l;
    const V *d = pyr + (N - (N >> (l - 1)));
    const V *c = ((l - to - 1) & 1) ? Q : P;         // c_l (l < J)
    V *cn = ((l - to - 2) & 1) ? Q : P;              // c_{l-1} (l - 1 > to)
    auto load_hbm = [&](int kc, V &e, V &o) {
      e = scaled(U::kE, cJ[kc]);
      o = scaled(U::kO, d[kc]);
    };
    auto load_lds = [&](int kc, V &e, V &o) {
      e = scaled(U::kE, c[kc]);
      o = scaled(U::kO, d[kc]);
    };
    auto store_lds = [&](int k, V e, V o) { store_pair(cn + 2 * k, e, o); };
    auto store_hbm = [&](int k, V e, V o) { stream_pair(out + 2 * k, e, o); };
    auto level = [&](auto load) {
      if (l - 1 == to)
        unlift_level<F, UNROLL>(L, load, store_hbm);
      else
        unlift_level<F, UNROLL>(L, load, store_lds);
    };
    if (l == J)
      level(load_hbm);
    else
      level(load_lds);
    __syncthreads();
  }
}

// LDS of one pulse.
size_t synth_lds_bytes(int, int N, int to) {
  const size_t Lmax = (size_t)(N >> (to + 1));
  return (Lmax + Lmax / 2) * 8;
}

template <int F>
static hipError_t launch_synth_t(int J, int to, int N, const void *pyr, long long count, void *out,
                                 hipStream_t st) {
  using V = typename ElemOf<F>::T;
  const size_t shm = synth_lds_bytes(F, N, to);
  static std::atomic<bool> attr_set{false};  // set once per process (calls may race: both set it)
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)synth_many<F>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(synth_many<F>, dim3((unsigned)count), dim3(SynthCfg<F>::kThreads), shm, st, J, to,
                     N, static_cast<const V *>(pyr), static_cast<V *>(out));
  return hipGetLastError();
}

hipError_t launch_synth(int filter, int J, int to, int N, const void *pyr, long long count,
                        void *out, hipStream_t st) {
  switch (filter) {
    case F_LEGALL53: return launch_synth_t<F_LEGALL53>(J, to, N, pyr, count, out, st);
    case F_CDF97: return launch_synth_t<F_CDF97>(J, to, N, pyr, count, out, st);
    case F_D4: return launch_synth_t<F_D4>(J, to, N, pyr, count, out, st);
    case F_LEGALL53_INT: return launch_synth_t<F_LEGALL53_INT>(J, to, N, pyr, count, out, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sidwt
