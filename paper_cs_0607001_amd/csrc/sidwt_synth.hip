// Coarse-to-fine formation for gfx950: the inverse of the y-side (dual
// analysis) lifting, level by level (eq. (21): the finer approximation is
// synthesized from the coarser approximation and detail by the lifting steps
// undone in reverse order).  Input: the critical pyramid that sidwt_lift_many
// writes, d_1 | d_2 | ... | d_J | c_J (N elements per pulse); output: the
// approximation c_to (N >> to elements; c_0 is the zero-padded pulse).  The
// correlation of a finer plane needs c_l of that level, so a caller that
// correlated the coarse planes first can form the finer ones from the stored
// pyramid without lifting the pulse again (Sec. V).
#include <type_traits>

#include "sidwt_device.hpp"

namespace sidwt {

constexpr int kSynthThreads = 512;

// One level, in place: E holds c_l, O holds d_l (L pairs each), both already
// multiplied by kE / kO (the inverse of the final diagonal scaling); on
// return E holds the even and O the odd samples of c_{l-1} (for D4: O[k] is
// sample 2k - 1, the pairing of the forward steps).  A pass that reads only
// the array it does not write works in place; D4 needs one scratch array T
// (kBuffers = 3).
template <int F> struct YSynth;

template <> struct YSynth<F_LEGALL53> {
  // undo diag(1, 2), then [1 0; -(1+z)/4 1], then [1 (1+z^-1)/2; 0 1]
  static constexpr float kE = 1.0f, kO = 0.5f;
  static constexpr int kBuffers = 2;
  __device__ static void run(float2 *E, float2 *O, float2 *, int L, int tid, int nt) {
    for (int k = tid; k < L; k += nt) {
      const int k1 = k + 1 == L ? 0 : k + 1;
      O[k] = fma2(0.25f, add2(E[k], E[k1]), O[k]);
    }
    __syncthreads();
    for (int k = tid; k < L; k += nt) {
      const int km = k == 0 ? L - 1 : k - 1;
      E[k] = fma2(-0.5f, add2(O[km], O[k]), E[k]);
    }
    __syncthreads();
  }
};

template <> struct YSynth<F_CDF97> {
  // undo diag(1/x, x), then the four steps d, g, b, a in reverse order
  static constexpr float kE = C97::xi, kO = C97::inv_xi;
  static constexpr int kBuffers = 2;
  __device__ static void run(float2 *E, float2 *O, float2 *, int L, int tid, int nt) {
    for (int k = tid; k < L; k += nt) {
      const int k1 = k + 1 == L ? 0 : k + 1;
      O[k] = fma2(C97::d, add2(E[k], E[k1]), O[k]);
    }
    __syncthreads();
    for (int k = tid; k < L; k += nt) {
      const int km = k == 0 ? L - 1 : k - 1;
      E[k] = fma2(C97::g, add2(O[km], O[k]), E[k]);
    }
    __syncthreads();
    for (int k = tid; k < L; k += nt) {
      const int k1 = k + 1 == L ? 0 : k + 1;
      O[k] = fma2(C97::b, add2(E[k], E[k1]), O[k]);
    }
    __syncthreads();
    for (int k = tid; k < L; k += nt) {
      const int km = k == 0 ? L - 1 : k - 1;
      E[k] = fma2(C97::a, add2(O[km], O[k]), E[k]);
    }
    __syncthreads();
  }
};

template <> struct YSynth<F_D4> {
  // undo eq. (17): e1 = c / ka, o2 = d / kb (the load scalings);
  // o1[k] = o2[k+1] - e1[k+1] (undoes [1 0; 1 z^-1]), into the scratch T;
  // e = e1 - u0 o1[k] - u1 o1[k-1]; o = o1 + sqrt3 e
  static constexpr float kE = 1.0f / CD4::ka, kO = 1.0f / CD4::kb;
  static constexpr int kBuffers = 3;
  __device__ static void run(float2 *E, float2 *O, float2 *T, int L, int tid, int nt) {
    for (int k = tid; k < L; k += nt) {
      const int k1 = k + 1 == L ? 0 : k + 1;
      T[k] = add2(O[k1], scale2(-1.0f, E[k1]));
    }
    __syncthreads();
    for (int k = tid; k < L; k += nt) {
      const int km = k == 0 ? L - 1 : k - 1;
      const float2 e = fma2(-CD4::u1, T[km], fma2(-CD4::u0, T[k], E[k]));
      E[k] = e;
      O[k] = fma2(CD4::s3, e, T[k]);
    }
    __syncthreads();
  }
};

template <> struct YSynth<F_LEGALL53_INT> {
  // exact inverse of the reversible steps: o += (e[k] + e[k+1] + 2) >> 2,
  // then e -= (o[k-1] + o[k] + 1) >> 1
  static constexpr float kE = 1.0f, kO = 1.0f;  // unused (no scaling)
  static constexpr int kBuffers = 2;
  __device__ static void run(int2 *E, int2 *O, int2 *, int L, int tid, int nt) {
    for (int k = tid; k < L; k += nt) {
      const int k1 = k + 1 == L ? 0 : k + 1;
      O[k].x += (E[k].x + E[k1].x + 2) >> 2;
      O[k].y += (E[k].y + E[k1].y + 2) >> 2;
    }
    __syncthreads();
    for (int k = tid; k < L; k += nt) {
      const int km = k == 0 ? L - 1 : k - 1;
      E[k].x -= (O[km].x + O[k].x + 1) >> 1;
      E[k].y -= (O[km].y + O[k].y + 1) >> 1;
    }
    __syncthreads();
  }
};

template <class V> __device__ __forceinline__ V scaled(float s, V v) { return scale2(s, v); }
template <> __device__ __forceinline__ int2 scaled<int2>(float, int2 v) { return v; }

// One workgroup per pulse.  LDS: X and Y (and T for D4) of Lmax = N >> (to
// + 1) elements.  Level l: X = c_l (scaled by kE), Y = d_l (scaled by kO);
// after the steps c_{l-1} goes to HBM at the last level, else it is
// interleaved into X, already scaled for the next level: top-down chunks of
// one pair per thread, each read before a barrier and written after it (a
// chunk from pair c0 on writes X[2 c0 ...], which no lower chunk reads).
template <int F>
__global__ __launch_bounds__(kSynthThreads) void synth_many(
    int J, int to, int N, const typename ElemOf<F>::T *__restrict__ pyr_all,
    typename ElemOf<F>::T *__restrict__ out_all) {
  using V = typename ElemOf<F>::T;
  using Y = YSynth<F>;
  constexpr bool OB = YLift<F>::kOddBefore;
  extern __shared__ __align__(16) char smem_synth[];
  const int Lmax = N >> (to + 1);
  V *X = reinterpret_cast<V *>(smem_synth);
  V *Yb = X + Lmax;
  V *T = Yb + Lmax;   // allocated for D4 only
  const V *pyr = pyr_all + (long long)blockIdx.x * N;
  V *out = out_all + (long long)blockIdx.x * (N >> to);
  const int tid = threadIdx.x, nt = blockDim.x;
  {
    const int L = N >> J;
    const V *c = pyr + (N - (N >> J));
    for (int k = tid; k < L; k += nt) X[k] = scaled(Y::kE, c[k]);
  }
  for (int l = J; l > to; --l) {
    const int L = N >> l;
    const V *d = pyr + (N - (N >> (l - 1)));
    for (int k = tid; k < L; k += nt) Yb[k] = scaled(Y::kO, d[k]);
    __syncthreads();
    Y::run(X, Yb, T, L, tid, nt);
    if (l - 1 == to) {
      for (int k = tid; k < L; k += nt) {
        out[2 * k] = X[k];
        out[2 * k + 1] = Yb[OB ? (k + 1 == L ? 0 : k + 1) : k];   // OB: Yb[k] is sample 2k - 1
      }
    } else {
      for (int c0 = ((L - 1) / nt) * nt; c0 >= 0; c0 -= nt) {
        const int k = c0 + tid;
        V ev{}, ov{};
        if (k < L) {
          ev = X[k];
          ov = Yb[OB ? (k + 1 == L ? 0 : k + 1) : k];
        }
        __syncthreads();
        if (k < L) {
          X[2 * k] = scaled(Y::kE, ev);
          X[2 * k + 1] = scaled(Y::kE, ov);
        }
        __syncthreads();
      }
    }
    __syncthreads();
  }
}

// LDS of one pulse.
template <int F> size_t synth_lds_bytes_t(int N, int to) {
  return (size_t)YSynth<F>::kBuffers * (N >> (to + 1)) * 8;
}
size_t synth_lds_bytes(int filter, int N, int to) {
  return filter == F_D4 ? synth_lds_bytes_t<F_D4>(N, to) : synth_lds_bytes_t<F_CDF97>(N, to);
}

template <int F>
static hipError_t launch_synth_t(int J, int to, int N, const void *pyr, long long count, void *out,
                                 hipStream_t st) {
  using V = typename ElemOf<F>::T;
  const size_t shm = synth_lds_bytes_t<F>(N, to);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)synth_many<F>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(synth_many<F>, dim3((unsigned)count), dim3(kSynthThreads), shm, st, J, to,
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
