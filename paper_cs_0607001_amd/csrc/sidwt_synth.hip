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

// One level: E holds c_l, O holds d_l (L pairs each); on return E holds the
// even and O the odd samples of c_{l-1} (for D4: O[k] is sample 2k - 1, the
// pairing of the forward steps).  T is scratch of L elements.  Every pass
// reads only the array it does not write, with a barrier after it.
template <int F> struct YSynth;

template <> struct YSynth<F_LEGALL53> {
  // undo: diag(1, 2), then [1 0; -(1+z)/4 1], then [1 (1+z^-1)/2; 0 1]
  __device__ static void run(float2 *E, float2 *O, float2 *, int L, int tid, int nt) {
    for (int k = tid; k < L; k += nt) {
      const int k1 = k + 1 == L ? 0 : k + 1;
      O[k] = fma2(0.25f, add2(E[k], E[k1]), scale2(0.5f, O[k]));
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
  // undo: diag(1/x, x), then the four steps d, g, b, a in reverse order
  __device__ static void run(float2 *E, float2 *O, float2 *, int L, int tid, int nt) {
    for (int k = tid; k < L; k += nt) {
      E[k] = scale2(C97::xi, E[k]);
      O[k] = scale2(C97::inv_xi, O[k]);
    }
    __syncthreads();
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
  // undo eq. (17): e1 = c / ka, o2 = d / kb; o1[k] = o2[k+1] - e1[k+1]
  // (undoes [1 0; 1 z^-1]); e = e1 - u0 o1[k] - u1 o1[k-1]; o = o1 + sqrt3 e
  __device__ static void run(float2 *E, float2 *O, float2 *T, int L, int tid, int nt) {
    const float ika = 1.0f / CD4::ka, ikb = 1.0f / CD4::kb;
    for (int k = tid; k < L; k += nt) {
      const int k1 = k + 1 == L ? 0 : k + 1;
      T[k] = add2(scale2(ikb, O[k1]), scale2(-ika, E[k1]));
    }
    __syncthreads();
    for (int k = tid; k < L; k += nt) {
      const int km = k == 0 ? L - 1 : k - 1;
      const float2 e = fma2(-CD4::u1, T[km], fma2(-CD4::u0, T[k], scale2(ika, E[k])));
      E[k] = e;
      O[k] = fma2(CD4::s3, e, T[k]);
    }
    __syncthreads();
  }
};

template <> struct YSynth<F_LEGALL53_INT> {
  // exact inverse of the reversible steps: o += (e[k] + e[k+1] + 2) >> 2,
  // then e -= (o[k-1] + o[k] + 1) >> 1
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

// One workgroup per pulse.  LDS: E, O, C of Lmax = N >> (to + 1) elements;
// C carries c_{l-1} to the next level (and is the D4 scratch before that).
template <int F>
__global__ __launch_bounds__(kSynthThreads) void synth_many(
    int J, int to, int N, const typename ElemOf<F>::T *__restrict__ pyr_all,
    typename ElemOf<F>::T *__restrict__ out_all) {
  using V = typename ElemOf<F>::T;
  constexpr bool OB = YLift<F>::kOddBefore;
  extern __shared__ __align__(16) char smem_synth[];
  const int Lmax = N >> (to + 1);
  V *E = reinterpret_cast<V *>(smem_synth);
  V *O = E + Lmax;
  V *C = O + Lmax;
  const V *pyr = pyr_all + (long long)blockIdx.x * N;
  V *out = out_all + (long long)blockIdx.x * (N >> to);
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int l = J; l > to; --l) {
    const int L = N >> l;
    const V *d = pyr + (N - (N >> (l - 1)));
    const V *c = l == J ? pyr + (N - (N >> J)) : C;
    for (int k = tid; k < L; k += nt) {
      E[k] = c[k];
      O[k] = d[k];
    }
    __syncthreads();
    YSynth<F>::run(E, O, C, L, tid, nt);
    V *dst = l - 1 == to ? out : C;
    for (int k = tid; k < L; k += nt) {
      dst[2 * k] = E[k];
      if (OB)
        dst[2 * k + 1] = O[k + 1 == L ? 0 : k + 1];   // O[k] is sample 2k - 1
      else
        dst[2 * k + 1] = O[k];
    }
    __syncthreads();
  }
}

size_t synth_lds_bytes(int N, int to) { return (size_t)3 * (N >> (to + 1)) * 8; }

template <int F>
static hipError_t launch_synth_t(int J, int to, int N, const void *pyr, long long count, void *out,
                                 hipStream_t st) {
  using V = typename ElemOf<F>::T;
  const size_t shm = synth_lds_bytes(N, to);
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
