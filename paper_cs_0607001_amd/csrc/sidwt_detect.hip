// Target declaration on the correlation planes for gfx950 (Sec. V-A,
// Fig. 6: targets are read off the magnitude of each scale's correlation
// as peaks above a level).  A lag s of a plane is a peak when its power
// p[s] = Re^2 + Im^2 exceeds p[s-1], is not below p[s+1] (the first sample
// of a flat top; lags are circular) and is not below rel * max(p).  Every
// decision uses single precision with one rounding per operation (no fused
// multiply-add), so it is reproducible off the GPU.
//
// One workgroup per (pulse, plane): a block maximum (the powers kept in LDS
// when the plane fits), then the lags in chunks of eight per thread; each
// chunk's peaks are compacted in lag order by wave ballots and one scan of
// their counts, so the output order is deterministic and no atomics are
// used.
#include <atomic>

#include <hip/hip_runtime.h>

namespace sidwt {

constexpr int kDetectThreads = 256;

// Each square and the sum rounded separately: contraction into a fused
// multiply-add is switched off here (the compiler would otherwise form one).
__device__ __forceinline__ float plane_power(float2 z) {
#pragma clang fp contract(off)
  const float a = z.x * z.x;
  const float b = z.y * z.y;
  return a + b;
}

// LDS: the plane's powers (N floats) when they fit, so the plane is read
// from HBM once; otherwise the neighbours are re-read from global memory.
template <bool LDS>
__global__ __launch_bounds__(kDetectThreads) void detect_peaks(
    const float2 *__restrict__ planes, long long pulse_stride, int J, int N, float rel,
    int max_peaks, int *__restrict__ lags, float *__restrict__ db, int *__restrict__ found) {
  constexpr int NW = kDetectThreads / 64;
  constexpr int U = 4;  // independent loads in flight per thread
  __shared__ float wmax[NW];
  extern __shared__ float sp[];
  const long long item = blockIdx.x;  // pulse * J + plane
  const long long pulse = item / J;
  const int j = (int)(item - pulse * J);
  const float2 *R = planes + pulse * pulse_stride + (long long)j * N;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  float m = 0.f;
  if ((reinterpret_cast<uintptr_t>(R) & 15) == 0 && (N & 1) == 0) {
    // two complex values per 16-byte load, 2U loads in flight per thread
    const float4 *R4 = reinterpret_cast<const float4 *>(R);
    const int N2 = N >> 1;
    for (int q0 = tid; q0 < N2; q0 += 2 * U * kDetectThreads) {
      float4 v[2 * U];
#pragma unroll
      for (int u = 0; u < 2 * U; ++u) {
        const int q = q0 + u * kDetectThreads;
        v[u] = q < N2 ? R4[q] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < 2 * U; ++u) {
        const int q = q0 + u * kDetectThreads;
        const float p0 = plane_power(make_float2(v[u].x, v[u].y));
        const float p1 = plane_power(make_float2(v[u].z, v[u].w));
        if (LDS && q < N2) {
          sp[2 * q] = p0;
          sp[2 * q + 1] = p1;
        }
        m = fmaxf(m, fmaxf(p0, p1));
      }
    }
  } else {
    for (int s0 = tid; s0 < N; s0 += U * kDetectThreads) {
      float2 v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int s = s0 + u * kDetectThreads;
        v[u] = s < N ? R[s] : make_float2(0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int s = s0 + u * kDetectThreads;
        const float p = plane_power(v[u]);
        if (LDS && s < N) sp[s] = p;
        m = fmaxf(m, p);
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if (lane == 0) wmax[wave] = m;
  __syncthreads();
  float M = wmax[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) M = fmaxf(M, wmax[w]);
  const float thr = rel * M;
  auto power_at = [&](int s) { return LDS ? sp[s] : plane_power(R[s]); };

  int *ol = lags + item * max_peaks;
  float *od = db + item * max_peaks;
  // Lags in chunks of CU * 256: thread tid tests lags c0 + u * 256 + tid
  // (u < CU), so peaks in (u, wave, lane) order are in lag order; one
  // exclusive scan of the per-(u, wave) ballot counts places them.
  constexpr int CU = 8;
  __shared__ int wpre[CU * NW + 1];
  int base = 0;
  for (int c0 = 0; c0 < N; c0 += CU * kDetectThreads) {
    unsigned long long bal[CU];
    bool pk[CU];
    float psv[CU];
#pragma unroll
    for (int u = 0; u < CU; ++u) {
      const int s = c0 + u * kDetectThreads + tid;
      pk[u] = false;
      psv[u] = 0.f;
      if (s < N) {
        const float ps = power_at(s);
        const float pl = power_at(s == 0 ? N - 1 : s - 1);
        const float pr = power_at(s + 1 == N ? 0 : s + 1);
        pk[u] = ps > pl && ps >= pr && ps >= thr;
        psv[u] = ps;
      }
      bal[u] = __ballot(pk[u]);
    }
    __syncthreads();  // every wave has read the previous chunk's offsets
    if (lane == 0) {
#pragma unroll
      for (int u = 0; u < CU; ++u) wpre[u * NW + wave] = __popcll(bal[u]);
    }
    __syncthreads();
    if (tid == 0) {
      int acc = 0;
      for (int x = 0; x < CU * NW; ++x) {
        const int c = wpre[x];
        wpre[x] = acc;
        acc += c;
      }
      wpre[CU * NW] = acc;
    }
    __syncthreads();
    const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
    for (int u = 0; u < CU; ++u) {
      if (pk[u]) {
        const int k = base + wpre[u * NW + wave] + __popcll(bal[u] & below);
        if (k < max_peaks) {
          ol[k] = c0 + u * kDetectThreads + tid;
          od[k] = 10.f * log10f(psv[u] / M);
        }
      }
    }
    base += wpre[CU * NW];
  }
  if (tid == 0) found[item] = base;
}

constexpr int kDetectLdsBytes = 160 * 1024 - 256;  // beside the static arrays (160 B)

hipError_t launch_detect(const void *planes, long long pulse_stride, int J, int N, long long count,
                         float rel, int max_peaks, int *lags, float *db, int *found,
                         hipStream_t st) {
  const size_t lds = (size_t)N * 4;
  if (lds <= (size_t)kDetectLdsBytes) {
    static std::atomic<bool> attr_set{false};  // set once per process (calls may race: both set it)
    if (!attr_set) {
      hipError_t e = hipFuncSetAttribute((const void *)detect_peaks<true>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         kDetectLdsBytes);
      if (e != hipSuccess) return e;
      attr_set = true;
    }
    hipLaunchKernelGGL(detect_peaks<true>, dim3((unsigned)(count * J)), dim3(kDetectThreads), lds,
                       st, static_cast<const float2 *>(planes), pulse_stride, J, N, rel,
                       max_peaks, lags, db, found);
  } else {
    hipLaunchKernelGGL(detect_peaks<false>, dim3((unsigned)(count * J)), dim3(kDetectThreads), 0,
                       st, static_cast<const float2 *>(planes), pulse_stride, J, N, rel,
                       max_peaks, lags, db, found);
  }
  return hipGetLastError();
}

}  // namespace sidwt
