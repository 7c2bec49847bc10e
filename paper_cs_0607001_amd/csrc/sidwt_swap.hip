// Roles-exchanged correlation for gfx950: the received pulse gets the
// redundant (all-shift) y-side analysis and the reference only its critical
// x-side one (Sec. I: the redundant transform may sit on either signal; the
// approximation form of eq. (20a) at every scale).  Plane j, lag s:
//
//   R'_j[s] = sum_k conj(a_j[k]) * Y_{j,s mod 2^j}[k + s / 2^j]
//
// where a_j is the level-j x-side approximation of the reference (phase 0 of
// the plan's tree; a_0 is the reference itself) and Y_{j,p} is the level-j
// y-side approximation of the received pulse advanced by p samples
// (0 <= p < 2^j; Y_{0,0} is the pulse).  A shift of the pulse shifts every
// plane by exactly as many lags.
//
// Two kernels:
//  * swap_tree_level: level j of the redundant tree (approximations only),
//    phase-major (phase p of level j at p * (N >> j) of the level's block),
//    from level j - 1: child p = p' + 2^(j-1) b is the lifting of parent
//    phase p' advanced by b samples.  Register windows with lane-shift taps.
//  * swap_correlate: one workgroup per (pulse, plane) (pulses too long for
//    that: swap_correlate_chunks, one per (pulse, plane, phase, group of
//    tiles)); the phases go to LDS, extended by the weight span so no window
//    wraps, in 16-way polyphase order as re and im planes grouped in quads
//    (one 16-byte read gives a row four consecutive offsets), and every
//    phase is a Toeplitz-blocked real GEMM on v_mfma_f32_32x32x2_f32: row i
//    of a tile holds lags 16 i .. 16 i + 15, the K axis runs over (offset v,
//    re/im) and the 32 columns over (lag t within the block, re/im) with
//    B[v][t] = conj(a)[v - t].
#include <atomic>

#include "sidwt_lift.hpp"
#include "sidwt_swap.hpp"

namespace sidwt {

constexpr int kSwapTreeThreads = 256;
constexpr int kSwapThreads = 512;
constexpr int kSwapRT = 2;  // row tiles per wave sharing one weight fragment

__device__ __forceinline__ f32x16 swap_mfma(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Redundant tree.  One level of one phase: the y-side lifting of a parent
// sequence of Lp samples (sample(i), i < Lp, circular) advanced by b
// samples, L = Lp / 2 outputs (store(k, v)), in register windows of 64
// lanes with lane-shift taps, U windows per wave at a time (the loads of
// all U in flight together; 4 measured no faster than 2 from global memory).
// ---------------------------------------------------------------------------
template <int F, int U, class Sample, class Store>
__device__ __forceinline__ void tree_phase(int Lp, int b, Sample sample, Store store) {
  using Lf = YLift<F>;
  constexpr bool OB = Lf::kOddBefore;
  constexpr int OWN = 64 - Lf::HL - Lf::HR;
  const int L = Lp >> 1;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int nwin = (L + OWN - 1) / OWN;
  const bool wide = L >= 64;  // every index a stored output needs lies in [-HL, L + HR)
  for (int w0 = wave * U; w0 < nwin; w0 += nw * U) {
    float2 e[U], o[U];
    int kk[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = (w0 + u) * OWN - Lf::HL + lane;
      kk[u] = k;
      int kc;
      if (wide) {
        kc = k < 0 ? k + L : (k >= L ? k - L : k);
        kc = kc < L ? kc : L - 1;  // windows past the end only stay in bounds
      } else {
        kc = pos_mod(k, L);
      }
      const int ie = 2 * kc + b;  // < Lp
      const int io = OB ? (ie == 0 ? Lp - 1 : ie - 1) : (ie + 1 == Lp ? 0 : ie + 1);
      e[u] = sample(ie);
      o[u] = sample(io);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) Lf::run(e[u], o[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = kk[u];
      if (lane >= Lf::HL && lane < 64 - Lf::HR && k < L && (w0 + u) < nwin) store(k, e[u]);
    }
  }
}

__device__ __forceinline__ void store_stream2(float2 *p, float2 v) {
  typedef float f2 __attribute__((ext_vector_type(2)));
  __builtin_nontemporal_store(f2{v.x, v.y}, reinterpret_cast<f2 *>(p));
}

// Level j of the tree, block (pulse, child phase p): L = N >> j pairs from
// parent phase p mod 2^(j-1) advanced by p >> (j-1).  Level 1 reads the
// pulse (n valid samples, zero beyond); deeper levels read level j - 1 of
// the workspace (N elements per pulse and level).
template <int F>
__global__ __launch_bounds__(kSwapTreeThreads) void swap_tree_level(
    int j, int N, const float2 *__restrict__ parent_all, long long parent_stride, int n_valid,
    float2 *__restrict__ child_all, long long child_stride) {
  const int P = 1 << j;
  long long pulse;
  int p;
  swap_tree_block(blockIdx.x, gridDim.x, j, pulse, p);
  const int pp = p & ((P >> 1) - 1);  // parent phase (0 at level 1)
  const int b = p >> (j - 1);         // advance of the parent, in its samples
  const int Lp = N >> (j - 1);
  const float2 *par = parent_all + pulse * parent_stride + (long long)pp * Lp;
  float2 *child = child_all + pulse * child_stride + (long long)p * (N >> j);
  tree_phase<F, 2>(
      Lp, b, [&](int i) { return rx_sample(par, n_valid, i); },
      [&](int k, float2 v) { store_stream2(child + k, v); });
}

// Levels j and j + 1 in one pass, block (pulse, level-j phase p): the child
// is lifted from its parent into LDS (and written out), then both of its
// children at level j + 1 (phases p and p + 2^j: the child advanced by 0 and
// by 1 sample) are lifted from LDS.  The parent level is read once per
// child instead of once per level, and one launch serves two levels.
template <int F>
__global__ __launch_bounds__(kSwapTreeThreads) void swap_tree_level2(
    int j, int N, const float2 *__restrict__ parent_all, long long parent_stride, int n_valid,
    float2 *__restrict__ child_all, long long child_stride) {
  extern __shared__ __align__(16) float2 sm_tree[];
  const int P = 1 << j;
  long long pulse;
  int p;
  swap_tree_block(blockIdx.x, gridDim.x, j, pulse, p);
  const int pp = p & ((P >> 1) - 1);
  const int b = p >> (j - 1);
  const int Lp = N >> (j - 1), L = N >> j, L2 = N >> (j + 1);
  const float2 *par = parent_all + pulse * parent_stride + (long long)pp * Lp;
  float2 *child = child_all + pulse * child_stride + (long long)p * L;
  tree_phase<F, 2>(
      Lp, b, [&](int i) { return rx_sample(par, n_valid, i); },
      [&](int k, float2 v) {
        sm_tree[k] = v;
        store_stream2(child + k, v);
      });
  __syncthreads();
  float2 *grand = child_all + pulse * child_stride + (long long)N;  // level j + 1
#pragma unroll
  for (int b2 = 0; b2 < 2; ++b2) {
    float2 *g = grand + (long long)(p + (b2 << j)) * L2;
    tree_phase<F, 2>(
        L, b2, [&](int i) { return sm_tree[i]; }, [&](int k, float2 v) { store_stream2(g + k, v); });
  }
}

// ---------------------------------------------------------------------------
// Correlation of one plane of one pulse.
// ---------------------------------------------------------------------------

// LDS geometry of one work item of plane j: ntp tiles of 32 rows (16 lags
// per row) per phase; extended phase window E = 16 (32 ntp) + K + 15
// elements rounded up to a multiple of 16, sub-sequence length S = E / 16.
// A whole-plane item takes every tile of every phase; a chunk item (long
// pulses) at most kSwapChunkTiles tiles of one phase.
constexpr int kSwapChunkTiles = 16;
// Zero-padded weights: 16 entries before, K + kSwapWPad - 16 after the
// start (the offsets run in groups of four up to K + 17, a column t >= 0
// reads entry v - t + 16 <= K + 33).
constexpr int kSwapWPad = 36;

struct SwapGeom {
  int L, tiles_per_phase, ntp, S, K;
  __host__ __device__ SwapGeom(int N, int j, int K_, int chunk) : K(K_) {
    L = N >> j;
    const int R = (L + 15) / 16;
    tiles_per_phase = (R + 31) / 32;
    ntp = chunk ? (tiles_per_phase < kSwapChunkTiles ? tiles_per_phase : kSwapChunkTiles)
                : tiles_per_phase;
    S = (16 * 32 * ntp + K + 15 + 15) / 16;
  }
  __host__ __device__ int phase_words() const { return 16 * S * 2; }  // re + im planes
  __host__ __device__ int chunks() const { return (tiles_per_phase + ntp - 1) / ntp; }
};

__host__ __device__ inline size_t swap_lds_bytes_geom(int N, int j, int K, int chunk) {
  const SwapGeom g(N, j, K, chunk);
  return ((size_t)(chunk ? 1 : (1 << j)) * g.phase_words() + 2 * (size_t)(K + kSwapWPad)) * 4;
}

// One item: phases p_begin .. p_begin + np_ - 1 of plane j, tiles rt0 ..
// rt0 + ntp - 1 of each (rows 32 rt0 ..), for one pulse.
__device__ __forceinline__ void swap_item(int j, int N, const SwapGeom &g, int p_begin, int np_,
                                          int rt0, int ntp, const float2 *src0, int n,
                                          const SwapDesc &wd, float *outp, float *smem) {
  const int K = g.K, lo = wd.lo[j];
  const int P = 1 << j;
  const int L = g.L, S = g.S;
  float *ys = smem;                                               // np_ phases x 16 S complex
  float2 *wp = reinterpret_cast<float2 *>(ys + np_ * g.phase_words());  // K + kSwapWPad
  const int tid = threadIdx.x, nt = blockDim.x;

  // weights: wp[u + 16] = conj(a[lo + u]) for 0 <= u < K, zero around
  for (int u = tid; u < K + kSwapWPad; u += nt) {
    const int k = u - 16;
    float2 w = make_float2(0.f, 0.f);
    if (k >= 0 && k < K) {
      const float2 a = wd.a[j][k];
      w = make_float2(a.x, -a.y);
    }
    wp[u] = w;
  }
  // phases, extended: element e of phase slot q is Y_p[(512 rt0 + e + lo)
  // mod L]; its re and im go to two planes of 16 S words, each in four
  // groups of four sub-sequences: e = 16 i + 4 k + t lands at word
  // 4 S k + 4 i + t, so the four consecutive offsets one row needs are one
  // aligned 16-byte quad and the 32 rows of a tile read consecutive quads
  const int E = 16 * S, base = 512 * rt0 + lo;
  for (int q = 0; q < np_; ++q) {
    const float2 *src = src0 + (long long)(p_begin + q) * L;
    float *dre = ys + q * g.phase_words();
    float *dim = dre + E;
    for (int e = tid; e < E; e += nt) {
      const int i = pos_mod(base + e, L);
      float2 v;
      if (j == 0)
        v = i < n ? src[i] : make_float2(0.f, 0.f);
      else
        v = src[i];
      const int w = 4 * S * ((e & 15) >> 2) + 4 * (e >> 4) + (e & 3);
      dre[w] = v.x;
      dim[w] = v.y;
    }
  }
  __syncthreads();

  const int lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  const int row = lane & 31, kc = lane >> 5;      // A fragment: row, re/im
  const int col = lane & 31;                      // B fragment column
  const int bt = col >> 1, bc = col & 1;          // lag within the block, re/im
  const int ntiles = np_ * ntp;
  const int Kp = K + 15;                          // offsets v in [0, K + 15)
  for (int t0 = wave * kSwapRT; t0 < ntiles; t0 += nw * kSwapRT) {
    // tile t: phase slot t / ntp, local rows 32 * (t % ntp) ..
    int abase[kSwapRT];
#pragma unroll
    for (int r = 0; r < kSwapRT; ++r) {
      const int t = min(t0 + r, ntiles - 1);
      const int q = t / ntp, rt = t - q * ntp;
      abase[r] = q * g.phase_words() + kc * E + 4 * (rt * 32 + row);
    }
    f32x16 acc[kSwapRT];
#pragma unroll
    for (int r = 0; r < kSwapRT; ++r)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[r][i] = 0.f;
    // offsets in groups of four: one 16-byte A read per tile, four MFMAs;
    // offsets past K + 14 meet zero weights (wp is zero beyond K)
    for (int v0 = 0; v0 < Kp; v0 += 4) {
      const int off = 4 * S * ((v0 & 15) >> 2) + 4 * (v0 >> 4);
      float4 a[kSwapRT];
#pragma unroll
      for (int r = 0; r < kSwapRT; ++r)
        a[r] = *reinterpret_cast<const float4 *>(ys + abase[r] + off);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float2 w = wp[v0 + t - bt + 16];
        // K index 0 multiplies Re(y), 1 multiplies Im(y):
        // Re(out) = Re y Re w - Im y Im w ; Im(out) = Re y Im w + Im y Re w
        const float bv = kc == 0 ? (bc == 0 ? w.x : w.y) : (bc == 0 ? -w.y : w.x);
#pragma unroll
        for (int r = 0; r < kSwapRT; ++r) {
          const float av = t == 0 ? a[r].x : t == 1 ? a[r].y : t == 2 ? a[r].z : a[r].w;
          acc[r] = swap_mfma(av, bv, acc[r]);
        }
      }
    }
    // register i of lane l: row 8 (i / 4) + 4 (l / 32) + i % 4, column l % 32.
    // The lane's address is formed once; register i adds a uniform offset of
    // rows; a tile whose 32 rows are all inside the plane stores unguarded.
    typedef __attribute__((address_space(1))) float gf;
#pragma unroll
    for (int r = 0; r < kSwapRT; ++r) {
      const int t = t0 + r;
      if (t >= ntiles) break;
      const int q = t / ntp, rt = t - q * ntp;
      const int p = p_begin + q;
      const int rr0 = (rt0 + rt) * 32 + 4 * (lane >> 5);
      const int lag0 = 16 * rr0 + bt;
      gf *o0 = (gf *)outp + 2 * ((long long)lag0 * P + p) + bc;
      const long long rs2 = 32LL * P;  // floats per row of 16 lags
      if (16 * ((rt0 + rt) * 32 + 31) + 15 < L) {
#pragma unroll
        for (int i = 0; i < 16; ++i) o0[rs2 * (8 * (i >> 2) + (i & 3))] = acc[r][i];
      } else {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int dr = 8 * (i >> 2) + (i & 3);
          if (lag0 + 16 * dr < L) o0[rs2 * dr] = acc[r][i];
        }
      }
    }
  }
}

// Whole planes: one workgroup per (pulse, plane), heaviest planes (j = 0)
// first in launch order.
__global__ __launch_bounds__(kSwapThreads) void swap_correlate(
    int J, int N, int count, const float2 *__restrict__ rx_all, long long rx_stride, int n,
    const float2 *__restrict__ tree_all, long long tree_stride, SwapDesc wd,
    float2 *__restrict__ out_all, long long out_stride) {
  extern __shared__ __align__(16) float smem_swap[];
  const int j = blockIdx.x / count;
  const long long pulse = blockIdx.x - (long long)j * count;
  const SwapGeom g(N, j, wd.len[j], 0);
  const float2 *src0 = j == 0 ? rx_all + pulse * rx_stride
                              : tree_all + pulse * tree_stride + (long long)(j - 1) * N;
  float *outp = reinterpret_cast<float *>(out_all + pulse * out_stride + (long long)j * N);
  swap_item(j, N, g, 0, 1 << j, 0, g.tiles_per_phase, src0, n, wd, outp, smem_swap);
}

// Long pulses: one workgroup per (plane, pulse, phase, chunk of at most
// kSwapChunkTiles tiles); item0[j] = first item of plane j.
struct SwapChunks {
  int item0[kMaxLevels + 2];
};

__global__ __launch_bounds__(kSwapThreads) void swap_correlate_chunks(
    int J, int N, int count, const float2 *__restrict__ rx_all, long long rx_stride, int n,
    const float2 *__restrict__ tree_all, long long tree_stride, SwapDesc wd, SwapChunks ck,
    float2 *__restrict__ out_all, long long out_stride) {
  extern __shared__ __align__(16) float smem_swap[];
  int j = 0;
  while (j + 1 < J && (long long)blockIdx.x >= ck.item0[j + 1]) ++j;
  const SwapGeom g(N, j, wd.len[j], 1);
  const int per_pulse = (1 << j) * g.chunks();
  const long long local = blockIdx.x - (long long)ck.item0[j];
  const long long pulse = local / per_pulse;
  const int rem = (int)(local - pulse * per_pulse);
  const int p = rem / g.chunks(), c = rem - p * g.chunks();
  const int rt0 = c * g.ntp;
  const int ntp = min(g.ntp, g.tiles_per_phase - rt0);
  const float2 *src0 = j == 0 ? rx_all + pulse * rx_stride
                              : tree_all + pulse * tree_stride + (long long)(j - 1) * N;
  float *outp = reinterpret_cast<float *>(out_all + pulse * out_stride + (long long)j * N);
  swap_item(j, N, g, p, 1, rt0, ntp, src0, n, wd, outp, smem_swap);
}

// ---------------------------------------------------------------------------
// Launch helpers (C++ linkage, used by sidwt_api.cpp).
// ---------------------------------------------------------------------------
size_t swap_lds_bytes(int N, int j, int K, int chunk) { return swap_lds_bytes_geom(N, j, K, chunk); }


// A level's child phase held in LDS for the two-level pass: at most this
// many complex elements (64 KB); longer levels run one level per launch.
constexpr int kSwapTree2MaxL = 8192;

template <int F>
static hipError_t launch_swap_tree_t(int J, int N, const void *rx, long long n, long long count,
                                     long long rx_stride, void *tree, hipStream_t st) {
  float2 *t = static_cast<float2 *>(tree);
  const long long ts = (long long)(J - 1) * N;
  static std::atomic<bool> attr{false};  // set once per process (calls may race: both set it)
  if (!attr) {
    const hipError_t e = hipFuncSetAttribute((const void *)swap_tree_level2<F>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             kSwapTree2MaxL * (int)sizeof(float2));
    if (e != hipSuccess) return e;
    attr = true;
  }
  for (int j = 1; j < J;) {
    const float2 *par = j == 1 ? static_cast<const float2 *>(rx) : t + (long long)(j - 2) * N;
    const long long ps = j == 1 ? rx_stride : ts;
    const int nv = j == 1 ? (int)n : (N >> (j - 1));
    if (j + 1 < J && (N >> j) <= kSwapTree2MaxL) {
      hipLaunchKernelGGL(swap_tree_level2<F>, dim3((unsigned)(count << j)),
                         dim3(kSwapTreeThreads), (size_t)(N >> j) * sizeof(float2), st, j, N,
                         par, ps, nv, t + (long long)(j - 1) * N, ts);
      j += 2;
    } else {
      hipLaunchKernelGGL(swap_tree_level<F>, dim3((unsigned)(count << j)),
                         dim3(kSwapTreeThreads), 0, st, j, N, par, ps, nv,
                         t + (long long)(j - 1) * N, ts);
      j += 1;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_swap(int filter, int J, int N, const void *rx, long long n, long long count,
                       long long rx_stride, void *tree, const SwapDesc &wd, size_t lds_bytes,
                       int chunked, void *out, long long out_stride, hipStream_t st) {
  hipError_t e;
  switch (filter) {
    case F_LEGALL53: e = launch_swap_tree_t<F_LEGALL53>(J, N, rx, n, count, rx_stride, tree, st); break;
    case F_CDF97: e = launch_swap_tree_t<F_CDF97>(J, N, rx, n, count, rx_stride, tree, st); break;
    case F_D4: e = launch_swap_tree_t<F_D4>(J, N, rx, n, count, rx_stride, tree, st); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  static std::atomic<bool> attr_set{false};  // set once per process (calls may race: both set it)
  if (!attr_set) {
    e = hipFuncSetAttribute((const void *)swap_correlate, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void *)swap_correlate_chunks,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  if (!chunked) {
    hipLaunchKernelGGL(swap_correlate, dim3((unsigned)(count * J)), dim3(kSwapThreads), lds_bytes,
                       st, J, N, (int)count, static_cast<const float2 *>(rx), rx_stride, (int)n,
                       static_cast<const float2 *>(tree), (long long)(J - 1) * N, wd,
                       static_cast<float2 *>(out), out_stride);
    return hipGetLastError();
  }
  SwapChunks ck;
  long long items = 0;
  for (int j = 0; j < J; ++j) {
    ck.item0[j] = (int)items;
    const SwapGeom g(N, j, wd.len[j], 1);
    items += count * (long long)(1 << j) * g.chunks();
  }
  ck.item0[J] = (int)items;
  if (items > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(swap_correlate_chunks, dim3((unsigned)items), dim3(kSwapThreads), lds_bytes,
                     st, J, N, (int)count, static_cast<const float2 *>(rx), rx_stride, (int)n,
                     static_cast<const float2 *>(tree), (long long)(J - 1) * N, wd, ck,
                     static_cast<float2 *>(out), out_stride);
  return hipGetLastError();
}

}  // namespace sidwt
