// Integer planes on int8 matrix cores, gfx950.
//
// fused_correlate_i8<WL>: one workgroup per int16 I/Q pulse.  The reversible
// 5/3 y-side lifting (Fig. 7) runs level by level in LDS exactly as in the
// FP64 form of the fused kernel; each new level's two bands are written as
// balanced base-256 digit planes (three int8 digits per component), and the
// level is correlated against the plan's phases (eq. (15), (20)/(20a)) as a
// Toeplitz-blocked GEMM on v_mfma_i32_32x32x32_i8: the A operand is a row
// of 8 lag offsets x (re, im) of one digit plane, the B operand the plan's
// digit panels (I8Tile), and the digit products of each shift class a + w
// accumulate in int32 (exact: at most 3 digit pairs per class, products of
// at most 2^14, K below 2^15 per pass), combined in int64 at the store.
#include <atomic>

#include "sidwt_device.hpp"
#include "sidwt_host.hpp"
#include "sidwt_lift.hpp"

namespace sidwt {

typedef int i32x2 __attribute__((ext_vector_type(2)));
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x16 __attribute__((ext_vector_type(16)));

// Balanced base-256 digits (d in [-128, 127]) of |x| < 2^23, as the two
// bytes (re digit, im digit) of each digit plane.
__device__ __forceinline__ void put_digits(char *planes, int pb, int b, int ws, int ext, int L,
                                          int k, int2 v) {
  int xr = v.x, xi = v.y;
  unsigned short h[kI8DataLimbs];
#pragma unroll
  for (int a = 0; a < kI8DataLimbs; ++a) {
    const int dr = ((xr + 128) & 255) - 128, di = ((xi + 128) & 255) - 128;
    xr = (xr - dr) >> 8;
    xi = (xi - di) >> 8;
    h[a] = (unsigned short)((dr & 255) | ((di & 255) << 8));
  }
  char *base = planes + b * kI8DataLimbs * pb;
  int j0 = k - ws;  // almost always in [0, L): the division only for the rest
  if (j0 < 0 || j0 >= L) j0 = pos_mod(j0, L);
  for (int j = j0; j < ext; j += L) {
#pragma unroll
    for (int a = 0; a < kI8DataLimbs; ++a)
      *reinterpret_cast<unsigned short *>(base + a * pb + 2 * j) = h[a];
  }
}

// 16 bytes of a digit plane at byte offset p: 16-, 8- or 4-byte aligned for
// T = 8, 4, 2 (rows T elements = 2T bytes apart).
template <int T>
__device__ __forceinline__ i32x4 load_a(const char *p) {
  if constexpr (T == 8) {
    return *reinterpret_cast<const i32x4 *>(p);
  } else if constexpr (T == 4) {
    const i32x2 x = *reinterpret_cast<const i32x2 *>(p);
    const i32x2 y = *reinterpret_cast<const i32x2 *>(p + 8);
    return i32x4{x.x, x.y, y.x, y.y};
  } else {
    const int *q = reinterpret_cast<const int *>(p);
    return i32x4{q[0], q[1], q[2], q[3]};
  }
}

// Rows [row0, row0 + R) of plane l-1 of one pulse, from digit planes whose
// position 0 is row row0's first element (pb bytes per plane): units (32
// lag-block rows, one column tile) go to the waves round-robin.  Rows past
// the last (p1 >= R) read row R - 1 and are not stored.
template <int WL, int T>
__device__ void correlate_i8_level(int N, int l, int ctiles, const I8Tile *__restrict__ tiles,
                                   const signed char *__restrict__ panels, const char *planes,
                                   int pb, int row0, int R, long long *__restrict__ outp) {
  constexpr int NC = kI8DataLimbs + WL - 1;   // shift classes a + w
  const int P = 1 << l;
  const int rtiles = (R + 31) >> 5;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nw = blockDim.x >> 6;
  const int g = lane >> 5;
  for (int unit = wave; unit < rtiles * ctiles; unit += nw) {
    const int rt = unit % rtiles, ct = unit / rtiles;
    const int p1 = min(rt * 32 + (lane & 31), R - 1);   // rows past R: read, not stored
    i32x16 acc[NC];
#pragma unroll
    for (int s = 0; s < NC; ++s)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[s][i] = 0;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int u0 = tiles[ct].u0[b], nch = tiles[ct].nch[b];
      const char *pa = planes + b * kI8DataLimbs * pb + 2 * (T * p1 + u0 + 8 * g);
      const signed char *pw = panels + tiles[ct].off[b] + 16 * lane;
      for (int c = 0; c < nch; ++c) {
        i32x4 A[kI8DataLimbs], B[WL];
#pragma unroll
        for (int w = 0; w < WL; ++w)
          B[w] = *reinterpret_cast<const i32x4 *>(pw + (c * WL + w) * kI8ChunkBytes);
#pragma unroll
        for (int a = 0; a < kI8DataLimbs; ++a) A[a] = load_a<T>(pa + a * pb + 32 * c);
#pragma unroll
        for (int a = 0; a < kI8DataLimbs; ++a)
#pragma unroll
          for (int w = 0; w < WL; ++w)
            acc[a + w] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[a], B[w], acc[a + w], 0, 0, 0);
      }
    }
    // register i of lane: row 8 (i / 4) + 4 g + i % 4 of the unit, column
    // lane % 32 = 2 cc + (re/im out); lag T P p1 + 16 ct + cc.  The lane's
    // address is formed once; register i adds a uniform row offset.  Units
    // whose rows and lags are all inside the plane store without guards.
    const int col = lane & 31;
    const int cc = col >> 1, ro = col & 1;
    const long long rs = (long long)T * P;                 // lags per row
    const int pr0 = rt * 32 + 4 * g;
    const long long s0 = rs * (row0 + pr0) + 16 * ct + cc;
    typedef __attribute__((address_space(1))) long long gll;
    gll *o0 = (gll *)outp + 2 * s0 + ro;
    const long long rs2 = 2 * rs;                          // elements per row of lags
    const bool full = rt * 32 + 32 <= R && rs * (row0 + rt * 32 + 31) + 16 * ct + 15 < N;
    // the class sums combine as sum_c acc_c 256^c in int64: for c < 4 one
    // 32 x 32 -> 64-bit multiply-add each (the factors are kept opaque so
    // they are not turned into 64-bit shifts), for c = 4 an add to the high
    // word
    int f[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      f[c] = 1 << (8 * c);
      asm volatile("" : "+s"(f[c]));
    }
    auto value = [&](int i) {
      long long v = acc[0][i];
#pragma unroll
      for (int c = 1; c < NC; ++c) {
        if (c < 4)
          v += (long long)acc[c][i] * (long long)f[c];
        else
          v += (long long)acc[c][i] << 32;
      }
      return v;
    };
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int dr = 8 * (i >> 2) + (i & 3);
      // rows past R and lags of the last row past L - 1 are not stored
      if (full || (pr0 + dr < R && s0 + rs * dr < N))
        __builtin_nontemporal_store(value(i), o0 + rs2 * dr);
    }
  }
}

template <int WL>
__global__ __launch_bounds__(kFusedThreads) void fused_correlate_i8(
    I8Layout lay, const I8Tile *__restrict__ tiles, const signed char *__restrict__ panels,
    const short2 *__restrict__ rx_all, long long n, long long rx_stride,
    long long *__restrict__ out_all, long long out_stride, unsigned plane_mask,
    const I8Ptrs *__restrict__ ptrs) {
  extern __shared__ __align__(16) char sm_i8[];
  const short2 *rx = ptrs ? ptrs[blockIdx.x].rx : rx_all + (long long)blockIdx.x * rx_stride;
  long long *out = ptrs ? ptrs[blockIdx.x].out : out_all + (long long)blockIdx.x * out_stride * 2;
  const int N = lay.N, pb = lay.plane_bytes;
  int2 *c_odd = reinterpret_cast<int2 *>(sm_i8);
  int2 *c_even = reinterpret_cast<int2 *>(sm_i8 + lay.c_even);
  char *planes = sm_i8 + lay.planes;
  for (int l = 1; l <= lay.J; ++l) {
    const int L = N >> l;
    int2 *cdst = (l & 1) ? c_odd : c_even;
    const int ws0 = lay.ws[l][0], ws1 = lay.ws[l][1];
    const int ex0 = lay.ext[l][0], ex1 = lay.ext[l][1];
    const bool keep_c = l < lay.J;
    auto store = [&](int k, int2 c, int2 d) {
      if (keep_c) cdst[k] = c;
      put_digits(planes, pb, 0, ws0, ex0, L, k, c);
      put_digits(planes, pb, 1, ws1, ex1, L, k, d);
    };
    if (l == 1) {
      lift_level<F_LEGALL53_INT, 2>(
          L,
          [&](int kc, int2 &e, int2 &o) {
            e = rx_sample(rx, (int)n, 2 * kc);
            o = rx_sample(rx, (int)n, 2 * kc + 1);
          },
          store);
    } else {
      const int2 *csrc = (l & 1) ? c_even : c_odd;
      lift_level<F_LEGALL53_INT, 1>(
          L,
          [&](int kc, int2 &e, int2 &o) {
            e = csrc[2 * kc];
            o = csrc[2 * kc + 1];
          },
          store);
    }
    __syncthreads();
    if ((plane_mask >> (l - 1)) & 1u) {
      long long *op = out + 2LL * (l - 1) * N;
      const int T = lay.T[l], R = (L + T - 1) / T;
      const I8Tile *tl = tiles + lay.tile_base[l];
      switch (T) {
        case 8: correlate_i8_level<WL, 8>(N, l, lay.ntiles[l], tl, panels, planes, pb, 0, R, op); break;
        case 4: correlate_i8_level<WL, 4>(N, l, lay.ntiles[l], tl, panels, planes, pb, 0, R, op); break;
        default: correlate_i8_level<WL, 2>(N, l, lay.ntiles[l], tl, panels, planes, pb, 0, R, op); break;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Pulses beyond one workgroup's LDS: the y-side lifting of one level into
// the HBM pyramid (one workgroup per pulse and 4096 pairs), then the blocks.
// ---------------------------------------------------------------------------
constexpr int kI8LiftPairs = 4096;

__global__ __launch_bounds__(256) void i8_lift_level(int l, int N, const short2 *__restrict__ rx_all,
                                                     long long n, long long rx_stride,
                                                     int2 *__restrict__ pyr, int chunks,
                                                     const I8Ptrs *__restrict__ ptrs) {
  const long long pulse = blockIdx.x / chunks;
  const int ch = blockIdx.x - (int)(pulse * chunks);
  const int np = N >> l;
  const int k0 = ch * kI8LiftPairs, k1 = min(np, k0 + kI8LiftPairs);
  int2 *base = pyr + pulse * 2LL * N;
  int2 *c = base + scratch_level_off(N, l);
  int2 *d = c + np;
  auto store = [&](int k, int2 cv, int2 dv) {
    c[k] = cv;
    d[k] = dv;
  };
  if (l == 1) {
    const short2 *rx = ptrs ? ptrs[pulse].rx : rx_all + pulse * rx_stride;
    lift_level_range<F_LEGALL53_INT, 2>(
        np, k0, k1,
        [&](int kc, int2 &e, int2 &o) {
          e = rx_sample(rx, (int)n, 2 * kc);
          o = rx_sample(rx, (int)n, 2 * kc + 1);
        },
        store);
  } else {
    const int2 *src = base + scratch_level_off(N, l - 1);
    lift_level_range<F_LEGALL53_INT, 2>(
        np, k0, k1,
        [&](int kc, int2 &e, int2 &o) {
          e = src[2 * kc];
          o = src[2 * kc + 1];
        },
        store);
  }
}

template <int WL>
__global__ __launch_bounds__(kFusedThreads) void i8_blocks(
    I8TilePlan tp, const I8Tile *__restrict__ tiles, const signed char *__restrict__ panels,
    const int2 *__restrict__ pyr, long long *__restrict__ out_all, long long out_stride,
    const I8Ptrs *__restrict__ ptrs) {
  extern __shared__ __align__(16) char sm_i8b[];
  const long long pulse = blockIdx.x / tp.nblocks;
  const I8Block bk = tp.blocks[blockIdx.x - (int)(pulse * tp.nblocks)];
  const int N = tp.N, l = bk.level, L = N >> l, T = tp.T[l], pb = tp.plane_bytes;
  const int2 *c = pyr + pulse * 2LL * N + scratch_level_off(N, l);
  for (int b = 0; b < 2; ++b) {
    const int2 *src = c + (b ? L : 0);
    const int W = T * bk.rows + tp.K[l][b];
    const int q0 = tp.ws[l][b] + T * bk.r0;
    for (int j = threadIdx.x; j < W; j += blockDim.x)
      put_digits(sm_i8b, pb, b, 0, W, 1 << 30, j, src[pos_mod(q0 + j, L)]);
  }
  __syncthreads();
  long long *op = (ptrs ? ptrs[pulse].out : out_all + pulse * out_stride * 2) + 2LL * (l - 1) * N;
  const I8Tile *tl = tiles + tp.tile_base[l];
  switch (T) {
    case 8: correlate_i8_level<WL, 8>(N, l, tp.ntiles[l], tl, panels, sm_i8b, pb, bk.r0, bk.rows, op); break;
    case 4: correlate_i8_level<WL, 4>(N, l, tp.ntiles[l], tl, panels, sm_i8b, pb, bk.r0, bk.rows, op); break;
    default: correlate_i8_level<WL, 2>(N, l, tp.ntiles[l], tl, panels, sm_i8b, pb, bk.r0, bk.rows, op); break;
  }
}

// Lifting of every level into pyr (2N int32 pairs per pulse), then one
// launch over (pulse, block).
hipError_t launch_i8_blocks(const I8TilePlan &tp, const I8Tile *tiles, const signed char *panels,
                            const void *rx, long long n, long long count, long long rx_stride,
                            void *pyr, void *out, long long out_stride, const I8Ptrs *ptrs,
                            hipStream_t st) {
  const int N = tp.N;
  int2 *py = static_cast<int2 *>(pyr);
  for (int l = 1; l <= tp.J; ++l) {
    const int chunks = ((N >> l) + kI8LiftPairs - 1) / kI8LiftPairs;
    if (count * chunks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(i8_lift_level, dim3((unsigned)(count * chunks)), dim3(256), 0, st, l, N,
                       static_cast<const short2 *>(rx), n, rx_stride, py, chunks, ptrs);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (count * tp.nblocks > 0x7fffffff) return hipErrorInvalidValue;
  const size_t lds = (size_t)2 * kI8DataLimbs * tp.plane_bytes;
  const void *fn = tp.WL == 1 ? (const void *)i8_blocks<1>
                 : tp.WL == 2 ? (const void *)i8_blocks<2> : (const void *)i8_blocks<3>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     host::kLdsWords * 4);
  if (e != hipSuccess) return e;
  const dim3 grid((unsigned)(count * tp.nblocks)), block(kFusedThreads);
  long long *o = static_cast<long long *>(out);
  switch (tp.WL) {
    case 1: hipLaunchKernelGGL(i8_blocks<1>, grid, block, lds, st, tp, tiles, panels, py, o, out_stride, ptrs); break;
    case 2: hipLaunchKernelGGL(i8_blocks<2>, grid, block, lds, st, tp, tiles, panels, py, o, out_stride, ptrs); break;
    case 3: hipLaunchKernelGGL(i8_blocks<3>, grid, block, lds, st, tp, tiles, panels, py, o, out_stride, ptrs); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int WL>
static hipError_t launch_i8_t(const I8Layout &lay, const I8Tile *tiles, const signed char *panels,
                              const void *rx, long long n, long long count, long long rx_stride,
                              void *out, long long out_stride, unsigned planes, const I8Ptrs *ptrs,
                              hipStream_t st) {
  static std::atomic<bool> attr{false};  // set once per process (calls may race: both set it)
  if (!attr) {
    const hipError_t e = hipFuncSetAttribute((const void *)fused_correlate_i8<WL>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             host::kLdsWords * 4);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(fused_correlate_i8<WL>, dim3((unsigned)count), dim3(kFusedThreads),
                     (size_t)lay.total, st, lay, tiles, panels,
                     static_cast<const short2 *>(rx), n, rx_stride, static_cast<long long *>(out),
                     out_stride, planes, ptrs);
  return hipGetLastError();
}

hipError_t launch_fused_i8(const I8Layout &lay, const I8Tile *tiles, const signed char *panels,
                           const void *rx, long long n, long long count, long long rx_stride,
                           void *out, long long out_stride, unsigned planes, const I8Ptrs *ptrs,
                           hipStream_t st) {
  switch (lay.WL) {
    case 1: return launch_i8_t<1>(lay, tiles, panels, rx, n, count, rx_stride, out, out_stride, planes, ptrs, st);
    case 2: return launch_i8_t<2>(lay, tiles, panels, rx, n, count, rx_stride, out, out_stride, planes, ptrs, st);
    case 3: return launch_i8_t<3>(lay, tiles, panels, rx, n, count, rx_stride, out, out_stride, planes, ptrs, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sidwt
