// Reference-bank correlation on 16-bit MFMA with a split-precision (hi+lo)
// correction, for gfx950.
//
// For one pulse and one level l the correlation of eq. (20)/(20a) against
// every eligible reference of a bank is a single real GEMM: rows are lags p
// of the level (consecutive), columns are (reference e, phase r, re/im out),
// K is the lag offset u (re/im in).  The data operand (the pulse's c_l, d_l
// as a Hankel matrix) is shared by all references.  Every FP32 operand x is
// split into hi = h(x s) and lo = h(x s - hi) in FP16 or BF16 (h), with a
// power-of-two scale s (weights: per reference and level, chosen when the
// bank is built; data: per work item from its window's largest magnitude),
// and a product is accumulated in FP32 as hi*hi + hi*lo + lo*hi on
// v_mfma_f32_32x32x16_{f16,bf16}; the output is divided by both scales.
#include <type_traits>

#include "sidwt_device.hpp"

namespace sidwt {

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <bool BF16> struct Half;
template <> struct Half<false> {
  using S = _Float16;
  using V8 = f16x8;
  __device__ static f32x16 mma(V8 a, V8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};
template <> struct Half<true> {
  using S = __bf16;
  using V8 = bf16x8;
  __device__ static f32x16 mma(V8 a, V8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

// Two 16-bit values (re, im) packed in one 32-bit word.
template <bool BF16>
__device__ __forceinline__ unsigned pack2(float re, float im) {
  using S = typename Half<BF16>::S;
  S a = (S)re, b = (S)im;
  unsigned short ua, ub;
  __builtin_memcpy(&ua, &a, 2);
  __builtin_memcpy(&ub, &b, 2);
  return (unsigned)ua | ((unsigned)ub << 16);
}

template <bool BF16>
__device__ __forceinline__ float unpack_lo(unsigned w) {
  using S = typename Half<BF16>::S;
  unsigned short u = (unsigned short)(w & 0xffff);
  S v;
  __builtin_memcpy(&v, &u, 2);
  return (float)v;
}
template <bool BF16>
__device__ __forceinline__ float unpack_hi(unsigned w) {
  using S = typename Half<BF16>::S;
  unsigned short u = (unsigned short)(w >> 16);
  S v;
  __builtin_memcpy(&v, &u, 2);
  return (float)v;
}

template <class V8>
__device__ __forceinline__ V8 load8(const unsigned *p) {
  unsigned w[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) w[i] = p[i];
  V8 v;
  __builtin_memcpy(&v, w, 16);
  return v;
}

constexpr int kBankThreads = 256;  // 4 waves; each wave owns 64 rows x 64 columns
constexpr int kBankRows = 256;     // rows per item
constexpr int kBankPairs = 64;     // (reference, phase) pairs per item
constexpr int kBankKChunk = 32;    // lag offsets staged per chunk

// LDS: data windows [band][hi/lo][W] words (W = kBankRows + Umax), then the
// staged weights [pair][array: hi re-col, hi im-col, lo re-col, lo im-col][32].
template <bool BF16>
__global__ __launch_bounds__(kBankThreads) void bank_items(
    const BankReq *__restrict__ reqs, const BankItem *__restrict__ items,
    const BankRefLevel *__restrict__ rl, int Jmax, const int *__restrict__ lo_lb,
    const unsigned *__restrict__ wts, const float2 *__restrict__ scratch, int Wmax) {
  using H = Half<BF16>;
  using V8 = typename H::V8;
  extern __shared__ __align__(16) unsigned sm_bank[];
  __shared__ float s_max;
  const BankItem it = items[blockIdx.x];
  const BankReq &q = reqs[it.req];
  const int l = it.level, P = 1 << l, L = q.N >> l, N = q.N;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int Umax = max(it.U[0], it.U[1]);
  const int W = kBankRows + Umax;
  unsigned *dat = sm_bank;                      // [b][hilo][Wmax]
  unsigned *ws = sm_bank + 4 * Wmax;            // [pair][4][32]
  const float2 *band0 = scratch + q.scratch + scratch_level_off(N, l);

  // Data windows: element i of band b is c_l / d_l at (row0 + lo + i) mod L.
  if (tid == 0) s_max = 0.f;
  __syncthreads();
  float mx = 0.f;
  for (int b = 0; b < 2; ++b) {
    const float2 *src = band0 + (b ? L : 0);
    const int e0 = it.row0 + lo_lb[2 * l + b];
    for (int i = tid; i < W; i += nt) {
      const float2 x = src[pos_mod(e0 + i, L)];
      mx = fmaxf(mx, fmaxf(fabsf(x.x), fabsf(x.y)));
    }
  }
  for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
  if (lane == 0) atomicMax(reinterpret_cast<int *>(&s_max), __float_as_int(mx));
  __syncthreads();
  int ex = 0;
  (void)frexpf(s_max, &ex);
  const float sd = s_max > 0.f ? ldexpf(1.f, 14 - ex) : 1.f;  // largest |x| sd < 2^14
  const float inv_sd = 1.f / sd;
  for (int b = 0; b < 2; ++b) {
    const float2 *src = band0 + (b ? L : 0);
    const int e0 = it.row0 + lo_lb[2 * l + b];
    unsigned *hi = dat + (2 * b) * Wmax;
    unsigned *lo = hi + Wmax;
    for (int i = tid; i < W; i += nt) {
      const float2 x = src[pos_mod(e0 + i, L)];
      const float xr = x.x * sd, xi = x.y * sd;
      const unsigned h = pack2<BF16>(xr, xi);
      hi[i] = h;
      lo[i] = pack2<BF16>(xr - unpack_lo<BF16>(h), xi - unpack_hi<BF16>(h));
    }
  }

  // Wave roles: rows [64 wave, 64 wave + 64) of the item, all 4 column tiles.
  const int rloc = 64 * wave + (lane & 31);      // row of the first row tile
  const int g = lane >> 5;                        // K half: offsets 4g..4g+3
  const int col = lane & 31;
  const int co = col & 1;
  const bool active = 64 * wave < it.rows;
  f32x16 acc[2][4];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[h][t][i] = 0.f;

  for (int b = 0; b < 2; ++b) {
    const unsigned *dhi = dat + (2 * b) * Wmax;
    const unsigned *dlo = dhi + Wmax;
    for (int k0 = 0; k0 < it.U[b]; k0 += kBankKChunk) {
      __syncthreads();
      // stage weights of the item's pairs for offsets [k0, k0 + 32)
      for (int x = tid; x < kBankPairs * 4 * kBankKChunk; x += nt) {
        const int u = x & (kBankKChunk - 1);
        const int a = (x >> 5) & 3;
        const int pl = x >> 7;
        unsigned w = 0;
        if (pl < it.npairs) {
          const int c = it.pair0 + pl;
          const int e = c >> l, r = c & (P - 1);
          const BankRefLevel &R = rl[e * (Jmax + 1) + l];
          const int Ue = R.U[b];
          if (k0 + u < Ue) w = wts[R.off[b] + ((long long)r * 4 + a) * Ue + k0 + u];
        }
        ws[x] = w;
      }
      __syncthreads();
      if (active) {
        const int steps = min(4, (it.U[b] - k0 + 7) >> 3);
        for (int st = 0; st < steps; ++st) {
          const int u0 = k0 + 8 * st + 4 * g;
          V8 ahi[2], alo[2];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            ahi[h] = load8<V8>(dhi + rloc + 32 * h + u0);
            alo[h] = load8<V8>(dlo + rloc + 32 * h + u0);
          }
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int pl = t * 16 + (col >> 1);
            const unsigned *wb = ws + (pl * 4) * kBankKChunk + 8 * st + 4 * g;
            const V8 bhi = load8<V8>(wb + co * kBankKChunk);
            const V8 blo = load8<V8>(wb + (2 + co) * kBankKChunk);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              acc[h][t] = H::mma(ahi[h], bhi, acc[h][t]);
              acc[h][t] = H::mma(ahi[h], blo, acc[h][t]);
              acc[h][t] = H::mma(alo[h], bhi, acc[h][t]);
            }
          }
        }
      }
    }
  }

  // register i of lane l: row 8*(i/4) + 4*(l/32) + i%4, column l%32
  if (!active) return;
  float *out = reinterpret_cast<float *>(q.out);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int pl = t * 16 + (col >> 1);
    if (pl >= it.npairs) continue;
    const int c = it.pair0 + pl;
    const int e = c >> l, r = c & (P - 1);
    const float scale = inv_sd * rl[e * (Jmax + 1) + l].inv_scale;
    float *o = out + 2 * (((long long)e * q.J + (l - 1)) * N) + 2LL * r + co;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int lr = 64 * wave + 32 * h + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
        if (lr < it.rows) {
          const long long s = (long long)P * (it.row0 + lr);
          __builtin_nontemporal_store(acc[h][t][i] * scale, o + 2 * s);
        }
      }
    }
  }
}

hipError_t launch_bank(bool bf16, const BankReq *reqs, const BankItem *items, int nitems,
                       const BankRefLevel *rl, int Jmax, const int *lo_lb, const unsigned *wts,
                       const float2 *scratch, int Wmax, hipStream_t st) {
  const size_t lds = (size_t)(4 * Wmax + kBankPairs * 4 * kBankKChunk) * 4;
  const void *fn = bf16 ? (const void *)bank_items<true> : (const void *)bank_items<false>;
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (nitems <= 0) return hipSuccess;
  if (bf16)
    hipLaunchKernelGGL(bank_items<true>, dim3(nitems), dim3(kBankThreads), lds, st, reqs, items, rl,
                       Jmax, lo_lb, wts, scratch, Wmax);
  else
    hipLaunchKernelGGL(bank_items<false>, dim3(nitems), dim3(kBankThreads), lds, st, reqs, items, rl,
                       Jmax, lo_lb, wts, scratch, Wmax);
  return hipGetLastError();
}

}  // namespace sidwt
