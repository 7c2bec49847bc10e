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

#include "sidwt_bank.hpp"

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

// 16-byte global load of a panel entry (4 words, 16-byte aligned).
template <class V8>
__device__ __forceinline__ V8 gload8(const unsigned *p) {
  const uint4 w = *reinterpret_cast<const uint4 *>(p);
  V8 v;
  __builtin_memcpy(&v, &w, 16);
  return v;
}

constexpr int kBankThreads = 256;  // 4 waves; a wave owns 64 rows x up to 4 column tiles
constexpr int kStageLd = 36;
constexpr int kBankFillRegs = 6;   // data window elements per thread and band held in registers       // staging row stride (floats): 32 columns + pad, 16-byte rows
// The 128 x 2 wave shape streams its panel steps into a per-wave LDS ring of
// kBankRing steps (2 tiles x hi/lo x 64 lanes x 16 bytes each) by direct
// global-to-LDS loads; the ring and the wave's output staging tile share
// one region of kBankWaveBytes.
constexpr int kBankRing = 3;
constexpr int kBankRingStepBytes = 2 * 2 * 64 * 16;
constexpr int kBankStageBytes = 64 * kStageLd * 4;   // one wave's output staging tile
constexpr int kBankStageBytesDeep = 32 * kStageLd * 4;   // the same, 32 rows (deep levels)
constexpr int kBankWaveBytes = kBankRing * kBankRingStepBytes > kBankStageBytes
                                   ? kBankRing * kBankRingStepBytes
                                   : kBankStageBytes;

// s_waitcnt with only the vector-memory count limited (gfx9 encoding:
// vmcnt bits 3:0 and 15:14, expcnt 6:4 and lgkmcnt 11:8 left at their
// maxima).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// The waves of one item.  Wave = (row group wr of 32 RT rows, tile group wt
// of TW column tiles): RT = 2, TW = 4 gives 64 rows x 4 tiles (any row
// block); RT = 4, TW = 2 gives 128 rows x 2 tiles (full 256-row blocks),
// which halves the panel loads per MFMA at the cost of twice the
// data-operand reads (used where the windows are longest); RT = 2, TW = 2
// (64 rows x 2 tiles, half the accumulators) serves the deep levels' kernel,
// which runs more workgroups per CU.
template <bool BF16, int RT, int TW = 8 / RT>
__device__ __forceinline__ void bank_waves(const BankSeg &q, const BankTile *tl,
                                           const BankRefLevel *__restrict__ rl, int Jmax,
                                           const unsigned *__restrict__ wts, const unsigned *dat,
                                           float *stg, int Wmax, int rows, int row0, int tile0,
                                           int ntiles, int wave, int lane, float inv_sd) {
  using H = Half<BF16>;
  using V8 = typename H::V8;
  static_assert((RT == 2 && (TW == 4 || TW == 2)) || (RT == 4 && TW == 2), "wave shape");
  constexpr int RWS = 32 * RT;
  const int l = q.level, P = 1 << l, N = q.N;
  const int rw = RT == 4 ? 2 : rows > 128 ? 4 : rows > 64 ? 2 : 1;
  const int wr = wave % rw, wt = wave / rw;
  const int rows_w = rows - RWS * wr;
  // The wave's tiles: TW consecutive ones, except in the 128 x 2 shape,
  // whose two wave columns take tiles (0, 3) and (1, 2) of the item's four:
  // a level's panels lengthen with the tile index (the bank is sorted by
  // reference length), so each column gets a long and a short one.
  int tix[TW];
  int nt_w = 0;
#pragma unroll
  for (int t = 0; t < TW; ++t) {
    const int k = RT == 4 ? (t == 0 ? wt : 3 - wt) : TW * wt + t;
    tix[t] = tile0 + k;
    if (k < ntiles) nt_w = t + 1;
  }
  if (RT == 4 && wt == 0 && ntiles < 4) nt_w = 1;   // tile 3 missing: column 0 keeps tile 0
  if (rows_w <= 0 || nt_w <= 0) return;          // no barrier follows
  const int nh = min(RT, (rows_w + 31) >> 5);    // 32-row tiles in use
  const int rloc = RWS * wr + (lane & 31);       // row of the first row tile
  const int g = lane >> 5;                        // K half: offsets 4g..4g+3 of a step
  f32x16 acc[RT][TW];
#pragma unroll
  for (int h = 0; h < RT; ++h)
#pragma unroll
    for (int t = 0; t < TW; ++t)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[h][t][i] = 0.f;

  if constexpr (RT == 4) for (int b = 0; b < 2; ++b) {
    const unsigned *dhi = dat + (2 * b) * Wmax;
    const unsigned *dlo = dhi + Wmax;
    int steps[TW];
    const unsigned *pw[TW];
    int S = 0;
#pragma unroll
    for (int t = 0; t < TW; ++t) {
      steps[t] = t < nt_w ? tl[tix[t]].steps[b] : 0;
      pw[t] = wts + (t < nt_w ? tl[tix[t]].off[b] : 0) + 4 * lane;
      S = max(S, steps[t]);
    }
    // The data operands (A) come from LDS one row tile ahead (two sets), so
    // few registers hold them.  Load indices are clamped to valid steps, so
    // no load sits under a branch; only the MFMAs of a tile past its own K
    // length are skipped.
    int last[TW];
#pragma unroll
    for (int t = 0; t < TW; ++t) last[t] = steps[t] > 0 ? steps[t] - 1 : 0;
    auto loadA = [&](int st, int h, V8 &AH, V8 &AL) {
      const int u0 = 8 * min(st, S - 1) + 4 * g;
      AH = load8<V8>(dhi + rloc + 32 * h + u0);
      AL = load8<V8>(dlo + rloc + 32 * h + u0);
    };
    if constexpr (RT == 4) {
      // Panel steps go to the wave's LDS ring kBankRing - 1 steps ahead
      // (direct loads: no registers held); before a step, its own loads
      // must have landed (the vector-memory count then holds only the
      // later steps' loads), and its two tiles' hi and lo are read from the
      // ring once.  A slot is refilled only after the step that read it
      // has its panel values in registers.
      char *ring = reinterpret_cast<char *>(stg);
      auto dma = [&](int st) {
        char *slot = ring + (st % kBankRing) * kBankRingStepBytes;
#pragma unroll
        for (int t = 0; t < TW; ++t) {
          const unsigned *pp = pw[t] + min(st, last[t]) * kBankStepWords;
#pragma unroll
          for (int hl = 0; hl < 2; ++hl)
            __builtin_amdgcn_global_load_lds(
                (const void __attribute__((address_space(1))) *)(pp + 256 * hl),
                (void __attribute__((address_space(3))) *)(slot + (2 * t + hl) * 1024), 16, 0,
                0);
        }
      };
      auto readB = [&](int st, V8(&BH)[TW], V8(&BL)[TW]) {
        const char *slot = ring + (st % kBankRing) * kBankRingStepBytes + 16 * lane;
#pragma unroll
        for (int t = 0; t < TW; ++t) {
          BH[t] = *reinterpret_cast<const V8 *>(slot + (2 * t) * 1024);
          BL[t] = *reinterpret_cast<const V8 *>(slot + (2 * t + 1) * 1024);
        }
      };
      // Order within a step: the next row tile's data operands are read
      // before this row tile's MFMAs (their latency runs under them); after
      // the last row tile the next step's panel slot is awaited and read.
      // The steps where both tiles are live and those where only the longer
      // one is run as two straight loops (the MFMAs of a finished tile are
      // dropped at compile time, so the code has no branches for the
      // waits to be placed around).  The 128 x 2 shape only runs full
      // 256-row blocks, so all four row tiles are always in use.
      constexpr int kOut = (kBankRing - 2) * 2 * TW;  // later steps' loads left in flight
      if (S > 0) {
        V8 bh[TW], bl[TW], ah[2], al[2];
#pragma unroll
        for (int k = 0; k < kBankRing - 1; ++k) dma(k);
        wait_vmcnt<kOut>();
        asm volatile("" ::: "memory");
        readB(0, bh, bl);
        loadA(0, 0, ah[0], al[0]);
        auto phase = [&](auto mask_c, int st0, int st1) {
          constexpr int MASK = decltype(mask_c)::value;
          for (int st = st0; st < st1; ++st) {
            __builtin_amdgcn_sched_barrier(0);
            dma(st + kBankRing - 1);
#pragma unroll
            for (int h = 0; h < RT; ++h) {
              if (h + 1 < RT)
                loadA(st, h + 1, ah[(h + 1) & 1], al[(h + 1) & 1]);
              else
                loadA(st + 1, 0, ah[(h + 1) & 1], al[(h + 1) & 1]);
              __builtin_amdgcn_sched_barrier(0);
#pragma unroll
              for (int t = 0; t < TW; ++t)
                if ((MASK >> t) & 1) {
                  acc[h][t] = H::mma(ah[h & 1], bh[t], acc[h][t]);
                  acc[h][t] = H::mma(ah[h & 1], bl[t], acc[h][t]);
                  acc[h][t] = H::mma(al[h & 1], bh[t], acc[h][t]);
                }
              __builtin_amdgcn_sched_barrier(0);
            }
            wait_vmcnt<kOut>();
            asm volatile("" ::: "memory");
            readB(st + 1, bh, bl);
          }
        };
        static_assert(TW == 2, "two tiles per wave in the 128 x 2 shape");
        const int both = min(steps[0], steps[1]);
        phase(std::integral_constant<int, 3>(), 0, both);
        if (steps[0] > both)
          phase(std::integral_constant<int, 1>(), both, steps[0]);
        else
          phase(std::integral_constant<int, 2>(), both, steps[1]);
        // the tail's clamped loads must land before the ring is refilled
        // (next band) or turned into the staging tile
        wait_vmcnt<0>();
        asm volatile("" ::: "memory");
      }
    }
  }
  if constexpr (RT == 2) {
    // One step sequence over both bands (band 0's steps, then band 1's),
    // so the panel prefetch runs across the band boundary instead of
    // starting cold twice.  Panel operands (B) come from global memory one
    // step ahead in two register sets; the data operands (A) come from LDS
    // one row tile ahead (two sets).  Load indices are clamped to valid
    // steps, so no load sits under a branch; only the MFMAs of a tile past
    // its own K length are skipped.
    int steps[2][TW], last[2][TW], Sb[2];
    long long woff[2][TW];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      Sb[b] = 0;
#pragma unroll
      for (int t = 0; t < TW; ++t) {
        steps[b][t] = t < nt_w ? tl[tix[t]].steps[b] : 0;
        woff[b][t] = t < nt_w ? tl[tix[t]].off[b] : 0;
        last[b][t] = steps[b][t] > 0 ? steps[b][t] - 1 : 0;
        Sb[b] = max(Sb[b], steps[b][t]);
      }
    }
    const int S = Sb[0] + Sb[1];
    const unsigned *wl = wts + 4 * lane;
    auto loadB = [&](int i, V8(&BH)[TW], V8(&BL)[TW]) {
      const bool b1 = i >= Sb[0];
      const int st = b1 ? i - Sb[0] : i;
#pragma unroll
      for (int t = 0; t < TW; ++t) {
        const unsigned *pp = wl + (b1 ? woff[1][t] : woff[0][t]) +
                             min(st, b1 ? last[1][t] : last[0][t]) * kBankStepWords;
        BH[t] = gload8<V8>(pp);
        BL[t] = gload8<V8>(pp + 256);
      }
    };
    auto loadA = [&](int i, int h, V8 &AH, V8 &AL) {
      const int ii = min(i, S - 1);
      const bool b1 = ii >= Sb[0];
      const int u0 = 8 * (b1 ? ii - Sb[0] : ii) + 4 * g;
      const unsigned *dh = dat + (b1 ? 2 * Wmax : 0) + rloc + 32 * h + u0;
      AH = load8<V8>(dh);
      AL = load8<V8>(dh + Wmax);
    };
    if (S > 0) {
      V8 bh[2][TW], bl[2][TW], ah[2], al[2];
      loadB(0, bh[0], bl[0]);
      loadA(0, 0, ah[0], al[0]);
      for (int s0 = 0; s0 < S; s0 += 2) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int i = s0 + k;
          if (i >= S) break;
          loadB(i + 1, bh[k ^ 1], bl[k ^ 1]);
          const bool b1 = i >= Sb[0];
          const int st = b1 ? i - Sb[0] : i;
#pragma unroll
          for (int h = 0; h < RT; ++h) {
            // next row tile's A (the first one of the next step after the last)
            if (h + 1 < RT)
              loadA(i, h + 1, ah[(h + 1) & 1], al[(h + 1) & 1]);
            else
              loadA(i + 1, 0, ah[(h + 1) & 1], al[(h + 1) & 1]);
            __builtin_amdgcn_sched_barrier(0);
            if (h == 0 || h < nh) {
#pragma unroll
              for (int t = 0; t < TW; ++t)
                if (st < (b1 ? steps[1][t] : steps[0][t])) {
                  acc[h][t] = H::mma(ah[h & 1], bh[k][t], acc[h][t]);
                  acc[h][t] = H::mma(ah[h & 1], bl[k][t], acc[h][t]);
                  acc[h][t] = H::mma(al[h & 1], bh[k][t], acc[h][t]);
                }
            }
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      }
    }
  }

  // Output.  Accumulator register i of lane l holds row 8*(i/4) + 4*(l/32)
  // + i%4, column l%32 (column 2 pp + v: pair pp of the tile, v = re/im).
  // Each tile goes through the wave's staging area (64 rows at a time) and
  // leaves as 16-byte runs (2 consecutive phases of one reference at one
  // lag), ordered so a store instruction covers whole runs of
  // out[e][l-1][P p + r]: per reference of the tile Q = min(P, 16) pairs,
  // Q / 2 runs per lag.
  // (an opaque copy of the lane index keeps this index math from being
  // hoisted into the MFMA loop, where it would hold registers)
  int ln = lane;
  asm volatile("" : "+v"(ln));
  float *out = reinterpret_cast<float *>(q.out);
  const int pairs = q.E * P;
  const int lq = min(l, 4);                       // log2 Q
  const int lcpr = lq - 1;                        // log2 runs per lag
  // Rows staged at a time: 64 (two row tiles), or 32 in the deep levels'
  // 64 x 2 shape, whose smaller staging tile lets more workgroups share a CU.
  constexpr int SR = (RT == 2 && TW == 2) ? 32 : 64, LSR = SR == 32 ? 5 : 6;
  constexpr int CH = SR / 32;             // row tiles per staged chunk
  constexpr int NR = SR * 8 / 64;         // store rounds per chunk (8 runs per row)
  // Per-lane run of each of the NR store rounds (the same for every tile and
  // row chunk): staging row and first pair; row < SR and pp <= 14, so the
  // staging reads stay inside the tile.
  int srow[NR], spp[NR];
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    const int kk = 64 * j + ln;
    const int rest = kk >> lcpr;
    srow[j] = rest & (SR - 1);
    spp[j] = ((rest >> LSR) << lq) + 2 * (kk & ((1 << lcpr) - 1));
  }
#pragma unroll
  for (int t = 0; t < TW; ++t) {
    if (t >= nt_w) break;
    const int c0 = kBankTilePairs * tix[t];
    const int c = c0 + ((ln & 31) >> 1);
    const float scale =
        c < pairs ? inv_sd * rl[(c >> l) * (Jmax + 1) + l].inv_scale : 0.f;
#pragma unroll
    for (int hh = 0; hh < RT / CH; ++hh) {
      if (SR * hh >= rows_w) break;
#pragma unroll
      for (int h = 0; h < CH; ++h)
#pragma unroll
        for (int i = 0; i < 16; ++i)
          stg[(32 * h + 8 * (i >> 2) + 4 * (ln >> 5) + (i & 3)) * kStageLd + (ln & 31)] =
              acc[CH * hh + h][t][i] * scale;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // all the staging reads first, then the guarded stores
      f32x4 v[NR];
#pragma unroll
      for (int j = 0; j < NR; ++j)
        v[j] = *reinterpret_cast<const f32x4 *>(stg + srow[j] * kStageLd + 2 * spp[j]);
      const int rbase = row0 + RWS * wr + SR * hh;
      if (l >= 4) {
        // 2^l >= 16: the tile's 16 pairs are phases c0 mod 2^l .. of one
        // reference, so the run addresses differ from a uniform base only
        // by the lane's row and pair
        const int e = c0 >> l, r0 = c0 & (P - 1);
        float *ob = out + 2 * (((long long)e * q.J + (l - 1)) * N + (long long)P * rbase + r0);
#pragma unroll
        for (int j = 0; j < NR; ++j)
          if (SR * hh + srow[j] < rows_w && c0 + spp[j] < pairs)
            __builtin_nontemporal_store(
                v[j], reinterpret_cast<f32x4 *>(ob + 2 * (P * srow[j] + spp[j])));
      } else {
#pragma unroll
        for (int j = 0; j < NR; ++j) {
          const int cc = c0 + spp[j];
          if (SR * hh + srow[j] < rows_w && cc < pairs) {
            const int e = cc >> l, r = cc & (P - 1);
            float *o = out + 2 * (((long long)e * q.J + (l - 1)) * N +
                                  (long long)P * (rbase + srow[j]) + r);
            __builtin_nontemporal_store(v[j], reinterpret_cast<f32x4 *>(o));
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
}

// LDS: data windows [band][hi/lo][Wmax] words (W = 64 rw + umax of the
// item), then one region per wave: kBankWaveBytes (the 128 x 2 shape's
// panel ring, or the [64 rows][kStageLd]-float output staging tile) in the
// general kernel, a [32 rows][kStageLd] staging tile in the deep one.  In
// the 64 x 4 and 64 x 2 shapes the weights are read from their panels
// straight into registers (no LDS, no barrier in the K loop); the waves of
// an item that share tiles read the same panel lines close together in time.
// DEEP: the deep levels' instance (64 x 2 wave tiles, a 32-row staging tile
// alone per wave: no panel ring).
template <bool BF16, bool DEEP>
__device__ __forceinline__ void bank_item(
    const BankSeg *__restrict__ segs, const int2 *__restrict__ items,
    const BankTile *__restrict__ tiles, const int *__restrict__ tile_base,
    const BankRefLevel *__restrict__ rl, int Jmax, const int *__restrict__ lo_lb,
    const unsigned *__restrict__ wts,
    const float2 *__restrict__ scratch, int Wmax, unsigned *sm_bank, float &s_max, int &s_umax) {

  // Item: segment, row block and tile group (uniform across the block).
  const int2 it = items[blockIdx.x];
  const BankSeg sg = segs[it.x];
  const BankSeg &q = sg;                         // the request's fields
  const int l = sg.level, L = sg.L, N = q.N;
  const int k = it.y;
  const int kfull = (sg.nblocks - 1) * sg.g_full;
  int rb, grp;
  if (k < kfull) {
    rb = k / sg.g_full;
    grp = k - rb * sg.g_full;
  } else {
    rb = sg.nblocks - 1;
    grp = k - kfull;
  }
  const int row0 = 256 * rb;
  const int rows = min(256, L - row0);
  const int rw = rows > 128 ? 4 : rows > 64 ? 2 : 1;
  const int per = bank_tiles_per_item(rows);
  const int tile0 = grp * per * sg.gmul;
  const int ntiles = min(per * sg.gmul, sg.ntiles - tile0);
  const BankTile *tl = tiles + tile_base[l];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

  // Longest window of the item's tiles (at most kBankThreads tiles: one per
  // thread, then a wave and a block maximum).
  int um = 0;
  for (int t = tid; t < ntiles; t += nt)
    um = max(um, 8 * max(tl[tile0 + t].steps[0], tl[tile0 + t].steps[1]));
  for (int o = 32; o > 0; o >>= 1) um = max(um, __shfl_xor(um, o, 64));
  if (tid == 0) {
    s_umax = 0;
    s_max = 0.f;
  }
  __syncthreads();
  if (lane == 0) atomicMax(&s_umax, um);
  __syncthreads();
  const int umax = s_umax;
  const int W = 64 * rw + umax;
  unsigned *dat = sm_bank;                      // [b][hilo][Wmax]
  float *stg = reinterpret_cast<float *>(reinterpret_cast<char *>(sm_bank + 4 * Wmax) +
                                        wave * (DEEP ? kBankStageBytesDeep : kBankWaveBytes));
  const float2 *band0 = scratch + q.scratch + scratch_level_off(N, l);
  const int e0[2] = {row0 + lo_lb[2 * l], row0 + lo_lb[2 * l + 1]};

  // Data windows: element i of band b is c_l / d_l at (e0_b + i) mod L,
  // scaled by a power of two sd (largest |x| sd < 2^14) and split into hi
  // and lo.  Windows of up to kBankFillRegs elements per thread and band
  // are read once, every load in flight together, and kept in registers
  // across the block maximum; longer ones are read twice.
  auto split_store = [&](int b, int i, float2 x, float sd) {
    unsigned *hi = dat + (2 * b) * Wmax;
    const float xr = x.x * sd, xi = x.y * sd;
    const unsigned h = pack2<BF16>(xr, xi);
    hi[i] = h;
    hi[Wmax + i] = pack2<BF16>(xr - unpack_lo<BF16>(h), xi - unpack_hi<BF16>(h));
  };
  auto scale_of = [&](float m) {
    int ex = 0;
    (void)frexpf(m, &ex);
    return m > 0.f ? ldexpf(1.f, 14 - ex) : 1.f;
  };
  float mx = 0.f;
  float sd;
  if (W <= kBankFillRegs * kBankThreads) {
    float2 v[2][kBankFillRegs];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int k = 0; k < kBankFillRegs; ++k) {
        const int i = min(tid + k * kBankThreads, W - 1);
        v[b][k] = band0[(b ? L : 0) + pos_mod(e0[b] + i, L)];
      }
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int k = 0; k < kBankFillRegs; ++k)
        mx = fmaxf(mx, fmaxf(fabsf(v[b][k].x), fabsf(v[b][k].y)));
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    if (lane == 0) atomicMax(reinterpret_cast<int *>(&s_max), __float_as_int(mx));
    __syncthreads();
    sd = scale_of(s_max);
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int k = 0; k < kBankFillRegs; ++k) {
        const int i = tid + k * kBankThreads;
        if (i < W) split_store(b, i, v[b][k], sd);
      }
  } else {
    for (int b = 0; b < 2; ++b) {
      const float2 *src = band0 + (b ? L : 0);
      for (int i = tid; i < W; i += nt) {
        const float2 x = src[pos_mod(e0[b] + i, L)];
        mx = fmaxf(mx, fmaxf(fabsf(x.x), fabsf(x.y)));
      }
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
    if (lane == 0) atomicMax(reinterpret_cast<int *>(&s_max), __float_as_int(mx));
    __syncthreads();
    sd = scale_of(s_max);
    for (int b = 0; b < 2; ++b) {
      const float2 *src = band0 + (b ? L : 0);
      for (int i = tid; i < W; i += nt) split_store(b, i, src[pos_mod(e0[b] + i, L)], sd);
    }
  }
  const float inv_sd = 1.f / sd;
  __syncthreads();

  // The item's tile groups, one after another over the same data window
  // (each wave only touches its own staging area: no barrier in between).
  if constexpr (DEEP) {
    // half of a group's tiles per pass: the waves' 64 x 2 tiles cover
    // (4 / rw) x 2 = per / 2 of them
    for (int g0 = 0; g0 < ntiles; g0 += per / 2)
      bank_waves<BF16, 2, 2>(q, tl, rl, Jmax, wts, dat, stg, Wmax, rows, row0, tile0 + g0,
                             min(per / 2, ntiles - g0), wave, lane, inv_sd);
  } else {
    for (int g0 = 0; g0 < ntiles; g0 += per) {
      const int ng = min(per, ntiles - g0);
      if (sg.wide && rows == 256)
        bank_waves<BF16, 4>(q, tl, rl, Jmax, wts, dat, stg, Wmax, rows, row0, tile0 + g0, ng,
                            wave, lane, inv_sd);
      else
        bank_waves<BF16, 2>(q, tl, rl, Jmax, wts, dat, stg, Wmax, rows, row0, tile0 + g0, ng,
                            wave, lane, inv_sd);
    }
  }
}

template <bool BF16>
__global__ __launch_bounds__(kBankThreads, 2) void bank_items(
    const BankSeg *__restrict__ segs, const int2 *__restrict__ items,
    const BankTile *__restrict__ tiles, const int *__restrict__ tile_base,
    const BankRefLevel *__restrict__ rl, int Jmax, const int *__restrict__ lo_lb,
    const unsigned *__restrict__ wts, const float2 *__restrict__ scratch, int Wmax) {
  extern __shared__ __align__(16) unsigned sm_bank[];
  __shared__ float s_max;
  __shared__ int s_umax;
  bank_item<BF16, false>(segs, items, tiles, tile_base, rl, Jmax, lo_lb, wts, scratch, Wmax,
                         sm_bank, s_max, s_umax);
}

// The deep levels' items (short panels, bound by per-item latency and plane
// writes): fewer registers per wave and a 32-row staging tile, so four
// workgroups per CU.
template <bool BF16>
__global__ __launch_bounds__(kBankThreads, 4) void bank_items_deep(
    const BankSeg *__restrict__ segs, const int2 *__restrict__ items,
    const BankTile *__restrict__ tiles, const int *__restrict__ tile_base,
    const BankRefLevel *__restrict__ rl, int Jmax, const int *__restrict__ lo_lb,
    const unsigned *__restrict__ wts, const float2 *__restrict__ scratch, int Wmax) {
  extern __shared__ __align__(16) unsigned sm_bank[];
  __shared__ float s_max;
  __shared__ int s_umax;
  bank_item<BF16, true>(segs, items, tiles, tile_base, rl, Jmax, lo_lb, wts, scratch, Wmax,
                        sm_bank, s_max, s_umax);
}

size_t bank_lds_bytes(int Wmax, bool deep) {
  return (size_t)(4 * Wmax) * 4 + (size_t)4 * (deep ? kBankStageBytesDeep : kBankWaveBytes);
}

hipError_t launch_bank(bool bf16, bool deep, const BankSeg *segs, const int2 *items, int nitems,
                       const BankTile *tiles, const int *tile_base, const BankRefLevel *rl,
                       int Jmax, const int *lo_lb, const unsigned *wts, const float2 *scratch,
                       int Wmax, hipStream_t st) {
  const size_t lds = bank_lds_bytes(Wmax, deep);
  const void *fn = deep ? (bf16 ? (const void *)bank_items_deep<true>
                                : (const void *)bank_items_deep<false>)
                        : (bf16 ? (const void *)bank_items<true> : (const void *)bank_items<false>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (nitems <= 0) return hipSuccess;
  if (deep) {
    if (bf16)
      hipLaunchKernelGGL(bank_items_deep<true>, dim3(nitems), dim3(kBankThreads), lds, st, segs,
                         items, tiles, tile_base, rl, Jmax, lo_lb, wts, scratch, Wmax);
    else
      hipLaunchKernelGGL(bank_items_deep<false>, dim3(nitems), dim3(kBankThreads), lds, st, segs,
                         items, tiles, tile_base, rl, Jmax, lo_lb, wts, scratch, Wmax);
  } else {
    if (bf16)
      hipLaunchKernelGGL(bank_items<true>, dim3(nitems), dim3(kBankThreads), lds, st, segs,
                         items, tiles, tile_base, rl, Jmax, lo_lb, wts, scratch, Wmax);
    else
      hipLaunchKernelGGL(bank_items<false>, dim3(nitems), dim3(kBankThreads), lds, st, segs,
                         items, tiles, tile_base, rl, Jmax, lo_lb, wts, scratch, Wmax);
  }
  return hipGetLastError();
}

}  // namespace sidwt
