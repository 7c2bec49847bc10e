// Device-side building blocks of libsidwt (gfx950).
//
// Lifting factorisations of Sec. III of Bhattacharya & Mahapatra,
// "A Novel Application of Lifting Scheme for Multiresolution Correlation of
// Complex Radar Signals":
//   - LeGall 5/3, x-side P~(z^-1) and dual analysis P^T(z^-1)  (Sec. III-C, Case I)
//   - CDF 9/7 with Table I constants, both sides               (Sec. III-C, Case II)
//   - causal Daubechies-4, eq. (17), same matrix on both sides (Sec. III-B)
//   - reversible integer 5/3 (integer lifting with floor shifts)
// A factor matrix acting on the polyphase pair [e; o] is applied right-most
// first; "z e" is e[k+1], "z^-1 o" is o[k-1].  Pairs are (u[2k], u[2k+1]),
// except for the causal D4 form whose pairs are (u[2k], u[2k-1]).
// Real filters act on I and Q independently (Sec. IV).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sidwt {

enum FilterId : int { F_LEGALL53 = 1, F_CDF97 = 2, F_D4 = 3, F_LEGALL53_INT = 4 };

constexpr int kMaxLevels = 16;
// Threads per workgroup of the fused kernel (8 waves: two workgroups per CU
// give four waves per SIMD to hide LDS latency behind the MFMA pipe).
constexpr int kFusedThreads = 512;
// Per-wave LDS slot (words) for a partial 64x32 FP32 tile handed between
// waves, and the allocation the tile-only batch kernel needs for one slot
// per wave.
constexpr int kBalSlotWords = 2 * 16 * 64;
constexpr int kBalMinLdsBytes = (kFusedThreads / 64) * kBalSlotWords * 4;

// Per level l (1..J) and band b (0 = approximation a~, 1 = detail b~): the
// stored linear support [lo, lo+len) of every phase, and the element offset
// of phase 0 in the plan's coefficient buffer (phases are contiguous, each
// `len` elements long).
struct LevelDesc {
  int lo[2];
  int len[2];
  long long off[2];
};

struct PlanDesc {
  const void *coef;  // float2 (float filters) or int2 (integer filter)
  int filter;
  int J;
  int m;
  int pad_;
  LevelDesc lv[kMaxLevels + 1];  // index 1..J
};

// LDS layout of the fused kernel for one transform length N, computed on the
// host.  All offsets and sizes count 4-byte words.
//
// Level l (1..J) holds its approximation band c_l (b = 0) and detail band
// d_l (b = 1) of length L = N/2^l, each followed by a circular halo copy so
// the correlation's lag windows never wrap: element q < ext = L + halo is
// c[q mod L].  A band is two planes (re, im); a plane is T polyphase
// sub-sequences (element q lives in sub-sequence q mod T at index q / T,
// sub-sequences Ls words apart), so the rows of an MFMA tile, which step
// through the lag axis T elements apart, read consecutive words.  For
// complex64 bands with T >= 4 the sub-sequences are interleaved in groups of
// four: sub-sequences
// 4k..4k+3 share a 4*Ls-word block, index i of sub-sequence 4k + t at word
// 4i + t, so the four consecutive lag offsets one lane needs per MFMA group
// are one aligned 16-byte word quad (and the rows still read consecutive
// quads).
struct FusedLayout {
  int N;
  int J;
  int region_off[kMaxLevels + 1];    // start of level l (band 0, re plane)
  int band_size[kMaxLevels + 1];     // words per band (both planes)
  int plane_stride[kMaxLevels + 1];  // re plane -> im plane
  int Ls[kMaxLevels + 1];            // sub-sequence stride
  int ext[kMaxLevels + 1];           // valid elements per band incl. halo
  int T[kMaxLevels + 1];             // Toeplitz blocking of the lag axis
  int logT[kMaxLevels + 1];
  int lo[kMaxLevels + 1][2];         // lag-window start, aligned down to T
  int F[kMaxLevels + 1][2];          // front zero pad of the staged weights
  int U[kMaxLevels + 1][2];          // lag-window length (GEMM K per re/im)
  int V[kMaxLevels + 1][2];          // staged weight row length (complex)
  int pc[kMaxLevels + 1];            // phases staged per chunk
  int rows[kMaxLevels + 1];          // tile layouts: lag-block rows per tile
  int w_at[kMaxLevels + 1];          // weight staging area of level l (outside
                                     // the level's bands; 16-byte aligned)
  int w_off;                         // end of the band regions
  int total;                         // words of LDS
};

// ---------------------------------------------------------------------------
// Integer planes on int8 matrix cores (v_mfma_i32_32x32x32_i8).
//
// Every integer operand x is written in balanced base-256 digits
// x = sum_a d_a 256^a, d_a in [-128, 127] (kI8DataLimbs digits for the
// pulse's coefficients, WL for the plan's phases), and each real product is
// the sum of the digit products d_a(x) d_w(w) 256^(a+w): the int8 MFMAs
// accumulate one int32 sum per shift class a + w, combined in int64 at the
// end.  Exact while every class sum stays below 2^31 (digit products are at
// most 2^14 in magnitude) and the pulse's coefficients fit the digits.
//
// GEMM of one level l (P = 2^l phases, L = N/P lags per phase), Toeplitz
// blocked by T (T | L): rows are lag blocks p1 (lag p = T p1 + p0, p0 < T),
// columns (p0, phase r, re/im out) in tiles of 16 complex columns
// cc' = P p0 + r (output lag T P p1 + cc'), K the lag offset u (re/im in).
// A lane of the B operand holds 8 offsets x (re, im) of one column: tile
// tau's panel for band b is nch[b] chunks of 16 offsets starting at
// offset u0[b], each chunk WL digit blocks of 64 lanes x 16 bytes (lane
// order: column lane % 32 = 2 cc + (re/im out), offsets 8 (lane / 32) + 0..7
// of the chunk, byte 2k + (re/im in)).  Entry (u, column) is the embedded
// conj(w_r[u - p0 - delta_b]): re-out (w.re, w.im), im-out (-w.im, w.re),
// with delta_b = lo_b - ws_b the shift of the band's window start ws_b
// (lo_b aligned down to 8).
// ---------------------------------------------------------------------------
constexpr int kI8DataLimbs = 3;
constexpr int kI8MaxWeightLimbs = 3;
constexpr int kI8MaxLevels = 7;   // three data digits hold the pulse's level-7 coefficients
constexpr int kI8ChunkBytes = 64 * 16;

struct I8Tile {
  long long off[2];     // byte offset of band b's panel in the plan's panel buffer
  int u0[2];            // first lag offset of band b (a multiple of 8)
  int nch[2];           // chunks of 16 offsets of band b
};

// LDS of the int8 fused kernel (bytes).  c_l of odd levels at 0 (N/2 int2),
// of even levels at c_even (N/4 int2); the digit planes of the current
// level at planes: band b, digit a at planes + (b * kI8DataLimbs + a) *
// plane_bytes, position j (0 <= j < ext[l][b]) holding element
// (ws[l][b] + j) mod L as two bytes (re, im).
struct I8Layout {
  int N, J, WL;
  int T[kMaxLevels + 1];
  int ws[kMaxLevels + 1][2];
  int ext[kMaxLevels + 1][2];
  int ntiles[kMaxLevels + 1];
  int tile_base[kMaxLevels + 1];
  int c_even, planes, plane_bytes, total;
};

// Integer pulses beyond one workgroup's LDS on the int8 path: the pulse is
// lifted into an HBM pyramid (int32 pairs; c_l then d_l at
// scratch_level_off(N, l)), and each level's lag-block rows are cut into
// blocks whose digit windows fit LDS, one workgroup per (pulse, block).
// Block k covers rows [r0, r0 + rows) of its level; its digit planes hold
// positions j < T rows + K[l][b], element (ws[l][b] + T r0 + j) mod L.
constexpr int kI8MaxBlocks = 64;
struct I8Block {
  int level, r0, rows;
};
// Per-pulse pointers of a group of integer pulses of one plan and length
// (integer batches): given to the int8 kernels, pulse i reads rx and writes
// out from here instead of base + i * stride.
struct I8Ptrs {
  const short2 *rx;
  long long *out;
};
struct I8TilePlan {
  int N, J, WL, nblocks, plane_bytes;
  int T[kMaxLevels + 1];
  int ws[kMaxLevels + 1][2];
  int K[kMaxLevels + 1][2];
  int ntiles[kMaxLevels + 1];
  int tile_base[kMaxLevels + 1];
  I8Block blocks[kI8MaxBlocks];
};

// Uneven-batch descriptors (host builds them, the persistent kernel reads them).
struct BatchPulse {
  const void *rx;       // caller's pulse (complex64), n samples
  void *out;            // caller's planes, J x N complex64
  long long n;
  long long scratch;    // complex offset of this pulse's pyramid (long pulses)
  int N, J, plan, layout;
};

struct BatchItem {
  int kind;             // 0: whole pulse (fused), 1: lag tile of a long pulse
  int pulse;
  int level;            // kind 1: level l (plane l-1)
  int row0, rows;       // kind 1: lag-block rows [row0, row0 + rows)
  int pad_[3];
};

// Multi-level lifting of long pulses (uneven batches): a pass lifts levels
// l0..l1 of one pulse, block by block.  A block owns kLiftBlockIn samples of
// the pass's input level l0-1 (c_{l0-1}; the pulse itself for l0 = 1), i.e.
// kLiftBlockIn >> (l1 - l0 + 1) output pairs of level l1 and twice as many
// at each level above; it reads its input stretch once with halos that cover
// the lifting reach of every level of the pass (kLiftHalo samples beyond
// 2k .. 2k+1 per side and level: 2 HL + (odd member before) <= 5 and
// 2 HR <= 5 for every filter): level l0 straight from global memory into
// registers, the deeper levels from two alternating LDS buffers (level l0
// in the first, l0 + 1 in the second, and so on); it writes only its own
// outputs.  An input level of at most kLiftBlockIn samples is one block
// holding the whole (circular) level.
constexpr int kLiftBlockIn = 4096;
constexpr int kLiftHalo = 5;

struct LiftBlock {
  int pulse, l0, l1, blk;
};

__host__ __device__ inline bool lift_block_whole(int N, int l0) {
  return (N >> (l0 - 1)) <= kLiftBlockIn;
}

__host__ __device__ inline int lift_block_count(int N, int l0, int l1) {
  if (lift_block_whole(N, l0)) return 1;
  const int B = kLiftBlockIn >> (l1 - l0 + 1), L1 = N >> l1;
  return (L1 + B - 1) / B;
}

// Ranges of block blk, for l = l0 - 1 .. l1 (arrays indexed by level): the
// pairs [s, e) of level l the block computes (unwrapped; level l0 - 1: the
// input samples it loads) and its own pairs [os, oe) (l >= l0), which it
// writes to the pyramid.
__host__ __device__ inline void lift_block_ranges(int N, int l0, int l1, int blk, int *s, int *e,
                                                  int *os, int *oe) {
  if (lift_block_whole(N, l0)) {
    for (int l = l0 - 1; l <= l1; ++l) {
      s[l] = os[l] = 0;
      e[l] = oe[l] = N >> l;
    }
    return;
  }
  const int B = kLiftBlockIn >> (l1 - l0 + 1);
  for (int l = l0; l <= l1; ++l) {
    const int sh = l1 - l;
    os[l] = (blk * B) << sh;
    const int end = ((blk + 1) * B) << sh, len = N >> l;
    oe[l] = end < len ? end : len;
  }
  s[l1] = os[l1];
  e[l1] = oe[l1];
  for (int l = l1; l >= l0; --l) {
    s[l - 1] = 2 * s[l] - kLiftHalo;
    e[l - 1] = 2 * e[l] + kLiftHalo;
  }
  os[l0 - 1] = s[l0 - 1];
  oe[l0 - 1] = e[l0 - 1];
}

// LDS elements (complex) one block of the pass needs: the stretches of
// levels l0 and l0 + 1 (the two alternating buffers); none for a one-level
// pass, whose level goes to the pyramid only.
__host__ __device__ inline int lift_block_lds(int N, int l0, int l1) {
  if (l1 == l0) return 0;
  int s[kMaxLevels + 1], e[kMaxLevels + 1], os[kMaxLevels + 1], oe[kMaxLevels + 1];
  lift_block_ranges(N, l0, l1, 0, s, e, os, oe);
  return (e[l0] - s[l0]) + (e[l0 + 1] - s[l0 + 1]);
}

// Offset (complex elements) of c_l inside a pulse's scratch pyramid; d_l
// follows c_l.
__host__ __device__ inline long long scratch_level_off(int N, int l) {
  return 2LL * N - 4LL * (N >> l);
}

// ---------------------------------------------------------------------------
// Table I (t = 5/4) and the causal D4 constants of eq. (17).
// ---------------------------------------------------------------------------
struct C97 {
  static constexpr float a = -1.5f;
  static constexpr float b = -0.0625f;
  static constexpr float g = 0.8f;
  static constexpr float d = 0.46875f;
  static constexpr float xi = 1.13137084989847604f;      // 4 sqrt2 / 5
  static constexpr float inv_xi = 0.883883476483184406f; // 5 / (4 sqrt2)
};
struct CD4 {
  static constexpr float s3 = 1.73205080756887729f;          // sqrt3
  static constexpr float u0 = 0.433012701892219323f;         // sqrt3 / 4
  static constexpr float u1 = -0.0669872981077806766f;       // (sqrt3 - 2) / 4
  static constexpr float ka = 1.93185165257813657f;          // (sqrt3 + 1) / sqrt2
  static constexpr float kb = 0.517638090205041524f;         // (sqrt3 - 1) / sqrt2
};

// ---------------------------------------------------------------------------
// Lane neighbours inside a 64-wide wavefront (lane-1 / lane+1).  Lanes at the
// edge get their own value back; the window schedule never uses those.
// ---------------------------------------------------------------------------
// Neighbour lanes through DPP whole-wave shifts (a register-level modifier
// on GFX9-family parts, no LDS round trip): wave_shr:1 gives lane i the
// value of lane i-1, wave_shl:1 that of lane i+1; the edge lane keeps its
// own value (it only ever feeds halo lanes whose results are discarded).
__device__ __forceinline__ int dpp_prev(int v) {
  return __builtin_amdgcn_update_dpp(v, v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ int dpp_next(int v) {
  return __builtin_amdgcn_update_dpp(v, v, 0x130, 0xf, 0xf, false);
}
__device__ __forceinline__ float2 lane_prev(float2 v) {
  return make_float2(__int_as_float(dpp_prev(__float_as_int(v.x))),
                     __int_as_float(dpp_prev(__float_as_int(v.y))));
}
__device__ __forceinline__ float2 lane_next(float2 v) {
  return make_float2(__int_as_float(dpp_next(__float_as_int(v.x))),
                     __int_as_float(dpp_next(__float_as_int(v.y))));
}
__device__ __forceinline__ int2 lane_prev(int2 v) { return make_int2(dpp_prev(v.x), dpp_prev(v.y)); }
__device__ __forceinline__ int2 lane_next(int2 v) { return make_int2(dpp_next(v.x), dpp_next(v.y)); }

__device__ __forceinline__ float2 fma2(float s, float2 a, float2 c) {
  return make_float2(fmaf(s, a.x, c.x), fmaf(s, a.y, c.y));
}
__device__ __forceinline__ float2 add2(float2 a, float2 b) {
  return make_float2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ float2 scale2(float s, float2 a) {
  return make_float2(s * a.x, s * a.y);
}

// ---------------------------------------------------------------------------
// y-side (dual analysis, P^T(z^-1)) lifting of one level, one pair per lane.
// HL/HR: lanes at the window edges whose results are incomplete.
// On return e holds c (approximation), o holds d (detail).
// ---------------------------------------------------------------------------
template <int F> struct YLift;

template <> struct YLift<F_LEGALL53> {
  // Sec. III-C Case I: P^T(z^-1) = diag(1,2) [1 0; -(1+z)/4 1] [1 (1+z^-1)/2; 0 1]
  static constexpr int HL = 1, HR = 1;
  static constexpr bool kOddBefore = false;
  using V = float2;
  __device__ __forceinline__ static void run(float2 &e, float2 &o) {
    e = fma2(0.5f, add2(lane_prev(o), o), e);
    o = fma2(-0.25f, add2(e, lane_next(e)), o);
    o = scale2(2.0f, o);
  }
};

template <> struct YLift<F_CDF97> {
  // Sec. III-C Case II: P^T(z^-1) = diag(1/x, x) [1 0; -d(1+z) 1]
  //   [1 -g(1+z^-1); 0 1] [1 0; -b(1+z) 1] [1 -a(1+z^-1); 0 1]
  static constexpr int HL = 2, HR = 2;
  static constexpr bool kOddBefore = false;
  using V = float2;
  __device__ __forceinline__ static void run(float2 &e, float2 &o) {
    e = fma2(-C97::a, add2(lane_prev(o), o), e);
    o = fma2(-C97::b, add2(e, lane_next(e)), o);
    e = fma2(-C97::g, add2(lane_prev(o), o), e);
    o = fma2(-C97::d, add2(e, lane_next(e)), o);
    e = scale2(C97::inv_xi, e);
    o = scale2(C97::xi, o);
  }
};

template <> struct YLift<F_D4> {
  // Sec. III-B eq. (17): diag(ka, kb) [1 0; 1 z^-1] [1 u0 + u1 z^-1; 0 1] [1 0; -sqrt3 1]
  // on pairs (e, o) = (u[2k], u[2k-1]); the same matrix serves both sides.
  static constexpr int HL = 1, HR = 0;
  static constexpr bool kOddBefore = true;
  using V = float2;
  __device__ __forceinline__ static void run(float2 &e, float2 &o) {
    float2 o1 = fma2(-CD4::s3, e, o);
    float2 o1p = lane_prev(o1);
    float2 e1 = fma2(CD4::u1, o1p, fma2(CD4::u0, o1, e));
    float2 o2 = add2(e1, o1p);
    e = scale2(CD4::ka, e1);
    o = scale2(CD4::kb, o2);
  }
};

template <> struct YLift<F_LEGALL53_INT> {
  // Reversible integer 5/3, dual-analysis (update-first) order:
  //   e += (o[k-1] + o[k] + 1) >> 1 ;  o -= (e[k] + e[k+1] + 2) >> 2
  static constexpr int HL = 1, HR = 1;
  static constexpr bool kOddBefore = false;
  using V = int2;
  __device__ __forceinline__ static void run(int2 &e, int2 &o) {
    int2 op = lane_prev(o);
    e.x += (op.x + o.x + 1) >> 1;
    e.y += (op.y + o.y + 1) >> 1;
    int2 en = lane_next(e);
    o.x -= (e.x + en.x + 2) >> 2;
    o.y -= (e.y + en.y + 2) >> 2;
  }
};

template <int F> struct ElemOf { using T = float2; };
template <> struct ElemOf<F_LEGALL53_INT> { using T = int2; };

// Tap reach of the x-side analysis bands: out[k] depends on u[2k+i] for
// i in [lo, hi].  Used by the host to size the stored phase supports.
struct TapRange { int lo, hi; };

__host__ __device__ inline int floor_div(int a, int b) {
  int q = a / b;
  return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}
__host__ __device__ inline int pos_mod(int a, int b) {
  int r = a % b;
  return r < 0 ? r + b : r;
}

// Word offset of element q inside one plane of a band (see FusedLayout);
// grouped: complex64 bands (quads of sub-sequences when T >= 4).
__host__ __device__ inline int poly_off(int q, int logT, int Ls, bool grouped) {
  const int t = q & ((1 << logT) - 1), i = q >> logT;
  if (grouped && logT >= 2) return (t >> 2) * (4 * Ls) + 4 * i + (t & 3);
  return t * Ls + i;
}

// MFMA operand/accumulator vector types.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

}  // namespace sidwt
