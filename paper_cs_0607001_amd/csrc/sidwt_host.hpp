// Host-side planning of libsidwt: stored phase supports of a plan and the
// LDS layout of the fused kernel, plus a bounds audit of that layout.
// Pure host C++ (no device calls), shared by the C ABI implementation and
// the CPU-side layout checker.
#pragma once
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <vector>

#include "sidwt_device.hpp"

namespace sidwt {
namespace host {

constexpr int64_t kMaxRef = 8192;              // longest reference (tree kernel LDS)
constexpr int64_t kMaxN = int64_t(1) << 30;     // longest circular length
// LDS per workgroup on gfx950 is 160 KB; 256 bytes stay free for the
// kernels' static shared variables.
constexpr int kLdsWords = (160 * 1024 - 256) / 4;
constexpr int kLdsWordsTwoPerCu = 80 * 1024 / 4; // two workgroups per CU

inline bool is_int_filter(int f) { return f == F_LEGALL53_INT; }

// x-side analysis reach: band b at output k depends on u[2k+i], i in [lo, hi]
// (5/3: h~ spans -2..2, g~ spans 0..2; 9/7: -4..4 and -2..4; causal D4:
// -3..0).  The integer 5/3 has the reach of the float 5/3.
inline TapRange tap_range(int filter, int band) {
  switch (filter) {
    case F_LEGALL53:
    case F_LEGALL53_INT:
      return band == 0 ? TapRange{-2, 2} : TapRange{0, 2};
    case F_CDF97:
      return band == 0 ? TapRange{-4, 4} : TapRange{-2, 4};
    default:
      return TapRange{-3, 0};
  }
}

inline int ceil_div_i(int a, int b) { return -floor_div(-a, b); }

inline int64_t transform_length(int64_t n, int J) {
  int64_t q = int64_t(1) << J;
  return q * ((n + q - 1) / q);
}

// Stored linear supports of the phase pyramid, level by level.  The input
// support of level l includes the one-sample delay of the odd branch
// (shift-circulant tree).  Returns the number of complex elements.
inline long long plan_windows(int filter, int J, int m, PlanDesc *d) {
  long long off = 0;
  int in_lo = 0, in_len = m;
  for (int l = 1; l <= J; ++l) {
    for (int b = 0; b < 2; ++b) {
      TapRange tr = tap_range(filter, b);
      int k_first = ceil_div_i(in_lo - tr.hi, 2);
      int k_last = floor_div(in_lo + in_len - tr.lo, 2);
      d->lv[l].lo[b] = k_first;
      d->lv[l].len[b] = k_last - k_first + 1;
      d->lv[l].off[b] = off;
      off += (long long)d->lv[l].len[b] << l;
    }
    in_lo = d->lv[l].lo[0];
    in_len = d->lv[l].len[0];
  }
  return off;
}

// Integer plans accumulate integer products in FP64, which is exact while
// every partial sum stays below 2^53 in magnitude.  Per level, with the
// level l-1 approximations bounded by X:
//   pulse (y-side, update first): c = e + ((o[k-1] + o[k] + 1) >> 1) is the
//     lowpass (1/2, 1, 1/2) of l1 norm 2, so |c| <= 2X (the floor keeps the
//     rounded half-sum within X); d = o - ((c[k] + c[k+1] + 2) >> 2) gives
//     |d| <= X + X = 2X.  Both bands stay within 2X + 1, and the pulse
//     bound doubles every level (a full-scale DC pulse reaches it).
//   reference (x-side, predict first): d = o - ((e[k] + e[k+1]) >> 1),
//     highpass (-1/2, 1, -1/2) of l1 norm 2, |d| <= 2X + 1;
//     c = e + ((d[k-1] + d[k] + 2) >> 2) is the lowpass
//     (-1/8, 1/4, 3/4, 1/4, -1/8) of l1 norm 3/2 plus at most one unit of
//     rounding, |c| <= 1.5X + 2.
// An output of level l sums, over both bands' stored supports, complex
// products of such values (two real products per component), so each
// partial sum is bounded by
//   (2 Xp + 1)(2 Xr + 1) * 2 (len_0 + len_1),
// Xp, Xr the level l-1 approximation bounds of the pulse (any int16: 32768
// at level 0) and of the reference (its own peak component).
// int_level_bounds writes Xp, Xr of levels 0..J (arrays of J + 1).
inline void int_level_bounds(const PlanDesc &d, int ref_peak, double *xp, double *xr) {
  xp[0] = 32768.0;
  xr[0] = ref_peak;
  for (int l = 1; l <= d.J; ++l) {
    xp[l] = 2.0 * xp[l - 1] + 1.0;
    xr[l] = 1.5 * xr[l - 1] + 2.0;
  }
}

inline double int_level_sum_bound(const PlanDesc &d, int l, const double *xp, const double *xr) {
  const double terms = 2.0 * ((double)d.lv[l].len[0] + d.lv[l].len[1]);
  return (2.0 * xp[l - 1] + 1.0) * (2.0 * xr[l - 1] + 1.0) * terms;
}

inline bool int_sums_exact(const PlanDesc &d, int ref_peak) {
  double xp[kMaxLevels + 1], xr[kMaxLevels + 1];
  int_level_bounds(d, ref_peak, xp, xr);
  for (int l = 1; l <= d.J; ++l)
    if (int_level_sum_bound(d, l, xp, xr) >= 9007199254740992.0) return false;
  return true;
}

// ---------------------------------------------------------------------------
// Integer planes on int8 matrix cores: digit ranges, the plan's panels and
// the fused kernel's LDS layout (see I8Tile / I8Layout).
// ---------------------------------------------------------------------------

// Largest value n balanced base-256 digits hold: 127 (1 + 256 + ... ); the
// most negative one is -128 (1 + 256 + ...).
inline long long i8_max_pos(int n) {
  long long s = 0, p = 1;
  for (int i = 0; i < n; ++i, p *= 256) s += 127 * p;
  return s;
}

// Digits for the plan's phases: the fewest (at least 1) whose range holds
// every stored value and its negation (|v| <= maxabs); 0 if more than
// kI8MaxWeightLimbs would be needed.
inline int i8_weight_limbs(long long maxabs) {
  for (int n = 1; n <= kI8MaxWeightLimbs; ++n)
    if (i8_max_pos(n) >= maxabs) return n;
  return 0;
}

// The pulse's coefficients fit kI8DataLimbs digits at every level: the
// level-l bound 2 Xp_{l-1} + 1 (int_level_bounds, any int16 pulse).
inline bool i8_data_fits(const PlanDesc &d) {
  if (d.J > kI8MaxLevels) return false;
  double xp[kMaxLevels + 1], xr[kMaxLevels + 1];
  int_level_bounds(d, 0, xp, xr);
  for (int l = 1; l <= d.J; ++l)
    if (2.0 * xp[l - 1] + 1.0 > (double)i8_max_pos(kI8DataLimbs)) return false;
  return true;
}

// Window start of band b at level l: the stored support's first index
// aligned down to 8 (rows of the A operand then start on 16-byte
// boundaries), and delta = lo - ws.
inline int i8_window_start(const PlanDesc &d, int l, int b) {
  const int lo = d.lv[l].lo[b];
  return lo - pos_mod(lo, 8);
}

// The plan's B-operand panels (see I8Tile) for the widest blocking T = 8:
// T P / 16 = P / 2 tiles per level; a call with a smaller T uses the first
// T P / 16 of them (the columns cc' = P p0 + r of a tile do not depend on
// T).  coef: the plan's pyramid on the host as int32 (re, im) pairs, at the
// PlanDesc offsets.  The digits d(v, a) of every entry fill the panels.
inline void build_i8_panels(const PlanDesc &d, const int32_t *coef, int WL,
                            std::vector<I8Tile> *tiles, std::vector<int> *tile_base,
                            std::vector<signed char> *panels) {
  tiles->clear();
  panels->clear();
  tile_base->assign(kMaxLevels + 1, 0);
  for (int l = 1; l <= d.J; ++l) {
    const int P = 1 << l;
    const int nt = std::max(1, P / 2);
    (*tile_base)[l] = (int)tiles->size();
    for (int tau = 0; tau < nt; ++tau) {
      I8Tile t{};
      const int p0a = (16 * tau) >> l, p0b = (16 * tau + 15) >> l;
      for (int b = 0; b < 2; ++b) {
        const int len = d.lv[l].len[b];
        const int delta = d.lv[l].lo[b] - i8_window_start(d, l, b);
        const int u0 = (p0a + delta) & ~7;
        const int nch = (p0b + delta + len - u0 + 15) / 16;
        t.u0[b] = u0;
        t.nch[b] = nch;
        t.off[b] = (long long)panels->size();
        panels->resize(panels->size() + (size_t)nch * WL * kI8ChunkBytes, 0);
        signed char *pan = panels->data() + t.off[b];
        for (int c = 0; c < nch; ++c)
          for (int lane = 0; lane < 64; ++lane) {
            const int col = lane & 31, cc = col >> 1, ro = col & 1, g = lane >> 5;
            const int ccp = 16 * tau + cc, p0 = ccp >> l, r = ccp & (P - 1);
            for (int k = 0; k < 8; ++k) {
              const int i = u0 + 16 * c + 8 * g + k - p0 - delta;
              long long wr = 0, wi = 0;
              if (i >= 0 && i < len) {
                const int32_t *w = coef + 2 * (d.lv[l].off[b] + (long long)r * len + i);
                wr = w[0];
                wi = w[1];
              }
              for (int ci = 0; ci < 2; ++ci) {
                const long long v = ro == 0 ? (ci == 0 ? wr : wi) : (ci == 0 ? -wi : wr);
                long long x = v;
                for (int a = 0; a < WL; ++a) {
                  const long long dg = ((x + 128) & 255) - 128;
                  x = (x - dg) >> 8;
                  pan[((size_t)c * WL + a) * kI8ChunkBytes + 16 * lane + 2 * k + ci] =
                      (signed char)dg;
                }
              }
            }
          }
      }
      tiles->push_back(t);
    }
  }
}

// Toeplitz block of level l for the int8 path: 8, halved (down to 2) while
// the level has fewer than 32 lag-block rows and a tile stays full
// (T P >= 16).  The level has ceil(L / T) rows; lags of the last row past
// L - 1 are computed (their data wraps) but not stored.
inline int i8_level_T(int N, int l) {
  const int P = 1 << l, L = N >> l;
  int T = 8;
  while (T > 2 && T * P > 16 && L / T < 32) T >>= 1;
  return T;
}

// LDS layout of the int8 fused kernel for one transform length (see
// I8Layout); tiles / tile_base as build_i8_panels returns them.  0, or -5
// when the path does not apply (levels, blocking, LDS).
inline int make_i8_layout(const PlanDesc &d, int WL, const I8Tile *tiles, const int *tile_base,
                          int64_t N64, I8Layout *lay) {
  std::memset(lay, 0, sizeof(*lay));
  if (WL < 1 || WL > kI8MaxWeightLimbs || !i8_data_fits(d) || N64 > kLdsWords) return -5;
  const int N = (int)N64, J = d.J;
  lay->N = N;
  lay->J = J;
  lay->WL = WL;
  int pb = 0;
  for (int l = 1; l <= J; ++l) {
    const int T = i8_level_T(N, l);
    const int P = 1 << l, L = N >> l, R = (L + T - 1) / T;
    lay->T[l] = T;
    lay->ntiles[l] = T * P / 16;
    lay->tile_base[l] = tile_base[l];
    for (int b = 0; b < 2; ++b) {
      int kmax = 0;
      for (int tau = 0; tau < lay->ntiles[l]; ++tau) {
        const I8Tile &t = tiles[tile_base[l] + tau];
        kmax = std::max(kmax, t.u0[b] + 16 * t.nch[b]);
      }
      // rows p1 < R read positions T p1 + u0 + (0 .. 16 nch - 1)
      const int ext = (T * R + kmax + 7) & ~7;
      lay->ws[l][b] = i8_window_start(d, l, b);
      lay->ext[l][b] = ext;
      pb = std::max(pb, 2 * ext);
    }
  }
  lay->plane_bytes = (pb + 15) & ~15;
  lay->c_even = 4 * N;                        // after N/2 int2 of the odd levels
  lay->planes = (6 * N + 15) & ~15;           // after N/4 int2 of the even levels
  const long long total = (long long)lay->planes + 2LL * kI8DataLimbs * lay->plane_bytes;
  if (total > (long long)kLdsWords * 4) return -5;
  lay->total = (int)total;
  return 0;
}

// Block plan of an integer pulse too long for the fused int8 kernel (see
// I8TilePlan): per level the fused kernel's blocking T and window geometry,
// rows cut into blocks of a multiple of 32 rows whose digit windows stay
// within kI8TilePositions positions per plane.  0, or -5 when the path does
// not apply.
constexpr int kI8TilePositions = 8192;   // 6 planes x 16 KB of LDS
inline int make_i8_tile_plan(const PlanDesc &d, int WL, const I8Tile *tiles, const int *tile_base,
                             int64_t N64, I8TilePlan *tp) {
  std::memset(tp, 0, sizeof(*tp));
  if (WL < 1 || WL > kI8MaxWeightLimbs || !i8_data_fits(d) || N64 > kMaxN) return -5;
  const int N = (int)N64, J = d.J;
  tp->N = N;
  tp->J = J;
  tp->WL = WL;
  int pos = 0;
  for (int l = 1; l <= J; ++l) {
    const int T = i8_level_T(N, l);
    const int P = 1 << l, L = N >> l, R = (L + T - 1) / T;
    tp->T[l] = T;
    tp->ntiles[l] = T * P / 16;
    tp->tile_base[l] = tile_base[l];
    int kmax = 0;
    for (int b = 0; b < 2; ++b) {
      int k = 0;
      for (int tau = 0; tau < tp->ntiles[l]; ++tau) {
        const I8Tile &t = tiles[tile_base[l] + tau];
        k = std::max(k, t.u0[b] + 16 * t.nch[b]);
      }
      tp->ws[l][b] = i8_window_start(d, l, b);
      tp->K[l][b] = k;
      kmax = std::max(kmax, k);
    }
    int rb = ((kI8TilePositions - kmax) / T) & ~31;
    if (rb < 32) return -5;
    rb = std::min(rb, (R + 31) & ~31);
    for (int r0 = 0; r0 < R; r0 += rb) {
      if (tp->nblocks >= kI8MaxBlocks) return -5;
      tp->blocks[tp->nblocks++] = I8Block{l, r0, std::min(rb, R - r0)};
      pos = std::max(pos, T * std::min(rb, R - r0) + kmax);
    }
  }
  tp->plane_bytes = (2 * pos + 15) & ~15;
  return 0;
}

// Integer plans hold linear-support phases; they equal the circular
// integer lifting at length N only if no level's input support (plus the
// one-sample delay and the +-2 reach of the 5/3 steps) wraps around.
inline bool int_support_fits(const PlanDesc &d, int64_t N) {
  int64_t in_len = d.m;
  for (int l = 1; l <= d.J; ++l) {
    if (in_len + 5 > (N >> (l - 1))) return false;
    in_len = d.lv[l].len[0];
  }
  return true;
}

// Output columns per MFMA tile, in complex values: 16 for the FP32 32x32x2
// tiles, 8 for the FP64 16x16x4 tiles of the integer path.
inline int tile_cols(bool is_int) { return is_int ? 8 : 16; }

// LDS layout of the fused kernel (see FusedLayout); sizes in 4-byte words.
// Returns 0, or -5 (unsupported) when the pulse does not fit one workgroup.
inline int make_layout(const PlanDesc &d, int64_t N64, FusedLayout *lay) {
  std::memset(lay, 0, sizeof(*lay));
  if (N64 > kLdsWords) return -5;
  const bool is_int = is_int_filter(d.filter);
  const int N = (int)N64, J = d.J;
  const int ncol = tile_cols(is_int);
  lay->N = N;
  lay->J = J;
  for (int l = 1; l <= J; ++l) {
    const int P = 1 << l, L = N >> l;
    int T = P < ncol ? ncol / P : 1;
    while (L % T) T >>= 1;  // lag blocks must tile L exactly
    int logT = 0;
    while ((1 << logT) < T) ++logT;
    lay->T[l] = T;
    lay->logT[l] = logT;
    int halo = 0;
    for (int b = 0; b < 2; ++b) {
      const int lo = d.lv[l].lo[b], len = d.lv[l].len[b];
      const int delta = pos_mod(lo, T);  // window start aligned down to T
      lay->lo[l][b] = lo - delta;
      lay->F[l][b] = T - 1 + delta;
      int U = len + delta + T - 1;
      U = is_int ? (U + 1) & ~1 : (U + 3) & ~3;  // FP32: groups of 4 offsets
      lay->U[l][b] = U;
      // staged row >= U + T - 1 complex, an odd multiple of T (the phases of
      // one tile then fall on disjoint LDS banks)
      int k = (U + T - 1 + T - 1) / T;
      if ((k & 1) == 0) ++k;
      lay->V[l][b] = k * T;
      // rows start at multiples of T below L and read U offsets
      halo = std::max(halo, U - T + 1);
    }
    lay->ext[l] = L + halo;
    const int lsub = (lay->ext[l] + T - 1) / T;
    // integer tiles read two neighbouring sub-sequences at once: Ls = 16 mod
    // 64 puts them on different LDS banks
    lay->Ls[l] = is_int ? lsub + ((16 - lsub % 64) + 64) % 64 : lsub;
    lay->plane_stride[l] = ((T * lay->Ls[l] + 63) / 64) * 64 + 32;  // = 32 mod 64
    lay->band_size[l] = 2 * lay->plane_stride[l];
  }
  // Level l is lifted from c_{l-1} while it is written, so its region must
  // miss that band: at offset 0 when it fits below, else right after it.
  int total = 0;
  for (int l = 1; l <= J; ++l) {
    if (l == 1) {
      lay->region_off[l] = 0;
    } else {
      const int cstart = lay->region_off[l - 1];
      lay->region_off[l] = (2 * lay->band_size[l] <= cstart) ? 0 : cstart + lay->band_size[l - 1];
    }
    total = std::max(total, lay->region_off[l] + 2 * lay->band_size[l]);
  }
  total = (total + 3) & ~3;
  lay->w_off = total;
  // Weight staging (complex = 2 words): all phases when P < ncol (one tile's
  // columns span them), otherwise chunks of k*ncol phases within budget.
  int budget = std::max(0, kLdsWordsTwoPerCu - total);
  int need_min = 0;
  for (int l = 1; l <= J; ++l) {
    const int P = 1 << l;
    const int row = 2 * (lay->V[l][0] + lay->V[l][1]);
    need_min = std::max(need_min, (P < ncol ? P : ncol) * row);
  }
  if (need_min > budget) budget = kLdsWords - total;
  if (need_min > budget) return -5;
  // While plane l-1 is correlated only level l's bands are live, so its
  // staged weights may reuse any other part of the band area; only what
  // does not fit there goes after it.
  int end = total;
  for (int l = 1; l <= J; ++l) {
    const int P = 1 << l;
    const int row = 2 * (lay->V[l][0] + lay->V[l][1]);
    int pc = P;
    if (P >= ncol) pc = std::max(ncol, std::min(P, (budget / row) / ncol * ncol));
    lay->pc[l] = pc;
    const int need = pc * row;
    const int r0 = lay->region_off[l], r1 = r0 + 2 * lay->band_size[l];
    const int after = (r1 + 3) & ~3;
    if (need <= r0) {
      lay->w_at[l] = 0;
    } else if (after + need <= total) {
      lay->w_at[l] = after;
    } else {
      lay->w_at[l] = total;
      end = std::max(end, total + need);
    }
  }
  lay->total = end;
  return lay->total <= kLdsWords ? 0 : -5;
}

// Per-level geometry shared by the fused and tile layouts: Toeplitz block T
// (T | L), aligned lag windows, staged row lengths.
inline void level_geometry(const PlanDesc &d, int N, int l, bool is_int, FusedLayout *lay) {
  const int ncol = tile_cols(is_int);
  const int P = 1 << l, L = N >> l;
  int T = P < ncol ? ncol / P : 1;
  while (L % T) T >>= 1;
  int logT = 0;
  while ((1 << logT) < T) ++logT;
  lay->T[l] = T;
  lay->logT[l] = logT;
  for (int b = 0; b < 2; ++b) {
    const int lo = d.lv[l].lo[b], len = d.lv[l].len[b];
    const int delta = pos_mod(lo, T);
    lay->lo[l][b] = lo - delta;
    lay->F[l][b] = T - 1 + delta;
    int U = len + delta + T - 1;
    U = is_int ? (U + 1) & ~1 : (U + 3) & ~3;
    lay->U[l][b] = U;
    int k = (U + T - 1 + T - 1) / T;
    if ((k & 1) == 0) ++k;
    lay->V[l][b] = k * T;
  }
}

// Tile layout of a long pulse (float filters).  A tile of level l covers
// rows[l] lag-block rows (a multiple of 64), chosen so that its band window
// rows*T + U stays near `window` elements (at least 64 rows); LDS holds the
// window of both bands as polyphase re/im planes (band 0 at word 0, band 1
// at 2*plane_stride) and the staged weights at w_at.  Returns 0 or -5.
inline int make_tile_layout(const PlanDesc &d, int64_t N64, int window, FusedLayout *lay) {
  std::memset(lay, 0, sizeof(*lay));
  if (is_int_filter(d.filter) || window < 1 || N64 > (int64_t(1) << 28)) return -5;
  const int N = (int)N64, J = d.J, ncol = tile_cols(false);
  lay->N = N;
  lay->J = J;
  int total = 0;
  for (int l = 1; l <= J; ++l) {
    level_geometry(d, N, l, false, lay);
    const int P = 1 << l, L = N >> l, T = lay->T[l];
    const int Umax = std::max(lay->U[l][0], lay->U[l][1]);
    const int rows_total = L / T;
    // With fewer than 16 phases a level has one column tile, so its rows are
    // the only parallel axis: keep them a multiple of 512 (one 64-row pair
    // per wave of a 512-thread workgroup).  Otherwise column tiles of 16
    // phases spread the work and 64-row granularity suffices.
    const int gran = P < ncol ? 512 : 64;
    int rows = ((window - Umax) / T) / gran * gran;
    rows = std::max(gran, rows);
    rows = std::min(rows, (rows_total + 63) & ~63);
    lay->rows[l] = rows;
    const int W = rows * T + Umax;
    lay->ext[l] = W;
    lay->Ls[l] = (W + T - 1) / T;
    lay->plane_stride[l] = ((T * lay->Ls[l] + 63) / 64) * 64 + 32;
    lay->band_size[l] = 2 * lay->plane_stride[l];
    lay->region_off[l] = 0;
    lay->w_at[l] = 2 * lay->band_size[l];
    const int row = 2 * (lay->V[l][0] + lay->V[l][1]);
    int pc = P;
    if (P >= ncol) {
      int avail = kLdsWordsTwoPerCu - lay->w_at[l];
      if (avail < ncol * row) avail = kLdsWords - lay->w_at[l];
      pc = std::max(ncol, std::min(P, (avail / row) / ncol * ncol));
    }
    lay->pc[l] = pc;
    total = std::max(total, lay->w_at[l] + std::min(pc, P) * row);
  }
  lay->w_off = 0;
  lay->total = total;
  return total <= kLdsWords ? 0 : -5;
}

// Audit of a tile layout against the ranges tile items touch.
inline int tile_layout_violation(const PlanDesc &d, const FusedLayout &lay) {
  const int N = lay.N;
  for (int l = 1; l <= lay.J; ++l) {
    const int L = N >> l, T = lay.T[l], P = 1 << l;
    if (T < 1 || (1 << lay.logT[l]) != T || L % T) return 21;
    // grouped sub-sequences (T >= 4) are read as aligned word quads
    if (T >= 4 && ((lay.region_off[l] | lay.band_size[l] | lay.plane_stride[l]) & 3)) return 29;
    const int rows = lay.rows[l];
    if (rows < 64 || (rows & 63)) return 30;
    for (int b = 0; b < 2; ++b) {
      // window elements q < rows*T + U (the last row pair of a tile reads them)
      if ((rows * T + lay.U[l][b] + T - 1) / T > lay.Ls[l]) return 22;
      if (lay.U[l][b] + T - 2 >= lay.V[l][b]) return 23;
      if (lay.U[l][b] < d.lv[l].len[b] + lay.F[l][b]) return 24;
    }
    if (T * lay.Ls[l] + 32 > lay.plane_stride[l]) return 25;
    if (lay.w_at[l] < 4 * lay.plane_stride[l] || (lay.w_at[l] & 3)) return 26;
    const int row = 2 * (lay.V[l][0] + lay.V[l][1]);
    const int pc = lay.pc[l];
    if (P < 16 ? pc != P : (pc % 16 || pc < 16)) return 27;
    if (lay.w_at[l] + std::min(pc, P) * row > lay.total) return 28;
  }
  return lay.total > kLdsWords ? 29 : 0;
}

// Audit of a layout against the index ranges the fused kernel touches.
// Returns 0 if every access is inside its region and regions that are live
// together are disjoint; otherwise a positive code naming the failed check.
inline int layout_violation(const PlanDesc &d, const FusedLayout &lay) {
  const bool is_int = is_int_filter(d.filter);
  const int ncol = tile_cols(is_int);
  const int N = lay.N;
  for (int l = 1; l <= lay.J; ++l) {
    const int L = N >> l, T = lay.T[l], Ls = lay.Ls[l], P = 1 << l;
    if (T < 1 || (1 << lay.logT[l]) != T || L % T) return 1;
    // grouped sub-sequences (T >= 4) are read as aligned word quads
    if (!is_int && T >= 4 && ((lay.region_off[l] | lay.band_size[l] | lay.plane_stride[l]) & 3))
      return 16;
    // element q < ext: plane offset (q%T)*Ls + q/T must stay below T*Ls
    if ((lay.ext[l] + T - 1) / T > Ls) return 2;
    if (T * Ls + 32 > lay.plane_stride[l]) return 3;
    if (lay.band_size[l] != 2 * lay.plane_stride[l]) return 4;
    if (lay.region_off[l] + 2 * lay.band_size[l] > lay.w_off) return 5;
    if (l > 1) {  // level l must miss c_{l-1}
      const int a0 = lay.region_off[l], a1 = a0 + 2 * lay.band_size[l];
      const int b0 = lay.region_off[l - 1], b1 = b0 + lay.band_size[l - 1];
      if (a0 < b1 && b0 < a1) return 6;
    }
    for (int b = 0; b < 2; ++b) {
      // correlation rows start at q in [0, L-T] (multiples of T), offsets
      // u < U; the next level reads q < L
      if ((L - T) + lay.U[l][b] - 1 >= lay.ext[l]) return 7;
      // weight lookup v = u (+du) - p0 + T - 1 in [0, U + T - 2] < V
      if (lay.U[l][b] + T - 2 >= lay.V[l][b]) return 8;
      if (lay.F[l][b] < T - 1 || lay.F[l][b] > 2 * T - 2) return 9;
      // every tap t < len reachable for every p0 < T: u = t + p0 + F - (T-1) < U
      if (lay.U[l][b] < d.lv[l].len[b] + lay.F[l][b]) return 10;
      if (is_int ? (lay.U[l][b] & 1) : (lay.U[l][b] & 3)) return 11;
    }
    const int row = 2 * (lay.V[l][0] + lay.V[l][1]);
    const int pc = lay.pc[l];
    if (P < ncol ? pc != P : (pc % ncol || pc < ncol)) return 12;
    const int w0 = lay.w_at[l], w1 = w0 + std::min(pc, P) * row;
    if ((w0 & 3) || w0 < 0 || w1 > lay.total) return 13;
    const int r0 = lay.region_off[l], r1 = r0 + 2 * lay.band_size[l];
    if (w0 < r1 && r0 < w1) return 15;
  }
  if (lay.total > kLdsWords || (lay.w_off & 3)) return 14;
  return 0;
}

// Partial-sum slots (kBalSlotWords each) the balanced correlation needs for
// a whole-pulse layout: a level whose last round of MFMA tiles leaves more
// than half of a workgroup's NW waves idle (rem = 1 .. NW/2 tiles) cuts each
// of those tiles over NW / rem waves, whose rem * (NW / rem - 1) helpers
// hand over partial sums; 0 if no level does.  Mirrors the tile count of
// correlate_rows_f32_t.
inline int fused_bal_slots(const FusedLayout &lay) {
  constexpr int NW = kFusedThreads / 64;
  int slots = 0;
  for (int l = 1; l <= lay.J; ++l) {
    const int P = 1 << l;
    const int rows = (lay.N >> l) >> lay.logT[l];
    const int mpairs = (((rows + 31) >> 5) + 1) >> 1;
    const int pc = lay.pc[l] > 0 ? lay.pc[l] : P;
    const int last = P - ((P - 1) / pc) * pc;   // phases of the last column chunk
    const int rem = (mpairs * (P < 16 ? 1 : last >> 4)) % NW;
    if (rem >= 1 && rem <= NW / 2) slots = std::max(slots, rem * (NW / rem - 1));
  }
  return slots;
}

}  // namespace host
}  // namespace sidwt
