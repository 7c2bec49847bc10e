// HIP kernels of libsidwt for gfx950.
//
//   ref_tree_level<F>   x-side lifting of the reference phase tree (plan).
//   fused_correlate<F>  one workgroup per pulse: y-side lifting of all J
//                       levels in LDS, each level correlated against the
//                       plan's stored phases with MFMA as soon as it exists
//                       (for a few pulses, one workgroup per pulse and
//                       plane, each lifting up to its own level).
//   lift_many<F>        y-side lifting only, pyramid written to HBM.
//
// Method references (Bhattacharya & Mahapatra): shift-circulant phases
// Sec. II; dual analysis lifting Sec. III; per-scale correlation eq. (15),
// (20), (20a); the Fig. 5 even/odd tree; Fig. 7 lifting of the received
// signal.
#include <atomic>

#include <type_traits>

#include "sidwt_device.hpp"
#include "sidwt_host.hpp"
#include "sidwt_lift.hpp"

namespace sidwt {

// ===========================================================================
// Reference phase tree (plan creation).
//
// Level l, phase r < 2^l: the input is phase r' = r mod 2^(l-1) of level l-1
// delayed by one sample when r >= 2^(l-1) (shift-circulance, Sec. II; the
// even/odd tree of Fig. 5).  Lifting runs on a zero-extended linear buffer
// of pairs that covers the output supports with a margin.
// ===========================================================================

template <int F> struct XStepsLDS;

template <> struct XStepsLDS<F_LEGALL53> {
  // Sec. III-C Case I: P~(z^-1) = diag(1, 1/2) [1 (1+z^-1)/4; 0 1] [1 0; -(1+z)/2 1]
  __device__ static void run(float2 *e, float2 *o, float2 *, int np, int tid, int nt) {
    for (int k = tid; k < np; k += nt) {
      float2 en = (k + 1 < np) ? e[k + 1] : make_float2(0.f, 0.f);
      o[k] = fma2(-0.5f, add2(e[k], en), o[k]);
    }
    __syncthreads();
    for (int k = tid; k < np; k += nt) {
      float2 op = (k > 0) ? o[k - 1] : make_float2(0.f, 0.f);
      e[k] = fma2(0.25f, add2(op, o[k]), e[k]);
    }
    __syncthreads();
    for (int k = tid; k < np; k += nt) o[k] = scale2(0.5f, o[k]);
    __syncthreads();
  }
};

template <> struct XStepsLDS<F_CDF97> {
  // Sec. III-C Case II: P~(z^-1) = diag(x, 1/x) [1 d(1+z^-1); 0 1]
  //   [1 0; g(1+z) 1] [1 b(1+z^-1); 0 1] [1 0; a(1+z) 1]
  __device__ static void pred(float2 *e, float2 *o, int np, int tid, int nt, float c) {
    for (int k = tid; k < np; k += nt) {
      float2 en = (k + 1 < np) ? e[k + 1] : make_float2(0.f, 0.f);
      o[k] = fma2(c, add2(e[k], en), o[k]);
    }
    __syncthreads();
  }
  __device__ static void upd(float2 *e, float2 *o, int np, int tid, int nt, float c) {
    for (int k = tid; k < np; k += nt) {
      float2 op = (k > 0) ? o[k - 1] : make_float2(0.f, 0.f);
      e[k] = fma2(c, add2(op, o[k]), e[k]);
    }
    __syncthreads();
  }
  __device__ static void run(float2 *e, float2 *o, float2 *, int np, int tid, int nt) {
    pred(e, o, np, tid, nt, C97::a);
    upd(e, o, np, tid, nt, C97::b);
    pred(e, o, np, tid, nt, C97::g);
    upd(e, o, np, tid, nt, C97::d);
    for (int k = tid; k < np; k += nt) {
      e[k] = scale2(C97::xi, e[k]);
      o[k] = scale2(C97::inv_xi, o[k]);
    }
    __syncthreads();
  }
};

template <> struct XStepsLDS<F_D4> {
  // Sec. III-B eq. (17) on pairs (u[2k], u[2k-1]).  `tmp` is a third pair
  // buffer for the step that reads o[k-1] while replacing o.
  __device__ static void run(float2 *e, float2 *o, float2 *tmp, int np, int tid, int nt) {
    for (int k = tid; k < np; k += nt) o[k] = fma2(-CD4::s3, e[k], o[k]);
    __syncthreads();
    for (int k = tid; k < np; k += nt) {
      float2 op = (k > 0) ? o[k - 1] : make_float2(0.f, 0.f);
      e[k] = fma2(CD4::u1, op, fma2(CD4::u0, o[k], e[k]));
    }
    __syncthreads();
    // [1 0; 1 z^-1]: o[k] <- e[k] + o[k-1]
    for (int k = tid; k < np; k += nt) {
      float2 op = (k > 0) ? o[k - 1] : make_float2(0.f, 0.f);
      tmp[k] = add2(e[k], op);
    }
    __syncthreads();
    for (int k = tid; k < np; k += nt) {
      e[k] = scale2(CD4::ka, e[k]);
      o[k] = scale2(CD4::kb, tmp[k]);
    }
    __syncthreads();
  }
};

template <> struct XStepsLDS<F_LEGALL53_INT> {
  // reversible 5/3, x-side:  o -= (e[k]+e[k+1])>>1 ;  e += (o[k-1]+o[k]+2)>>2
  __device__ static void run(int2 *e, int2 *o, int2 *, int np, int tid, int nt) {
    for (int k = tid; k < np; k += nt) {
      int2 en = (k + 1 < np) ? e[k + 1] : make_int2(0, 0);
      o[k].x -= (e[k].x + en.x) >> 1;
      o[k].y -= (e[k].y + en.y) >> 1;
    }
    __syncthreads();
    for (int k = tid; k < np; k += nt) {
      int2 op = (k > 0) ? o[k - 1] : make_int2(0, 0);
      e[k].x += (op.x + o[k].x + 2) >> 2;
      e[k].y += (op.y + o[k].y + 2) >> 2;
    }
    __syncthreads();
  }
};

template <int F> struct XOddBefore { static constexpr bool v = false; };
template <> struct XOddBefore<F_D4> { static constexpr bool v = true; };

// One block per phase r.  `in` holds 2^(l-1) phases of in_len elements each
// (level 1: the reference itself, a single "phase").  Pair buffer covers
// k in [k0, k0 + np).
template <int F>
__global__ __launch_bounds__(256) void ref_tree_level(
    const typename ElemOf<F>::T *__restrict__ in, int in_lo, int in_len, int level,
    int k0, int np, typename ElemOf<F>::T *__restrict__ outA, int loA, int lenA,
    typename ElemOf<F>::T *__restrict__ outB, int loB, int lenB) {
  using V = typename ElemOf<F>::T;
  extern __shared__ __align__(16) char smem_tree[];
  V *e = reinterpret_cast<V *>(smem_tree);
  V *o = e + np;
  V *tmp = o + np;
  const int r = blockIdx.x;
  const int half = 1 << (level - 1);
  const int rp = (level == 1) ? 0 : (r & (half - 1));
  const int delay = r >> (level - 1);
  const V *src = in + (long long)rp * in_len;
  const int tid = threadIdx.x, nt = blockDim.x;
  auto sample = [&](int t) -> V {
    int i = t - delay - in_lo;
    V z;
    if (i >= 0 && i < in_len) return src[i];
    z.x = 0; z.y = 0;
    return z;
  };
  for (int kk = tid; kk < np; kk += nt) {
    int k = k0 + kk;
    e[kk] = sample(2 * k);
    o[kk] = XOddBefore<F>::v ? sample(2 * k - 1) : sample(2 * k + 1);
  }
  __syncthreads();
  XStepsLDS<F>::run(e, o, tmp, np, tid, nt);
  for (int t = tid; t < lenA; t += nt) outA[(long long)r * lenA + t] = e[loA + t - k0];
  for (int t = tid; t < lenB; t += nt) outB[(long long)r * lenB + t] = o[loB + t - k0];
}


template <int F> struct RxOf { using T = float2; using Out = float; };
template <> struct RxOf<F_LEGALL53_INT> { using T = short2; using Out = long long; };

// ===========================================================================
// Per-scale correlation of one level against the stored phases (eq. (20),
// (20a)): plane j = l-1, P = 2^l phases, L = N/2^l lags per phase,
//
//   R[P p + r] = sum_t conj(a_r[t]) c[(p + t) mod L] + conj(b_r[t]) d[(p + t) mod L]
//
// computed as a real GEMM.  Rows: lag blocks p1 (p = p1*T + p0).  Columns:
// (p0, r, re/im out) -- Toeplitz blocking of the lag axis, T*P columns of
// complex outputs per tile when P is small, plain phases when T = 1.
// K: lag offset u (data element q = p1*T + lo + u) times re/im in.  The
// complex product conj(w) c is the 2x2 real embedding
//   [out.re; out.im] = [w.re  w.im; -w.im  w.re] [c.re; c.im].
// FP32 path: v_mfma_f32_32x32x2_f32 (one lag offset per MFMA, T*P = 16).
// Integer path: v_mfma_f64_16x16x4_f64 on int32 data and phases, exact
// because every product and partial sum is an integer below 2^53.
// ===========================================================================

// One level as the correlation engine sees it: where the two bands sit in
// LDS (polyphase planes, see FusedLayout), the lag windows, the staged
// weight geometry, and the range of lag-block rows p1 to produce.
struct LevelView {
  int l, P, L, T, logT, Ls, plane_stride;
  int base[2];          // word offset of band b's re plane
  int lo[2];            // lag-window start (aligned to T)
  int U[2], V[2], F[2];
  int pc, w_at;
  int wrap;             // 1: band holds the whole level (+halo), row p1 starts at
                        //    element (p1*T + lo) mod L; 0: band holds a window
                        //    whose element 0 is row row_begin's first element
  int row_begin, row_end;
};

__device__ __forceinline__ LevelView fused_view(const FusedLayout &lay, int l) {
  LevelView v;
  v.l = l;
  v.P = 1 << l;
  v.L = lay.N >> l;
  v.T = lay.T[l];
  v.logT = lay.logT[l];
  v.Ls = lay.Ls[l];
  v.plane_stride = lay.plane_stride[l];
  for (int b = 0; b < 2; ++b) {
    v.base[b] = lay.region_off[l] + b * lay.band_size[l];
    v.lo[b] = lay.lo[l][b];
    v.U[b] = lay.U[l][b];
    v.V[b] = lay.V[l][b];
    v.F[b] = lay.F[l][b];
  }
  v.pc = lay.pc[l];
  v.w_at = lay.w_at[l];
  v.wrap = 1;
  v.row_begin = 0;
  v.row_end = v.L >> v.logT;
  return v;
}

// Stage phases r0..r0+pcc-1 of both bands as complex rows W[b][rr][v] with
// W[v] = w[v - F] (zero outside the stored support).
// KB coefficient loads per thread are issued before any of them is stored
// (more reads in flight; the tile items' kernel gains from it, while the
// whole-pulse kernel, whose registers are scarcer, keeps one).
template <int KB, class V>
__device__ __forceinline__ void stage_weights(const PlanDesc &plan, const LevelView &lv, int r0,
                                              int pcc, V *W) {
  // coefficients read as 8-byte words through a global-memory pointer
  static_assert(sizeof(V) == 8, "complex element of 8 bytes");
  typedef __attribute__((address_space(1))) const long long gw;
  const LevelDesc &ld = plan.lv[lv.l];
  // One loop per band, so that the band's support, offset and shift are
  // workgroup-uniform values read once (a per-lane band index would fetch
  // them from the descriptor in memory for every element, in series with
  // the coefficient load).
  V *Wb = W;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int Vb = lv.V[b], Fb = lv.F[b], len = ld.len[b];
    const gw *coef = (const gw *)plan.coef + ld.off[b] + (long long)r0 * len;
    const int tot = pcc * Vb;
    if constexpr (KB == 1) {
      for (int i = threadIdx.x; i < tot; i += blockDim.x) {
        const int rr = i / Vb;
        const int t = i - rr * Vb - Fb;
        V w;
        w.x = 0;
        w.y = 0;
        if (t >= 0 && t < len) w = __builtin_bit_cast(V, coef[(long long)rr * len + t]);
        Wb[i] = w;
      }
    } else {
      // entries outside the support (and indexes past tot) load the row's
      // first coefficient, which exists, and store zero (or nothing)
      const int nt = blockDim.x;
      for (int i0 = threadIdx.x; i0 < tot; i0 += KB * nt) {
        V w[KB];
        bool ok[KB];
#pragma unroll
        for (int k = 0; k < KB; ++k) {
          const int i = min(i0 + k * nt, tot - 1);
          const int rr = i / Vb;
          const int t = i - rr * Vb - Fb;
          ok[k] = t >= 0 && t < len;
          w[k] = __builtin_bit_cast(V, coef[ok[k] ? (long long)rr * len + t : 0]);
        }
#pragma unroll
        for (int k = 0; k < KB; ++k) {
          if (!ok[k]) {
            w[k].x = 0;
            w[k].y = 0;
          }
          if (i0 + k * nt < tot) Wb[i0 + k * nt] = w[k];
        }
      }
    }
    Wb += tot;
  }
}

__device__ __forceinline__ f32x16 mfma32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int row_start(const LevelView &v, int p1, int b) {
  return v.wrap ? (pos_mod(p1 * v.T + v.lo[b], v.L) >> v.logT) : (p1 - v.row_begin);
}

// FP32 correlation of rows [row_begin, row_end) of one level (32x32x2
// tiles, two row tiles per wave that share the weight operand), for a
// compile-time Toeplitz block TT.  outp is the plane's output (complex64 as
// float pairs), indexed by global lag.
//
// A tile's work is its G0 + G1 groups of four lag offsets (band 0, then
// band 1).  Tiles go to waves round-robin.  With BAL, on a level's last
// column chunk, when the last round would leave more than half of the waves
// idle, its rem tiles are each cut into NW / rem equal group ranges, one per
// wave: the partial sums pass through LDS slots of kBalSlotWords per wave
// (aliasing the band windows and weights, which are no longer read) and
// are added in wave order, so the result does not depend on timing.  The
// rem * (NW / rem - 1) slots (at most NW - 1) start at word slot_at of smf: 0 for a tile item (they alias its
// windows and weights, no longer read), the end of the layout for a whole
// pulse (whose bands stay live); the allocation must hold NW * kBalSlotWords
// words from there.
template <int TT, bool BAL>
__device__ __forceinline__ void correlate_rows_f32_t(const PlanDesc &plan, const LevelView &v, float *smf,
                                     float *__restrict__ outp, int slot_at) {
  constexpr int LT = TT == 1 ? 0 : TT == 2 ? 1 : TT == 4 ? 2 : 3;
  static_assert(TT == 1 || TT == 2 || TT == 4 || TT == 8, "Toeplitz block");
  const int P = v.P, l = v.l, Ls = v.Ls;
  const int nrows = v.row_end - v.row_begin;
  const int mtiles = (nrows + 31) >> 5;
  const int mpairs = (mtiles + 1) >> 1;
  const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  float2 *W = reinterpret_cast<float2 *>(smf + v.w_at);
  const int V0 = v.V[0], V1 = v.V[1];
  const int G0 = v.U[0] >> 2, GT = G0 + (v.U[1] >> 2);
  const int row = lane & 31;
  const int ci = lane >> 5;
  const int co = lane & 1;
  const int cc = (lane & 31) >> 1;
  const bool neg = (ci == 0) && (co == 1);
  for (int r0 = 0; r0 < P; r0 += v.pc) {
    const int pcc = min(v.pc, P - r0);
    stage_weights<BAL ? 4 : 1>(plan, v, r0, pcc, W);
    __syncthreads();
    // P < 16: one column tile holds all (p0, r) pairs, p0 < TT; otherwise
    // TT = 1 and each column tile holds 16 phases.
    const int ntn = (P < 16) ? 1 : (pcc >> 4);
    const int ntiles = mpairs * ntn;
    // Tile (mp, nt): row pair mp, column tile nt.  Column r / block offset
    // p0 of this lane; false for the columns of a P < 16 tile beyond TT
    // blocks (computed, never stored).
    auto place = [&](int nt, int &r, int &p0) {
      if (P < 16) {
        r = cc & (P - 1);
        p0 = cc >> l;
        const bool ok = p0 < TT;
        if (!ok) p0 = 0;
        return ok;
      }
      r = nt * 16 + cc;
      p0 = 0;
      return true;
    };
    // acc0/acc1 (row tiles 2*mp, 2*mp + 1) += groups [ga, gb) of tile (mp, nt).
    auto accumulate = [&](int mp, int nt, int ga, int gb, f32x16 &acc0, f32x16 &acc1) {
      int r, p0;
      (void)place(nt, r, p0);
      const int p1a = v.row_begin + mp * 64 + row;
      const int p1b = p1a + 32;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int G = v.U[b] >> 2;
        int glo = 0, ghi = G;
        if constexpr (BAL) {
          const int off = b ? G0 : 0;
          glo = max(ga - off, 0);
          ghi = min(gb - off, G);
          if (glo >= ghi) continue;
        }
        const float *pl = smf + v.base[b] + ci * v.plane_stride;
        const int ia = row_start(v, p1a, b), ib = row_start(v, p1b, b);  // sub-sequence index
        const float *wp = reinterpret_cast<const float *>(W + (b ? pcc * V0 : 0) + r * (b ? V1 : V0)) +
                          2 * (TT - 1 - p0) + (ci ^ co);
        // The four data values of group g (lag offsets 4g..4g+3) of a row
        // whose first element has sub-sequence index i.
        auto data = [&](int i, int g, float(&A)[4]) {
          if constexpr (TT >= 4) {
            // one quad: block g mod (TT/4), index i + g / (TT/4)
            constexpr int GB = TT / 4, LGB = LT - 2;
            const f32x4 q4 = *reinterpret_cast<const f32x4 *>(
                pl + (g & (GB - 1)) * (4 * Ls) + 4 * (i + (g >> LGB)));
#pragma unroll
            for (int q = 0; q < 4; ++q) A[q] = q4[q];
          } else if constexpr (TT == 2) {
            // offsets u = 4g + q: sub-sequence q & 1, index i + 2g + q / 2
            const float *p = pl + i + 2 * g;
#pragma unroll
            for (int q = 0; q < 4; ++q) A[q] = p[(q & 1) * Ls + (q >> 1)];
          } else {
            const float *p = pl + i + 4 * g;
#pragma unroll
            for (int q = 0; q < 4; ++q) A[q] = p[q];
          }
        };
        // Groups of 4 lag offsets in two register sets (x, y): the loads of
        // a group are issued one whole group of MFMAs before its use, with
        // no register moves in between (a move would make the wave wait
        // for the loads it just issued).  TWO: both row tiles; otherwise
        // only the first (the second lies past the level's last row).
        auto kloop = [&](auto two_c) {
          constexpr bool TWO = decltype(two_c)::value;
          auto load = [&](int g, float(&A0)[4], float(&A1)[4], float(&Wt)[4]) {
            data(ia, g, A0);
            if constexpr (TWO) data(ib, g, A1);
            const float *w = wp + 8 * g;
#pragma unroll
            for (int q = 0; q < 4; ++q) Wt[q] = w[2 * q];
          };
          auto mma = [&](const float(&A0)[4], const float(&A1)[4], const float(&Wt)[4]) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const float wq = neg ? -Wt[q] : Wt[q];
              acc0 = mfma32(A0[q], wq, acc0);
              if constexpr (TWO) acc1 = mfma32(A1[q], wq, acc1);
            }
          };
          float xa0[4], xa1[4] = {}, xw[4], ya0[4], ya1[4] = {}, yw[4];
          load(glo, xa0, xa1, xw);
          for (int g = glo; g < ghi; g += 2) {
            load(min(g + 1, ghi - 1), ya0, ya1, yw);
            __builtin_amdgcn_sched_barrier(0);
            mma(xa0, xa1, xw);
            __builtin_amdgcn_sched_barrier(0);
            load(min(g + 2, ghi - 1), xa0, xa1, xw);
            __builtin_amdgcn_sched_barrier(0);
            if (g + 1 < ghi) mma(ya0, ya1, yw);
            __builtin_amdgcn_sched_barrier(0);
          }
        };
        // rows of the second tile (uniform over the wave) are never stored
        // when it starts at or past the level's end: with BAL (the tile
        // items, whose deepest levels have 16-32 rows) its products are
        // skipped; the whole-pulse kernel's levels fill their tile pairs
        if (!BAL || v.row_begin + mp * 64 + 32 < v.row_end)
          kloop(std::true_type{});
        else if constexpr (BAL)
          kloop(std::false_type{});
      }
    };
    auto store = [&](int mp, int nt, const f32x16 &acc0, const f32x16 &acc1) {
      int r, p0;
      if (!place(nt, r, p0)) return;
      // With BAL the lane index is made opaque here so that the compiler
      // cannot precompute these addresses ahead of the MFMA loop (which would
      // hold them in registers through it).
      int ln = lane;
      if constexpr (BAL) asm volatile("" : "+v"(ln));
      // register i of lane l: row 8*(i/4) + 4*(l/32) + i%4, column l%32.
      // The lane's address is formed once; register (h, i) adds a uniform
      // offset of rows; a tile pair whose 64 rows are all in range stores
      // without guards.
      const int pr0 = v.row_begin + mp * 64 + 4 * (ln >> 5);
      const long long s0 = (long long)P * (pr0 * TT + p0) + r0 + r;
      typedef __attribute__((address_space(1))) float gf;
      gf *o0 = (gf *)outp + 2 * s0 + co;
      const long long rs2 = 2LL * P * TT;  // floats per row of lags
      const bool full = v.row_begin + mp * 64 + 64 <= v.row_end;
      if (full) {
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int i = 0; i < 16; ++i)
            __builtin_nontemporal_store(h ? acc1[i] : acc0[i],
                                        o0 + rs2 * (h * 32 + 8 * (i >> 2) + (i & 3)));
      } else {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const int dr = h * 32 + 8 * (i >> 2) + (i & 3);
            if (pr0 + dr < v.row_end)
              __builtin_nontemporal_store(h ? acc1[i] : acc0[i], o0 + rs2 * dr);
          }
        }
      }
    };
    auto zero = [](f32x16 &a) {
#pragma unroll
      for (int i = 0; i < 16; ++i) a[i] = 0.f;
    };
    // Whole tiles round-robin; with BAL, on a level's last chunk, the
    // rem = ntiles mod NW tiles of an incomplete last round (rem <= NW / 2)
    // are each cut into c = NW / rem group ranges, one per wave.
    constexpr int NW = kFusedThreads / 64;  // both batch kernels run kFusedThreads
    int rem = 0;
    if constexpr (BAL) {
      if (r0 + pcc == P && ntiles % NW <= NW / 2) rem = ntiles % NW;
    }
    for (int tile = wave; tile < ntiles - rem; tile += nw) {
      const int mp = tile % mpairs, nt = tile / mpairs;
      f32x16 acc0, acc1;
      zero(acc0);
      zero(acc1);
      accumulate(mp, nt, 0, GT, acc0, acc1);
      store(mp, nt, acc0, acc1);
    }
    if (rem > 0) {
      const int c = NW / rem;
      const int part = wave % c;
      const int tile = ntiles - rem + wave / c;
      const int mp = tile % mpairs, nt = tile / mpairs;
      f32x16 acc0, acc1;
      zero(acc0);
      zero(acc1);
      if (wave < rem * c) accumulate(mp, nt, part * GT / c, (part + 1) * GT / c, acc0, acc1);
      __syncthreads();  // every wave is done with the windows and weights
      if (wave < rem * c && part > 0) {
        // compact slots: the c - 1 helpers of each cut tile, in wave order
        f32x4 *sl = reinterpret_cast<f32x4 *>(
                        smf + slot_at + ((wave / c) * (c - 1) + part - 1) * kBalSlotWords) +
                    lane;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          sl[k * 64] = f32x4{acc0[4 * k], acc0[4 * k + 1], acc0[4 * k + 2], acc0[4 * k + 3]};
          sl[(k + 4) * 64] = f32x4{acc1[4 * k], acc1[4 * k + 1], acc1[4 * k + 2], acc1[4 * k + 3]};
        }
      }
      __syncthreads();
      if (wave < rem * c && part == 0) {
        for (int k2 = 1; k2 < c; ++k2) {  // in wave order: the sum does not depend on timing
          const f32x4 *sl = reinterpret_cast<const f32x4 *>(
                                smf + slot_at + ((wave / c) * (c - 1) + k2 - 1) * kBalSlotWords) +
                            lane;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const f32x4 a = sl[k * 64], b = sl[(k + 4) * 64];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              acc0[4 * k + j] += a[j];
              acc1[4 * k + j] += b[j];
            }
          }
        }
        store(mp, nt, acc0, acc1);
      }
    }
    __syncthreads();
  }
}

template <bool BAL = false>
__device__ __forceinline__ void correlate_rows_f32(const PlanDesc &plan, const LevelView &v, float *smf,
                                   float *__restrict__ outp, int slot_at = 0) {
  switch (v.T) {
    case 8: correlate_rows_f32_t<8, BAL>(plan, v, smf, outp, slot_at); break;
    case 4: correlate_rows_f32_t<4, BAL>(plan, v, smf, outp, slot_at); break;
    case 2: correlate_rows_f32_t<2, BAL>(plan, v, smf, outp, slot_at); break;
    default: correlate_rows_f32_t<1, BAL>(plan, v, smf, outp, slot_at); break;
  }
}

// Integer correlation of one whole level (FP64 16x16x4 tiles, two row
// tiles per wave sharing the weight operand).
__device__ void correlate_level_int(const PlanDesc &plan, const LevelView &v, int *smi,
                                    long long *__restrict__ outp) {
  const int P = v.P, l = v.l, L = v.L, T = v.T, logT = v.logT, Ls = v.Ls;
  const int Mrows = v.row_end;
  const int mtiles = (Mrows + 15) >> 4;
  const int mpairs = (mtiles + 1) >> 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int2 *W = reinterpret_cast<int2 *>(smi + v.w_at);
  const int V0 = v.V[0], V1 = v.V[1];
  const int row = lane & 15;
  const int kq = lane >> 4;
  const int du = kq >> 1;
  const int ci = kq & 1;
  const int co = lane & 1;
  const int cc = (lane & 15) >> 1;
  const bool neg = (ci == 0) && (co == 1);
  for (int r0 = 0; r0 < P; r0 += v.pc) {
    const int pcc = min(v.pc, P - r0);
    stage_weights<1>(plan, v, r0, pcc, W);
    __syncthreads();
    const int ntn = (P < 8) ? 1 : (pcc >> 3);
    const int ntiles = mpairs * ntn;
    for (int tile = wave; tile < ntiles; tile += nw) {
      const int mp = tile % mpairs;
      const int ntile = tile / mpairs;
      int r, p0;
      bool colok;
      if (P < 8) {
        r = cc & (P - 1);
        p0 = cc >> l;
        colok = p0 < T;
        if (!colok) p0 = 0;
      } else {
        r = ntile * 8 + cc;
        p0 = 0;
        colok = true;
      }
      const int p1a = mp * 32 + row;
      const int p1b = p1a + 16;
      f64x4 acc0 = {0, 0, 0, 0};
      f64x4 acc1 = {0, 0, 0, 0};
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int steps = v.U[b] >> 1;
        const int *pl = smi + v.base[b] + ci * v.plane_stride;
        const int qa = pos_mod(p1a * T + v.lo[b], L);
        const int qb = pos_mod(p1b * T + v.lo[b], L);
        const int *wp = reinterpret_cast<const int *>(W + (b ? pcc * V0 : 0) + r * (b ? V1 : V0)) +
                        2 * (du - p0 + T - 1) + (ci ^ co);
        for (int st = 0; st < steps; ++st) {
          const int u = 2 * st + du;
          const int a0 = pl[poly_off(qa + u, logT, Ls, false)];
          const int a1 = pl[poly_off(qb + u, logT, Ls, false)];
          int wv = wp[4 * st];
          wv = neg ? -wv : wv;
          wv = colok ? wv : 0;
          const double wd = (double)wv;
          acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a0, wd, acc0, 0, 0, 0);
          acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a1, wd, acc1, 0, 0, 0);
        }
      }
      if (colok) {
        // register i of lane l: row 4*i + l/16, column l%16
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int pp1 = mp * 32 + h * 16 + 4 * i + (lane >> 4);
            if (pp1 < Mrows) {
              const long long s = (long long)P * (pp1 * T + p0) + r0 + r;
              outp[2 * s + co] = (long long)(h ? acc1[i] : acc0[i]);
            }
          }
        }
      }
    }
    __syncthreads();
  }
}

// Store one lifted pair of level l (c into band 0, d into band 1) with its
// halo copies.
template <class V, class S>
__device__ __forceinline__ void store_pair(S *sm, const FusedLayout &lay, int l, int k, V c, V d) {
  const int L = lay.N >> l;
  S *b0 = sm + lay.region_off[l];
  S *b1 = b0 + lay.band_size[l];
  const int ps = lay.plane_stride[l];
  constexpr bool grouped = std::is_same<V, float2>::value;
  for (int q = k; q < lay.ext[l]; q += L) {
    const int o = poly_off(q, lay.logT[l], lay.Ls[l], grouped);
    b0[o] = c.x;
    b0[o + ps] = c.y;
    b1[o] = d.x;
    b1[o + ps] = d.y;
  }
}

template <class V, class S>
__device__ __forceinline__ V load_elem(const S *sm, const FusedLayout &lay, int l, int q) {
  const S *b0 = sm + lay.region_off[l];
  const int o = poly_off(q, lay.logT[l], lay.Ls[l], std::is_same<V, float2>::value);
  V v;
  v.x = b0[o];
  v.y = b0[o + lay.plane_stride[l]];
  return v;
}

// ===========================================================================
// Fused kernel: one workgroup per pulse.  Level 1 is lifted straight from
// HBM; every level's bands are correlated as soon as they exist, then the
// next level is lifted from c_l.  Odd and even levels live in alternating
// LDS regions so that c_l stays intact while level l+1 is written.  With
// BAL (float filters), levels whose last round of tiles would leave most
// waves idle cut those tiles over the waves (see correlate_rows_f32_t),
// with partial-sum slots from word lay.total of smem.
// ===========================================================================
template <int F, bool BAL = false>
__device__ __forceinline__ void fused_pulse(const PlanDesc &plan, const FusedLayout &lay,
                            const typename RxOf<F>::T *__restrict__ rx, long long n,
                            typename RxOf<F>::Out *__restrict__ out, char *smem,
                            unsigned planes = ~0u) {
  constexpr bool INT = (F == F_LEGALL53_INT);
  using V = typename ElemOf<F>::T;
  using S = typename std::conditional<INT, int, float>::type;
  constexpr bool OB = YLift<F>::kOddBefore;
  S *sm = reinterpret_cast<S *>(smem);
  const int N = lay.N;

  // Level 1 straight from HBM (pairs split at load, zero padding n..N-1).
  lift_level<F, 2>(
      N >> 1,
      [&](int kc, V &e, V &o) {
        e = rx_sample(rx, n, 2 * kc);
        o = rx_sample(rx, n, OB ? (kc == 0 ? N - 1 : 2 * kc - 1) : 2 * kc + 1);
      },
      [&](int k, V c, V d) { store_pair(sm, lay, 1, k, c, d); });
  __syncthreads();

  // levels past the last requested plane's are not lifted
  const int lmax = 32 - __builtin_clz(planes & ((2u << (lay.J - 1)) - 1u));
  for (int l = 1; l <= lmax; ++l) {
    // plane l-1 only if requested (a coarse-scale subset costs only its own
    // correlation; every level up to it is still lifted)
    if ((planes >> (l - 1)) & 1u) {
      if constexpr (INT) {
        correlate_level_int(plan, fused_view(lay, l), sm, out + 2LL * (l - 1) * N);
      } else {
        correlate_rows_f32<BAL>(plan, fused_view(lay, l), sm, out + 2LL * (l - 1) * N, lay.total);
      }
    }
    if (l < lmax) {
      const int np = N >> (l + 1);
      const int Lin = N >> l;
      lift_level<F, 1>(
          np,
          [&](int kc, V &e, V &o) {
            e = load_elem<V>(sm, lay, l, 2 * kc);
            o = load_elem<V>(sm, lay, l, OB ? (kc == 0 ? Lin - 1 : 2 * kc - 1) : 2 * kc + 1);
          },
          [&](int k, V c, V d) { store_pair(sm, lay, l + 1, k, c, d); });
    }
    __syncthreads();
  }
}

template <int F, bool BAL>
__global__ __launch_bounds__(kFusedThreads) void fused_correlate(PlanDesc plan, FusedLayout lay,
                                                                const void *__restrict__ rx_all,
                                                                long long n, long long rx_stride,
                                                                void *__restrict__ out_all,
                                                                long long out_stride,
                                                                unsigned planes, int split) {
  using RxT = typename RxOf<F>::T;
  using OutT = typename RxOf<F>::Out;
  extern __shared__ __align__(16) char smem_fused[];
  // split = J: one workgroup per (pulse, plane), each lifting only the
  // levels its plane needs (few pulses: the planes run side by side)
  long long pulse = blockIdx.x;
  if (split) {
    pulse = blockIdx.x / split;
    planes &= 1u << (blockIdx.x - pulse * split);
    if (!planes) return;
  }
  fused_pulse<F, BAL>(plan, lay, reinterpret_cast<const RxT *>(rx_all) + pulse * rx_stride, n,
                      reinterpret_cast<OutT *>(out_all) + pulse * out_stride * 2, smem_fused,
                      planes);
}

// ===========================================================================
// Uneven batches.  Long pulses are lifted into an HBM scratch pyramid (c_l
// then d_l for l = 1..J, 2N complex per pulse) in multi-level passes; one
// persistent kernel then pulls work items from an atomic counter: whole
// short pulses (fused path above) and lag tiles (rows of one level) of long
// pulses, whose band windows are read from the scratch pyramid.
// ===========================================================================

// One block of a multi-level lifting pass (see LiftBlock): level l0 lifted
// from the input level in global memory (register windows, as the
// level-by-level kernel), then levels l0 + 1 .. l1 from the two LDS buffers
// in turn; each level's own pairs also go to the pyramid.  LDS reads through
// the circular index are clamped to the stretch (lanes past a window's end
// load values that are never used).
template <int F>
__device__ void lift_block(const BatchPulse &p, float2 *scratch, const LiftBlock &bk, float2 *sm) {
  constexpr bool OB = YLift<F>::kOddBefore;
  const int N = p.N, l0 = bk.l0, l1 = bk.l1;
  int s[kMaxLevels + 1], e[kMaxLevels + 1], os[kMaxLevels + 1], oe[kMaxLevels + 1];
  lift_block_ranges(N, l0, l1, bk.blk, s, e, os, oe);
  float2 *buf[2] = {sm, sm + (e[l0] - s[l0])};
  {
    const int Nin = N >> (l0 - 1), np = N >> l0, so = s[l0];
    const int o0 = os[l0], o1 = oe[l0];
    const bool keep = l1 > l0;
    float2 *c = scratch + p.scratch + scratch_level_off(N, l0);
    float2 *d = c + np;
    float2 *out = buf[0];
    auto store = [&](int k, float2 cv, float2 dv) {
      if (keep) out[k - so] = cv;
      if (k >= o0 && k < o1) {
        c[k] = cv;
        d[k] = dv;
      }
    };
    if (l0 == 1) {
      const float2 *rx = reinterpret_cast<const float2 *>(p.rx);
      const int n = (int)p.n;
      lift_level_range<F, 4>(
          np, s[l0], e[l0],
          [&](int kc, float2 &ev, float2 &ov) {
            ev = rx_sample_global(rx, n, 2 * kc);
            ov = rx_sample_global(rx, n, OB ? (kc == 0 ? Nin - 1 : 2 * kc - 1) : 2 * kc + 1);
          },
          store);
    } else {
      const float2 *src = scratch + p.scratch + scratch_level_off(N, l0 - 1);
      lift_level_range<F, 4>(
          np, s[l0], e[l0], [&](int kc, float2 &ev, float2 &ov) { pair_at<OB>(src, kc, np, ev, ov); },
          store);
    }
  }
  __syncthreads();
  for (int l = l0 + 1; l <= l1; ++l) {
    const float2 *in = buf[(l - l0 - 1) & 1];
    float2 *out = buf[(l - l0) & 1];
    const int Nin = N >> (l - 1), np = N >> l;
    const int S = s[l - 1], R = e[l - 1] - S, so = s[l];
    const int o0 = os[l], o1 = oe[l];
    const bool keep = l < l1;
    float2 *c = scratch + p.scratch + scratch_level_off(N, l);
    float2 *d = c + np;
    lift_level_range<F, 2>(
        np, s[l], e[l],
        [&](int kc, float2 &ev, float2 &ov) {
          // q - S lies in (-Nin, 2 Nin): one conditional wrap, no division
          auto at = [&](int q) {
            int i = q - S;
            i = i < 0 ? i + Nin : (i >= Nin ? i - Nin : i);
            return in[min(i, R - 1)];
          };
          ev = at(2 * kc);
          ov = at(OB ? (kc == 0 ? Nin - 1 : 2 * kc - 1) : 2 * kc + 1);
        },
        [&](int k, float2 cv, float2 dv) {
          if (keep) out[k - so] = cv;
          if (k >= o0 && k < o1) {
            c[k] = cv;
            d[k] = dv;
          }
        });
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void batch_lift_blocks(const PlanDesc *__restrict__ plans,
                                                         const BatchPulse *__restrict__ pulses,
                                                         const LiftBlock *__restrict__ blocks,
                                                         float2 *__restrict__ scratch) {
  extern __shared__ __align__(16) float2 sm_lift[];
  const LiftBlock bk = blocks[blockIdx.x];
  const BatchPulse &p = pulses[bk.pulse];
  switch (plans[p.plan].filter) {
    case F_LEGALL53: lift_block<F_LEGALL53>(p, scratch, bk, sm_lift); break;
    case F_CDF97: lift_block<F_CDF97>(p, scratch, bk, sm_lift); break;
    case F_D4: lift_block<F_D4>(p, scratch, bk, sm_lift); break;
    default: break;
  }
}

// Lag tile of a long pulse: level l, rows [row0, row0 + rows).  `tl` is the
// pulse's tile layout (per level: T, windows, staging geometry; bands start
// at word 0, band 1 at 2*plane_stride, weights at w_at).
template <bool BAL>
__device__ __forceinline__ void tile_item(const PlanDesc &plan, const FusedLayout &tl, const BatchPulse &p,
                          const BatchItem &it, const float2 *__restrict__ scratch, float *smf) {
  const int l = it.level;
  LevelView v;
  v.l = l;
  v.P = 1 << l;
  v.L = p.N >> l;
  v.T = tl.T[l];
  v.logT = tl.logT[l];
  v.Ls = tl.Ls[l];
  v.plane_stride = tl.plane_stride[l];
  for (int b = 0; b < 2; ++b) {
    v.base[b] = b * 2 * tl.plane_stride[l];
    v.lo[b] = tl.lo[l][b];
    v.U[b] = tl.U[l][b];
    v.V[b] = tl.V[l][b];
    v.F[b] = tl.F[l][b];
  }
  v.pc = tl.pc[l];
  v.w_at = tl.w_at[l];
  v.wrap = 0;
  v.row_begin = it.row0;
  v.row_end = min(it.row0 + it.rows, v.L >> v.logT);
  // Band windows: element q of band b is c_l / d_l at (row0*T + lo + q) mod L,
  // for q below (rows rounded up to 64)*T + U (the last row pair reads them;
  // rows never exceeds the layout's tile rows, a multiple of 64).
  const int rows64 = (it.rows + 63) & ~63;
  const float2 *src0 = scratch + p.scratch + scratch_level_off(p.N, l);
  // Each thread fetches 8 elements before storing any, so 8 HBM reads are
  // in flight instead of one: e is always a valid element index, so the
  // loads need no condition; only the LDS stores check q < Wb.
  constexpr int KB = 8;
  const int nt = blockDim.x;
  const int step = pos_mod(nt, v.L);
  for (int b = 0; b < 2; ++b) {
    const float2 *src = src0 + (b ? v.L : 0);
    const int Wb = rows64 * v.T + v.U[b];
    float *pl = smf + v.base[b];
    int e = pos_mod(it.row0 * v.T + v.lo[b] + (int)threadIdx.x, v.L);
    for (int q0 = threadIdx.x; q0 < Wb; q0 += KB * nt) {
      float2 x[KB];
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        x[k] = src[e];
        e += step;
        if (e >= v.L) e -= v.L;
      }
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        const int q = q0 + k * nt;
        if (q < Wb) {
          const int o = poly_off(q, v.logT, v.Ls, true);
          pl[o] = x[k].x;
          pl[o + v.plane_stride] = x[k].y;
        }
      }
    }
  }
  // No barrier here: the correlation stages its weights first and its
  // barrier after the staging also covers these window stores.
  correlate_rows_f32<BAL>(plan, v, smf, reinterpret_cast<float *>(p.out) + 2LL * (l - 1) * p.N);
}

// Persistent kernel over work items taken from an atomic counter.  The
// general instance runs whole-pulse items (the fused path of three filters,
// inlined) and tile items; the TILES_ONLY instance compiles only the tile
// path and spreads each tile item's work evenly over the waves (see
// correlate_rows_f32_t), which needs an LDS allocation of at least
// kBalMinLdsBytes.
template <bool TILES_ONLY>
__global__ __launch_bounds__(kFusedThreads) void batch_persistent(
    const PlanDesc *__restrict__ plans, const FusedLayout *__restrict__ lays,
    const BatchPulse *__restrict__ pulses, const BatchItem *__restrict__ items, int nitems,
    int *__restrict__ counter, const float2 *__restrict__ scratch) {
  extern __shared__ __align__(16) char smem_batch[];
  // Items are claimed one ahead: thread 0 holds the claim for the following
  // item while the current one runs (hiding the atomic's latency), and the
  // claimed index is published through alternating slots, so one barrier
  // per item both publishes it and ends every wave's use of the item's LDS.
  // The counter only grows, so every workgroup ends on a claim >= nitems.
  __shared__ int slot[2];
  if (threadIdx.x == 0) slot[0] = atomicAdd(counter, 1);
  __syncthreads();
  int i = __builtin_amdgcn_readfirstlane(slot[0]);
  for (int k = 1; i < nitems; k ^= 1) {
    int ahead = 0;
    if (threadIdx.x == 0) ahead = atomicAdd(counter, 1);
    const BatchItem it = items[i];
    const BatchPulse &p = pulses[it.pulse];
    const PlanDesc &plan = plans[p.plan];
    const FusedLayout &lay = lays[p.layout];
    bool whole = false;
    if constexpr (!TILES_ONLY) {
      if (it.kind == 0) {
        whole = true;
        const float2 *rx = reinterpret_cast<const float2 *>(p.rx);
        float *out = reinterpret_cast<float *>(p.out);
        switch (plan.filter) {
          case F_LEGALL53: fused_pulse<F_LEGALL53>(plan, lay, rx, p.n, out, smem_batch); break;
          case F_CDF97: fused_pulse<F_CDF97>(plan, lay, rx, p.n, out, smem_batch); break;
          case F_D4: fused_pulse<F_D4>(plan, lay, rx, p.n, out, smem_batch); break;
          default: break;
        }
      }
    }
    if (!whole && it.kind == 1)
      tile_item<TILES_ONLY>(plan, lay, p, it, scratch, reinterpret_cast<float *>(smem_batch));
    if (threadIdx.x == 0) slot[k] = ahead;
    __syncthreads();
    i = __builtin_amdgcn_readfirstlane(slot[k]);
  }
}

// Work counters of a batch's persistent launches, cleared by a kernel (a
// node that graph replays reproduce faithfully) rather than a memset.
__global__ void batch_reset(int *counters, int n) {
  if (blockIdx.x == 0 && (int)threadIdx.x < n) counters[threadIdx.x] = 0;
}

// ===========================================================================
// Lifting only: pyramid d_1 | ... | d_J | c_J written to HBM.
// LDS holds the current approximation (odd levels at [0, N/2), even levels
// at [N/2, 3N/4)).  The pulse is read and the pyramid written once, with
// streaming (non-temporal) stores.
// ===========================================================================
// Threads per workgroup (measured: 512 for the complex64 filters; 256 for
// the shorter int16 pulses, where more pulses in flight pay more).
template <int F> struct LiftCfg { static constexpr int kThreads = 512; };
template <> struct LiftCfg<F_LEGALL53_INT> { static constexpr int kThreads = 256; };

typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef int i32x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ void store_stream(float2 *p, float2 v) {
  __builtin_nontemporal_store(f32x2_t{v.x, v.y}, reinterpret_cast<f32x2_t *>(p));
}
__device__ __forceinline__ void store_stream(int2 *p, int2 v) {
  __builtin_nontemporal_store(i32x2_t{v.x, v.y}, reinterpret_cast<i32x2_t *>(p));
}

// Level-1 pair (samples i, i+1; i even, both < n) of an int16 I/Q pulse with
// one 8-byte load: measured much faster than two 4-byte loads per lane.
typedef short i16x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void rx_pair(const short2 *rx, int i, int2 &e, int2 &o) {
  const i16x4_t v = *reinterpret_cast<const i16x4_t *>(rx + i);
  e = make_int2(v[0], v[1]);
  o = make_int2(v[2], v[3]);
}

template <int F>
__global__ __launch_bounds__(LiftCfg<F>::kThreads) void lift_many(
    int J, int N, const void *__restrict__ rx_all, long long n, long long rx_stride,
    void *__restrict__ pyr_all) {
  using V = typename ElemOf<F>::T;
  using RxT = typename RxOf<F>::T;
  constexpr bool OB = YLift<F>::kOddBefore;
  extern __shared__ __align__(16) char smem_lift[];
  V *sm = reinterpret_cast<V *>(smem_lift);
  const long long pulse = blockIdx.x;
  const RxT *rx = reinterpret_cast<const RxT *>(rx_all) + pulse * rx_stride;
  V *pyr = reinterpret_cast<V *>(pyr_all) + pulse * (long long)N;
  const int ni = (int)n;                              // n <= N
  // int16 pulses: pair loads when the pulse is unpadded and 8-byte aligned
  // (decided once per pulse, so neither loader branches per load)
  const bool pair_loads = F == F_LEGALL53_INT && ni == N &&
                          (reinterpret_cast<uintptr_t>(rx) % (2 * sizeof(RxT))) == 0;
  for (int l = 1; l <= J; ++l) {
    const int np = N >> l;
    V *dg = pyr + (N - (N >> (l - 1)));               // d_l
    // c_l goes to LDS (levels < J) or to the pyramid (level J); the two
    // store lambdas keep each pointer's address space known to the compiler
    V *cs = sm + ((l & 1) ? 0 : (N >> 1));
    V *cg = pyr + (N - np);
    auto store_lds = [&](int k, V c, V d) {
      cs[k] = c;
      store_stream(dg + k, d);
    };
    auto store_hbm = [&](int k, V c, V d) {
      store_stream(cg + k, c);
      store_stream(dg + k, d);
    };
    auto level = [&](auto store) {
      // (complex64 pulses keep two 8-byte loads per lane: one 16-byte load
      // per pair measured no faster)
      if constexpr (F == F_LEGALL53_INT) {
        if (l == 1 && pair_loads) {
          lift_level<F, 4>(np, [&](int kc, V &e, V &o) { rx_pair(rx, 2 * kc, e, o); }, store);
          return;
        }
      }
      if (l == 1) {
        lift_level<F, 4>(
            np,
            [&](int kc, V &e, V &o) {
              e = rx_sample(rx, ni, 2 * kc);
              o = rx_sample(rx, ni, OB ? (kc == 0 ? N - 1 : 2 * kc - 1) : 2 * kc + 1);
            },
            store);
      } else {
        const V *cin = sm + (((l - 1) & 1) ? 0 : (N >> 1));
        lift_level<F, 2>(np, [&](int kc, V &e, V &o) { pair_at<OB>(cin, kc, np, e, o); }, store);
      }
    };
    if (l == J)
      level(store_hbm);
    else
      level(store_lds);
    __syncthreads();
  }
}

// Explicit instantiations are produced by the launch helpers below.
#define SIDWT_FOR_FILTERS(X) X(F_LEGALL53) X(F_CDF97) X(F_D4) X(F_LEGALL53_INT)

}  // namespace sidwt

// ---------------------------------------------------------------------------
// Launch helpers with C++ linkage, used by the host API (sidwt_api.cpp).
// ---------------------------------------------------------------------------
namespace sidwt {

template <int F>
static hipError_t launch_tree_t(const void *in, int in_lo, int in_len, int level, int k0, int np,
                                void *outA, int loA, int lenA, void *outB, int loB, int lenB,
                                hipStream_t st) {
  using V = typename ElemOf<F>::T;
  size_t shm = 3ull * np * sizeof(V);
  if (shm > 65536) {
    hipError_t e = hipFuncSetAttribute((const void *)ref_tree_level<F>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(ref_tree_level<F>, dim3(1u << level), dim3(256), shm, st,
                     reinterpret_cast<const V *>(in), in_lo, in_len, level, k0, np,
                     reinterpret_cast<V *>(outA), loA, lenA, reinterpret_cast<V *>(outB), loB, lenB);
  return hipGetLastError();
}

hipError_t launch_tree(int filter, const void *in, int in_lo, int in_len, int level, int k0,
                       int np, void *outA, int loA, int lenA, void *outB, int loB, int lenB,
                       hipStream_t st) {
  switch (filter) {
#define X(F) \
  case F:    \
    return launch_tree_t<F>(in, in_lo, in_len, level, k0, np, outA, loA, lenA, outB, loB, lenB, st);
    SIDWT_FOR_FILTERS(X)
#undef X
  }
  return hipErrorInvalidValue;
}

// Largest grid (pulses x planes) launched with one workgroup per plane.
constexpr int kFusedSplitMaxBlocks = 256;

template <int F>
static hipError_t launch_fused_t(const PlanDesc &plan, const FusedLayout &lay, const void *rx,
                                 long long n, long long count, long long rx_stride, void *out,
                                 long long out_stride, unsigned planes, hipStream_t st) {
  // The balanced instance needs partial-sum slots after the layout: taken
  // when they fit and cost no occupancy (two workgroups per CU still fit,
  // or there are no more pulses than CUs).
  const int slots = host::fused_bal_slots(lay);
  const size_t bal_words = (size_t)lay.total + (size_t)slots * kBalSlotWords;
  const bool bal = F != F_LEGALL53_INT && slots > 0 &&
                   (bal_words <= (size_t)host::kLdsWordsTwoPerCu ||
                    (count <= 256 && bal_words <= (size_t)host::kLdsWords));
  const size_t shm = (bal ? bal_words : (size_t)lay.total) * 4;
  static std::atomic<bool> attr_set{false};  // set once per process (calls may race: both set it)
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)fused_correlate<F, false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void *)fused_correlate<F, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  // A few pulses: one workgroup per (pulse, requested plane), so the planes
  // of a pulse run on different CUs at once (their lifting repeated up to
  // each plane's level) instead of one after another in one workgroup.
  const int split = count * plan.J <= kFusedSplitMaxBlocks ? plan.J : 0;
  const unsigned grid = (unsigned)(split ? count * split : count);
  if (bal)
    hipLaunchKernelGGL((fused_correlate<F, true>), dim3(grid), dim3(kFusedThreads), shm,
                       st, plan, lay, rx, n, rx_stride, out, out_stride, planes, split);
  else
    hipLaunchKernelGGL((fused_correlate<F, false>), dim3(grid), dim3(kFusedThreads),
                       shm, st, plan, lay, rx, n, rx_stride, out, out_stride, planes, split);
  return hipGetLastError();
}

hipError_t launch_fused(const PlanDesc &plan, const FusedLayout &lay, const void *rx, long long n,
                        long long count, long long rx_stride, void *out, long long out_stride,
                        unsigned planes, hipStream_t st) {
  switch (plan.filter) {
#define X(F) \
  case F:    \
    return launch_fused_t<F>(plan, lay, rx, n, count, rx_stride, out, out_stride, planes, st);
    SIDWT_FOR_FILTERS(X)
#undef X
  }
  return hipErrorInvalidValue;
}

template <int F>
static hipError_t launch_lift_t(int J, int N, const void *rx, long long n, long long count,
                                long long rx_stride, void *pyr, hipStream_t st) {
  const size_t shm = (size_t)(N / 2 + N / 4 + 1) * sizeof(typename ElemOf<F>::T);
  static std::atomic<bool> attr_set{false};  // set once per process (calls may race: both set it)
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)lift_many<F>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(lift_many<F>, dim3((unsigned)count), dim3(LiftCfg<F>::kThreads), shm, st, J,
                     N, rx, n, rx_stride, pyr);
  return hipGetLastError();
}

hipError_t launch_lift(int filter, int J, int N, const void *rx, long long n, long long count,
                       long long rx_stride, void *pyr, hipStream_t st) {
  switch (filter) {
#define X(F) \
  case F:    \
    return launch_lift_t<F>(J, N, rx, n, count, rx_stride, pyr, st);
    SIDWT_FOR_FILTERS(X)
#undef X
  }
  return hipErrorInvalidValue;
}

hipError_t batch_set_lds(size_t bytes) {
  hipError_t e = hipFuncSetAttribute((const void *)batch_persistent<false>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void *)batch_persistent<true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  return e;
}

hipError_t batch_occupancy(bool tiles_only, size_t lds_bytes, int *blocks_per_cu) {
  if (tiles_only)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, batch_persistent<true>,
                                                        kFusedThreads, lds_bytes);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, batch_persistent<false>,
                                                      kFusedThreads, lds_bytes);
}

// Zero counters[0..n), n <= 64.
hipError_t launch_batch_reset(int *counters, int n, hipStream_t st);

// One persistent launch over items [0, nitems) with its own counter, which
// must be zero (launch_batch_reset) when the launch starts.
hipError_t launch_batch_items(bool tiles_only, const PlanDesc *plans, const FusedLayout *lays,
                              const BatchPulse *pulses, const BatchItem *items, int nitems,
                              int *counter, float2 *scratch, int grid, size_t lds_bytes,
                              hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  if (tiles_only && lds_bytes < (size_t)kBalMinLdsBytes) return hipErrorInvalidValue;
  if (tiles_only)
    hipLaunchKernelGGL(batch_persistent<true>, dim3(grid), dim3(kFusedThreads), lds_bytes, st,
                       plans, lays, pulses, items, nitems, counter, scratch);
  else
    hipLaunchKernelGGL(batch_persistent<false>, dim3(grid), dim3(kFusedThreads), lds_bytes, st,
                       plans, lays, pulses, items, nitems, counter, scratch);
  return hipGetLastError();
}

hipError_t launch_batch_reset(int *counters, int n, hipStream_t st) {
  if (n < 1 || n > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(batch_reset, dim3(1), dim3(64), 0, st, counters, n);
  return hipGetLastError();
}

// Multi-level lifting passes: npass launches, pass k over nblocks[k]
// blocks starting at blocks[k], with lds[k] bytes per workgroup.
hipError_t launch_lift_passes(const PlanDesc *plans, const BatchPulse *pulses,
                              const LiftBlock *const *blocks, const int *nblocks,
                              const size_t *lds, int npass, float2 *scratch, hipStream_t st) {
  hipError_t e = hipSuccess;
  for (int k = 0; k < npass && e == hipSuccess; ++k) {
    if (nblocks[k] == 0) continue;
    hipLaunchKernelGGL(batch_lift_blocks, dim3(nblocks[k]), dim3(256), lds[k], st, plans, pulses,
                       blocks[k], scratch);
    e = hipGetLastError();
  }
  return e;
}


}  // namespace sidwt
