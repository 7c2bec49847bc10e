// HIP kernels of libsidwt for gfx950.
//
//   ref_tree_level<F>   x-side lifting of the reference phase tree (plan).
//   fused_correlate<F>  one workgroup per pulse: y-side lifting of all J
//                       levels in LDS, each level correlated against the
//                       plan's stored phases with MFMA as soon as it exists.
//   lift_many<F>        y-side lifting only, pyramid written to HBM.
//
// Method references (Bhattacharya & Mahapatra): shift-circulant phases
// Sec. II; dual analysis lifting Sec. III; per-scale correlation eq. (15),
// (20), (20a); the Fig. 5 even/odd tree; Fig. 7 lifting of the received
// signal.
#include <type_traits>

#include "sidwt_device.hpp"

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

// ===========================================================================
// y-side lifting of one level across the workgroup (Fig. 7).  Each wave
// takes windows of 64 consecutive pairs; HL/HR edge lanes only feed their
// neighbours (shuffles), the remaining lanes own their pair.  `load(kc, e,
// o)` fetches pair kc (0 <= kc < np) of the level input; `store(k, c, d)`
// receives the owned outputs.
// ===========================================================================
template <int F, int UNROLL, class Load, class Store>
__device__ __forceinline__ void lift_level(int np, Load load, Store store) {
  using L = YLift<F>;
  using V = typename L::V;
  constexpr int OWN = 64 - L::HL - L::HR;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int nwin = (np + OWN - 1) / OWN;
  for (int w0 = wave * UNROLL; w0 < nwin; w0 += nw * UNROLL) {
    V e[UNROLL], o[UNROLL];
    int kk[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      int k = (w0 + u) * OWN - L::HL + lane;
      kk[u] = k;
      load(pos_mod(k, np), e[u], o[u]);
    }
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) L::run(e[u], o[u]);
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      int k = kk[u];
      if (lane >= L::HL && lane < 64 - L::HR && k < np && (w0 + u) < nwin) store(k, e[u], o[u]);
    }
  }
}

// Pair kc of a circular sequence of length 2*np held in `src` (LDS or
// global); for the causal D4 form the odd member is u[2k-1].
template <bool ODD_BEFORE, class V>
__device__ __forceinline__ void pair_at(const V *src, int kc, int np, V &e, V &o) {
  e = src[2 * kc];
  o = ODD_BEFORE ? src[kc == 0 ? 2 * np - 1 : 2 * kc - 1] : src[2 * kc + 1];
}

// Level-1 input from the caller's pulse: complex64, or int16 I/Q widened to
// int32.  Samples at index >= n are the zero padding up to N.
__device__ __forceinline__ float2 rx_sample(const float2 *rx, long long n, int i) {
  return (i < n) ? rx[i] : make_float2(0.f, 0.f);
}
__device__ __forceinline__ int2 rx_sample(const short2 *rx, long long n, int i) {
  if (i < n) {
    short2 s = rx[i];
    return make_int2(s.x, s.y);
  }
  return make_int2(0, 0);
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

// Stage phases r0..r0+pcc-1 of both bands as complex rows W[b][rr][v] with
// W[v] = w[v - F] (zero outside the stored support).
template <class V>
__device__ __forceinline__ void stage_weights(const PlanDesc &plan, const FusedLayout &lay, int l,
                                              int r0, int pcc, V *W) {
  const V *coef = reinterpret_cast<const V *>(plan.coef);
  const LevelDesc &ld = plan.lv[l];
  const int V0 = lay.V[l][0], V1 = lay.V[l][1];
  const int tot0 = pcc * V0, tot = tot0 + pcc * V1;
  for (int i = threadIdx.x; i < tot; i += blockDim.x) {
    const int b = i >= tot0;
    const int j = b ? i - tot0 : i;
    const int Vb = b ? V1 : V0;
    const int rr = j / Vb;
    const int t = j - rr * Vb - lay.F[l][b];
    V w;
    w.x = 0;
    w.y = 0;
    if (t >= 0 && t < ld.len[b]) w = coef[ld.off[b] + (long long)(r0 + rr) * ld.len[b] + t];
    W[i] = w;
  }
}

__device__ __forceinline__ f32x16 mfma32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// FP32 correlation of level l (32x32x2 tiles, two row tiles per wave that
// share the weight operand).
__device__ void correlate_level_f32(const PlanDesc &plan, const FusedLayout &lay, int l,
                                    float *smf, float *__restrict__ outp) {
  const int N = lay.N, P = 1 << l, L = N >> l;
  const int T = lay.T[l], logT = lay.logT[l], Ls = lay.Ls[l];
  const int Mrows = L >> logT;
  const int mtiles = (Mrows + 31) >> 5;
  const int mpairs = (mtiles + 1) >> 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  float2 *W = reinterpret_cast<float2 *>(smf + lay.w_at[l]);
  const int V0 = lay.V[l][0], V1 = lay.V[l][1];
  const int row = lane & 31;
  const int ci = lane >> 5;
  const int co = lane & 1;
  const int cc = (lane & 31) >> 1;
  const bool neg = (ci == 0) && (co == 1);
  for (int r0 = 0; r0 < P; r0 += lay.pc[l]) {
    const int pcc = min(lay.pc[l], P - r0);
    stage_weights(plan, lay, l, r0, pcc, W);
    __syncthreads();
    // P < 16: one column tile holds all (p0, r) pairs, p0 < T; otherwise
    // T = 1 and each column tile holds 16 phases.
    const int ntn = (P < 16) ? 1 : (pcc >> 4);
    const int ntiles = mpairs * ntn;
    for (int tile = wave; tile < ntiles; tile += nw) {
      const int mp = tile % mpairs;
      const int ntile = tile / mpairs;
      int r, p0;
      bool colok;
      if (P < 16) {
        r = cc & (P - 1);
        p0 = cc >> l;
        colok = p0 < T;
        if (!colok) p0 = 0;
      } else {
        r = ntile * 16 + cc;
        p0 = 0;
        colok = true;
      }
      const int p1a = mp * 64 + row;
      const int p1b = p1a + 32;
      f32x16 acc0, acc1;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        acc0[i] = 0.f;
        acc1[i] = 0.f;
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int G = lay.U[l][b] >> 2;
        const float *pl = smf + lay.region_off[l] + b * lay.band_size[l] + ci * lay.plane_stride[l];
        const float *pa = pl + (pos_mod(p1a * T + lay.lo[l][b], L) >> logT);
        const float *pb = pl + (pos_mod(p1b * T + lay.lo[l][b], L) >> logT);
        const float *wp = reinterpret_cast<const float *>(W + (b ? pcc * V0 : 0) + r * (b ? V1 : V0)) +
                          2 * (T - 1 - p0) + (ci ^ co);
        float a0[4], a1[4], w[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int off = (q & (T - 1)) * Ls + (q >> logT);
          a0[q] = pa[off];
          a1[q] = pb[off];
          w[q] = wp[2 * q];
        }
        for (int g = 0; g < G; ++g) {
          float na0[4], na1[4], nw_[4];
          const int un = (g + 1 < G) ? 4 * (g + 1) : 4 * g;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int u = un + q;
            const int off = (u & (T - 1)) * Ls + (u >> logT);
            na0[q] = pa[off];
            na1[q] = pb[off];
            nw_[q] = wp[2 * u];
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            float wq = neg ? -w[q] : w[q];
            wq = colok ? wq : 0.f;
            acc0 = mfma32(a0[q], wq, acc0);
            acc1 = mfma32(a1[q], wq, acc1);
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            a0[q] = na0[q];
            a1[q] = na1[q];
            w[q] = nw_[q];
          }
        }
      }
      if (colok) {
        // register i of lane l: row 8*(i/4) + 4*(l/32) + i%4, column l%32
#pragma unroll
        for (int h = 0; h < 2; ++h) {
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const int pp1 = mp * 64 + h * 32 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
            if (pp1 < Mrows) {
              const long long s = (long long)P * (pp1 * T + p0) + r0 + r;
              __builtin_nontemporal_store(h ? acc1[i] : acc0[i], &outp[2 * s + co]);
            }
          }
        }
      }
    }
    __syncthreads();
  }
}

// Integer correlation of level l (FP64 16x16x4 tiles, two row tiles per
// wave sharing the weight operand).
__device__ void correlate_level_int(const PlanDesc &plan, const FusedLayout &lay, int l,
                                    int *smi, long long *__restrict__ outp) {
  const int N = lay.N, P = 1 << l, L = N >> l;
  const int T = lay.T[l], logT = lay.logT[l], Ls = lay.Ls[l];
  const int Mrows = L >> logT;
  const int mtiles = (Mrows + 15) >> 4;
  const int mpairs = (mtiles + 1) >> 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int2 *W = reinterpret_cast<int2 *>(smi + lay.w_at[l]);
  const int V0 = lay.V[l][0], V1 = lay.V[l][1];
  const int row = lane & 15;
  const int kq = lane >> 4;
  const int du = kq >> 1;
  const int ci = kq & 1;
  const int co = lane & 1;
  const int cc = (lane & 15) >> 1;
  const bool neg = (ci == 0) && (co == 1);
  for (int r0 = 0; r0 < P; r0 += lay.pc[l]) {
    const int pcc = min(lay.pc[l], P - r0);
    stage_weights(plan, lay, l, r0, pcc, W);
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
        const int steps = lay.U[l][b] >> 1;
        const int *pl = smi + lay.region_off[l] + b * lay.band_size[l] + ci * lay.plane_stride[l];
        const int qa = pos_mod(p1a * T + lay.lo[l][b], L);
        const int qb = pos_mod(p1b * T + lay.lo[l][b], L);
        const int *wp = reinterpret_cast<const int *>(W + (b ? pcc * V0 : 0) + r * (b ? V1 : V0)) +
                        2 * (du - p0 + T - 1) + (ci ^ co);
        for (int st = 0; st < steps; ++st) {
          const int u = 2 * st + du;
          const int a0 = pl[poly_off(qa + u, logT, Ls)];
          const int a1 = pl[poly_off(qb + u, logT, Ls)];
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
  for (int q = k; q < lay.ext[l]; q += L) {
    const int o = poly_off(q, lay.logT[l], lay.Ls[l]);
    b0[o] = c.x;
    b0[o + ps] = c.y;
    b1[o] = d.x;
    b1[o + ps] = d.y;
  }
}

template <class V, class S>
__device__ __forceinline__ V load_elem(const S *sm, const FusedLayout &lay, int l, int q) {
  const S *b0 = sm + lay.region_off[l];
  const int o = poly_off(q, lay.logT[l], lay.Ls[l]);
  V v;
  v.x = b0[o];
  v.y = b0[o + lay.plane_stride[l]];
  return v;
}

// ===========================================================================
// Fused kernel: one workgroup per pulse.  Level 1 is lifted straight from
// HBM; every level's bands are correlated as soon as they exist, then the
// next level is lifted from c_l.  Odd and even levels live in alternating
// LDS regions so that c_l stays intact while level l+1 is written.
// ===========================================================================
template <int F>
__global__ __launch_bounds__(kFusedThreads) void fused_correlate(PlanDesc plan, FusedLayout lay,
                                                                const void *__restrict__ rx_all,
                                                                long long n, long long rx_stride,
                                                                void *__restrict__ out_all,
                                                                long long out_stride) {
  constexpr bool INT = (F == F_LEGALL53_INT);
  using V = typename ElemOf<F>::T;
  using S = typename std::conditional<INT, int, float>::type;
  using RxT = typename RxOf<F>::T;
  using OutT = typename RxOf<F>::Out;
  constexpr bool OB = YLift<F>::kOddBefore;
  extern __shared__ __align__(16) char smem_fused[];
  S *sm = reinterpret_cast<S *>(smem_fused);
  const long long pulse = blockIdx.x;
  const RxT *rx = reinterpret_cast<const RxT *>(rx_all) + pulse * rx_stride;
  OutT *out = reinterpret_cast<OutT *>(out_all) + pulse * out_stride * 2;
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

  for (int l = 1; l <= lay.J; ++l) {
    if constexpr (INT) {
      correlate_level_int(plan, lay, l, sm, out + 2LL * (l - 1) * N);
    } else {
      correlate_level_f32(plan, lay, l, sm, out + 2LL * (l - 1) * N);
    }
    if (l < lay.J) {
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

// ===========================================================================
// Lifting only: pyramid d_1 | ... | d_J | c_J written to HBM.
// LDS holds the current approximation (odd levels at [0, N/2), even levels
// at [N/2, 3N/4)).
// ===========================================================================
template <int F>
__global__ __launch_bounds__(256) void lift_many(int J, int N, const void *__restrict__ rx_all,
                                                 long long n, long long rx_stride,
                                                 void *__restrict__ pyr_all) {
  using V = typename ElemOf<F>::T;
  using RxT = typename RxOf<F>::T;
  constexpr bool OB = YLift<F>::kOddBefore;
  extern __shared__ __align__(16) char smem_lift[];
  V *sm = reinterpret_cast<V *>(smem_lift);
  const long long pulse = blockIdx.x;
  const RxT *rx = reinterpret_cast<const RxT *>(rx_all) + pulse * rx_stride;
  V *pyr = reinterpret_cast<V *>(pyr_all) + pulse * (long long)N;
  for (int l = 1; l <= J; ++l) {
    const int np = N >> l;
    V *dg = pyr + (N - (N >> (l - 1)));               // d_l
    V *cl = (l == J) ? pyr + (N - np) : sm + ((l & 1) ? 0 : (N >> 1));
    if (l == 1) {
      lift_level<F, 4>(
          np,
          [&](int kc, V &e, V &o) {
            e = rx_sample(rx, n, 2 * kc);
            o = rx_sample(rx, n, OB ? (kc == 0 ? N - 1 : 2 * kc - 1) : 2 * kc + 1);
          },
          [&](int k, V c, V d) {
            cl[k] = c;
            dg[k] = d;
          });
    } else {
      const V *cin = sm + (((l - 1) & 1) ? 0 : (N >> 1));
      lift_level<F, 2>(
          np, [&](int kc, V &e, V &o) { pair_at<OB>(cin, kc, np, e, o); },
          [&](int k, V c, V d) {
            cl[k] = c;
            dg[k] = d;
          });
    }
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

template <int F>
static hipError_t launch_fused_t(const PlanDesc &plan, const FusedLayout &lay, const void *rx,
                                 long long n, long long count, long long rx_stride, void *out,
                                 long long out_stride, hipStream_t st) {
  size_t shm = (size_t)lay.total * 4;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)fused_correlate<F>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(fused_correlate<F>, dim3((unsigned)count), dim3(kFusedThreads), shm, st, plan, lay, rx,
                     n, rx_stride, out, out_stride);
  return hipGetLastError();
}

hipError_t launch_fused(const PlanDesc &plan, const FusedLayout &lay, const void *rx, long long n,
                        long long count, long long rx_stride, void *out, long long out_stride,
                        hipStream_t st) {
  switch (plan.filter) {
#define X(F) \
  case F:    \
    return launch_fused_t<F>(plan, lay, rx, n, count, rx_stride, out, out_stride, st);
    SIDWT_FOR_FILTERS(X)
#undef X
  }
  return hipErrorInvalidValue;
}

template <int F>
static hipError_t launch_lift_t(int J, int N, const void *rx, long long n, long long count,
                                long long rx_stride, void *pyr, hipStream_t st) {
  size_t shm = (size_t)(N / 2 + N / 4 + 1) * 8;
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void *)lift_many<F>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(lift_many<F>, dim3((unsigned)count), dim3(256), shm, st, J, N, rx, n,
                     rx_stride, pyr);
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

}  // namespace sidwt
