// Reference banks (C ABI part of libsidwt; declarations in include/sidwt.h).
//
// A bank holds E references (ascending length) of one float filter with a
// phase pyramid of Jmax levels each.  At creation every stored phase
// coefficient w of reference e and level l is scaled by a power of two s
// (the largest |w| of that reference and level maps below 2^14) and split
// into 16-bit hi = h(w s) and lo = h(w s - hi), in two column variants
// (re-out: (w.re, w.im), im-out: (-w.im, w.re)) so the MFMA weight operand
// needs no sign handling.  The split weights of a level are stored per
// column tile of 16 (reference, phase) pairs as panels in the order the MFMA
// lanes read them.  A request lifts its pulse into an HBM scratch pyramid and
// runs one GEMM work item per (level, up to 256 lags, up to 16 tiles).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstdint>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "../../include/sidwt.h"
#include "sidwt_bank.hpp"
#include "sidwt_host.hpp"

namespace sidwt {
hipError_t launch_bank(bool bf16, bool deep, const BankSeg *segs, const int2 *items, int nitems,
                       const BankTile *tiles, const int *tile_base, const BankRefLevel *rl,
                       int Jmax, const int *lo_lb, const unsigned *wts, const float2 *scratch,
                       int Wmax, hipStream_t st);
hipError_t launch_lift_passes(const PlanDesc *plans, const BatchPulse *pulses,
                              const LiftBlock *const *blocks, const int *nblocks,
                              const size_t *lds, int npass, float2 *scratch, hipStream_t st);
}  // namespace sidwt

extern "C++" const sidwt::PlanDesc *sidwt_plan_desc(const sidwt_plan *p);
// One-shot uneven batch over plan descriptors (sidwt_batch.cpp).
extern "C++" int sidwt_batch_oneshot(const sidwt::PlanDesc *const *descs, const int64_t *n,
                                     const void *const *rx, void *const *out, int count,
                                     hipStream_t st);

using namespace sidwt;
using namespace sidwt::host;

namespace {

// Levels lifted per pass of the request pyramids (one launch per pass:
// blocks of input samples with halos, every level of the pass written).
constexpr int kBankLiftDepth = 4;
// Panel steps (both bands, summed over an item's tiles) an item should run
// per data window, and the most tile groups one item may take.
constexpr double kBankItemSteps = 256.0;
constexpr int kBankMaxGroups = 16;
constexpr int kBankXcdRun = 16;     // consecutive items of a class kept on one XCD
// Levels from this one on (short panels: items bound by their latency and
// plane writes) run on the deep kernel, after the others, in a launch of
// their own -- when the other levels' items alone fill the chip for several
// rounds (kBankSplitItems: 256 CUs x 2 workgroups x 4).  A smaller call
// (serving at light load) keeps one launch of the general kernel, where
// the deep levels' items run beside the others instead of after them.
constexpr int kBankDeepLevel = 4;
constexpr long long kBankSplitItems = 2048;

int map_err(hipError_t e, const char *what = nullptr) {
  if (e == hipSuccess) return SIDWT_OK;
  if (what && std::getenv("SIDWT_DEBUG"))
    std::fprintf(stderr, "sidwt bank: %s: %s\n", what, hipGetErrorString(e));
  if (e == hipErrorOutOfMemory) return SIDWT_E_NOMEM;
  return SIDWT_E_DEVICE;
}

// 16-bit encodings (round to nearest even).
unsigned short to_f16(float x) {
  _Float16 h = (_Float16)x;
  unsigned short u;
  std::memcpy(&u, &h, 2);
  return u;
}
float from_f16(unsigned short u) {
  _Float16 h;
  std::memcpy(&h, &u, 2);
  return (float)h;
}
unsigned short to_bf16(float x) {
  unsigned u;
  std::memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);  // inf / nan
  const unsigned rounding = 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)((u + rounding) >> 16);
}
float from_bf16(unsigned short h) {
  unsigned u = (unsigned)h << 16;
  float x;
  std::memcpy(&x, &u, 4);
  return x;
}

template <class T>
int grow(T **p, size_t *cap, size_t need) {
  need = std::max<size_t>(need, 1);
  if (*cap >= need) return SIDWT_OK;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  *cap = 0;
  hipError_t e = hipMalloc(p, need * sizeof(T));
  if (e != hipSuccess) return map_err(e, "hipMalloc");
  *cap = need;
  return SIDWT_OK;
}

}  // namespace

// Per-call device buffers: request and item descriptors, lifting chunks and
// the scratch pyramids.  One workspace serves one stream at a time.
struct sidwt_bank_ws {
  BankSeg *d_segs = nullptr;
  size_t c_segs = 0;
  int2 *d_items = nullptr;
  size_t c_items = 0;
  BatchPulse *d_pulses = nullptr;
  size_t c_pulses = 0;
  LiftBlock *d_blocks = nullptr;
  size_t c_blocks = 0;
  float2 *d_scratch = nullptr;
  size_t c_scratch = 0;
  bool timing = false;
  bool timed = false;                // the last call recorded its events
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  // Pinned host staging of a call's four descriptor arrays (so their
  // uploads are asynchronous); up_done follows the last upload, and the next
  // call waits for it before rewriting the staging buffer.
  char *h_stage = nullptr;
  size_t c_stage = 0;
  hipEvent_t up_done = nullptr;
};

struct sidwt_bank {
  int filter = 0, Jmax = 0, E = 0, precision = 1;
  std::vector<int64_t> m;
  std::vector<sidwt_plan *> plans;   // one per reference (FP32 path, tests)
  PlanDesc desc0;                    // windows are shared by all references
  std::vector<BankRefLevel> rl;      // [e * (Jmax + 1) + l]
  std::vector<int> lo_lb;            // [2 l + b]
  std::vector<BankTile> tiles;       // [tile_base[l] + T]
  std::vector<long long> steps_pre;  // prefix sums of steps (both bands), [tile_base[l] + T + l]
  std::vector<int> tile_base;        // [l], l = 0..Jmax
  int Umax = 0;        // longest tile window (lag offsets), all levels
  int UmaxDeep = 0;    // the same from level kBankDeepLevel on
  long long weight_words = 0;
  // device
  unsigned *d_w = nullptr;
  BankTile *d_tiles = nullptr;
  int *d_tile_base = nullptr;
  BankRefLevel *d_rl = nullptr;
  int *d_lo = nullptr;
  PlanDesc *d_plan = nullptr;
  sidwt_bank_ws *ws = nullptr;      // default workspace
};

namespace {

// FP32 bank: every (request, eligible reference) pair as one pulse of a
// one-shot uneven batch, with the reference's plan descriptor cut to the
// request's J (its phases of levels 1..J are the same for any J <= Jmax).
int correlate_fp32(sidwt_bank *bk, const void *const *rx, const int64_t *n, const int *J,
                   void *const *out, int count, hipStream_t st) {
  std::map<std::pair<int, int>, int> at;   // (reference, J) -> descs index
  std::vector<std::pair<int, int>> key;    // per pulse
  std::vector<int64_t> ns;
  std::vector<const void *> rxs;
  std::vector<void *> outs;
  for (int i = 0; i < count; ++i) {
    if (!rx[i] || n[i] < 1 || J[i] < 1 || J[i] > bk->Jmax) return SIDWT_E_INVAL;
    const int64_t N = transform_length(n[i], J[i]);
    if ((N >> J[i]) < 2) return SIDWT_E_INVAL;
    const int E = (int)sidwt_bank_eligible(bk, n[i]);
    // (no eligible reference: an empty output, whose pointer may be NULL)
    if (E > 0 && (!out[i] || reinterpret_cast<uintptr_t>(out[i]) % 16)) return SIDWT_E_INVAL;
    for (int e = 0; e < E; ++e) {
      const std::pair<int, int> k(e, J[i]);
      if (!at.count(k)) at.emplace(k, (int)at.size());
      key.push_back(k);
      ns.push_back(n[i]);
      rxs.push_back(rx[i]);
      outs.push_back(static_cast<char *>(out[i]) + (size_t)e * J[i] * N * 8);
    }
  }
  if (key.empty()) return SIDWT_OK;
  if (key.size() > 0x7fffffff) return SIDWT_E_SIZE;
  std::vector<PlanDesc> descs(at.size());
  for (const auto &kv : at) {
    descs[kv.second] = *sidwt_plan_desc(bk->plans[kv.first.first]);
    descs[kv.second].J = kv.first.second;
  }
  std::vector<const PlanDesc *> dp(key.size());
  for (size_t q = 0; q < key.size(); ++q) dp[q] = &descs[at[key[q]]];
  return sidwt_batch_oneshot(dp.data(), ns.data(), rxs.data(), outs.data(), (int)key.size(), st);
}

}  // namespace

extern "C" {

int sidwt_bank_create(int filter, int Jmax, const void *const *refs, const int64_t *m, int count,
                      int precision, sidwt_bank **out) {
  if (!refs || !m || !out || count < 1 || Jmax < 1 || Jmax > SIDWT_MAX_LEVELS ||
      (precision != SIDWT_BANK_FP32 && precision != SIDWT_BANK_FP16 &&
       precision != SIDWT_BANK_BF16))
    return SIDWT_E_INVAL;
  if (filter != SIDWT_LEGALL53 && filter != SIDWT_CDF97 && filter != SIDWT_D4_CAUSAL)
    return filter == SIDWT_LEGALL53_INT ? SIDWT_E_UNSUPPORTED : SIDWT_E_INVAL;
  for (int e = 0; e < count; ++e) {
    if (!refs[e] || m[e] < 1) return SIDWT_E_INVAL;
    if (e > 0 && m[e] < m[e - 1]) return SIDWT_E_INVAL;  // ascending length
  }
  sidwt_bank *bk = new (std::nothrow) sidwt_bank();
  if (!bk) return SIDWT_E_NOMEM;
  bk->filter = filter;
  bk->Jmax = Jmax;
  bk->E = count;
  bk->precision = precision;
  const bool bf16 = precision == SIDWT_BANK_BF16;
  const bool fp32 = precision == SIDWT_BANK_FP32;  // plans only: no split weights
  int rc = SIDWT_OK;
  // split[e][l][b]: 4 arrays (hi re-out, hi im-out, lo re-out, lo im-out) of
  // len words for every phase r, as [r][a][u]
  std::vector<std::vector<unsigned>> split((size_t)count * (Jmax + 1) * 2);
  bk->rl.assign((size_t)count * (Jmax + 1), BankRefLevel{});
  for (int e = 0; e < count && !rc; ++e) {
    sidwt_plan *p = nullptr;
    rc = sidwt_plan_create(filter, Jmax, refs[e], m[e], &p);
    if (rc) break;
    bk->plans.push_back(p);
    bk->m.push_back(m[e]);
    const PlanDesc &d = *sidwt_plan_desc(p);
    if (e == 0) bk->desc0 = d;
    if (fp32) continue;
    long long total = 0;
    for (int l = 1; l <= Jmax; ++l) total += ((long long)d.lv[l].len[0] + d.lv[l].len[1]) << l;
    std::vector<float> coef(2 * (size_t)total);
    hipError_t he = hipMemcpy(coef.data(), d.coef, coef.size() * 4, hipMemcpyDeviceToHost);
    if (he != hipSuccess) { rc = map_err(he, "hipMemcpy (phases)"); break; }
    for (int l = 1; l <= Jmax; ++l) {
      float mx = 0.f;
      for (int b = 0; b < 2; ++b) {
        const size_t o = 2 * (size_t)d.lv[l].off[b], cnt = 2 * ((size_t)d.lv[l].len[b] << l);
        for (size_t i = 0; i < cnt; ++i) mx = std::max(mx, std::fabs(coef[o + i]));
      }
      int ex = 0;
      std::frexp(mx, &ex);
      const float s = mx > 0.f ? std::ldexp(1.f, 14 - ex) : 1.f;
      BankRefLevel &R = bk->rl[(size_t)e * (Jmax + 1) + l];
      R.inv_scale = 1.f / s;
      for (int b = 0; b < 2; ++b) {
        const int len = d.lv[l].len[b];
        R.len[b] = len;
        std::vector<unsigned> &w = split[((size_t)e * (Jmax + 1) + l) * 2 + b];
        w.assign(((size_t)4 * len) << l, 0u);
        for (int r = 0; r < (1 << l); ++r)
          for (int u = 0; u < len; ++u) {
            const size_t c = 2 * ((size_t)d.lv[l].off[b] + (size_t)r * len + u);
            const float wr = coef[c] * s, wi = coef[c + 1] * s;
            // column variants: re-out (wr, wi), im-out (-wi, wr); hi then lo
            const float v[2][2] = {{wr, wi}, {-wi, wr}};
            for (int co = 0; co < 2; ++co) {
              unsigned short h0, h1, l0, l1;
              if (bf16) {
                h0 = to_bf16(v[co][0]);
                h1 = to_bf16(v[co][1]);
                l0 = to_bf16(v[co][0] - from_bf16(h0));
                l1 = to_bf16(v[co][1] - from_bf16(h1));
              } else {
                h0 = to_f16(v[co][0]);
                h1 = to_f16(v[co][1]);
                l0 = to_f16(v[co][0] - from_f16(h0));
                l1 = to_f16(v[co][1] - from_f16(h1));
              }
              w[((size_t)r * 4 + co) * len + u] = (unsigned)h0 | ((unsigned)h1 << 16);
              w[((size_t)r * 4 + 2 + co) * len + u] = (unsigned)l0 | ((unsigned)l1 << 16);
            }
          }
      }
    }
  }
  // Panels: per level, per tile of 16 pairs c = e * 2^l + r, per band.
  std::vector<unsigned> words;
  if (!rc && !fp32) {
    bk->tile_base.assign(Jmax + 1, 0);
    for (int l = 1; l <= Jmax; ++l) {
      bk->tile_base[l] = (int)bk->tiles.size();
      const int P = 1 << l;
      const long long pairs = (long long)count * P;
      for (long long T = 0; T * kBankTilePairs < pairs; ++T) {
        BankTile tile{};
        for (int b = 0; b < 2; ++b) {
          int U = 0;
          for (int pl = 0; pl < kBankTilePairs; ++pl) {
            const long long c = T * kBankTilePairs + pl;
            if (c < pairs) U = std::max(U, bk->rl[(size_t)(c >> l) * (Jmax + 1) + l].len[b]);
          }
          const int steps = (U + 7) / 8;
          tile.steps[b] = steps;
          tile.off[b] = (long long)words.size();
          bk->Umax = std::max(bk->Umax, 8 * steps);
          if (l >= kBankDeepLevel) bk->UmaxDeep = std::max(bk->UmaxDeep, 8 * steps);
          words.resize(words.size() + (size_t)steps * kBankStepWords, 0u);
          unsigned *panel = words.data() + tile.off[b];
          for (int st = 0; st < steps; ++st)
            for (int hl = 0; hl < 2; ++hl)
              for (int lane = 0; lane < 64; ++lane) {
                const int col = lane & 31, g = lane >> 5;
                const long long c = T * kBankTilePairs + (col >> 1);
                if (c >= pairs) continue;
                const int e = (int)(c >> l), r = (int)(c & (P - 1));
                const int len = bk->rl[(size_t)e * (Jmax + 1) + l].len[b];
                const std::vector<unsigned> &w = split[((size_t)e * (Jmax + 1) + l) * 2 + b];
                const int a = 2 * hl + (col & 1);
                for (int k = 0; k < 4; ++k) {
                  const int u = 8 * st + 4 * g + k;
                  if (u < len)
                    panel[((size_t)(st * 2 + hl) * 64 + lane) * 4 + k] =
                        w[((size_t)r * 4 + a) * len + u];
                }
              }
        }
        bk->tiles.push_back(tile);
      }
    }
  }
  if (!rc && !fp32) {
    // per level: steps_pre[tile_base[l] + l - 1 + T] = steps of tiles [0, T)
    bk->steps_pre.clear();
    for (int l = 1; l <= Jmax; ++l) {
      const int t1 = l < Jmax ? bk->tile_base[l + 1] : (int)bk->tiles.size();
      long long acc = 0;
      bk->steps_pre.push_back(0);
      for (int T = bk->tile_base[l]; T < t1; ++T) {
        acc += bk->tiles[T].steps[0] + bk->tiles[T].steps[1];
        bk->steps_pre.push_back(acc);
      }
    }
  }
  if (!rc && !fp32) {
    bk->lo_lb.assign(2 * (Jmax + 1), 0);
    for (int l = 1; l <= Jmax; ++l)
      for (int b = 0; b < 2; ++b) bk->lo_lb[2 * l + b] = bk->desc0.lv[l].lo[b];
    bk->weight_words = (long long)words.size();
    hipError_t he = hipMalloc(&bk->d_w, std::max<size_t>(1, words.size()) * 4);
    if (he == hipSuccess && !words.empty())
      he = hipMemcpy(bk->d_w, words.data(), words.size() * 4, hipMemcpyHostToDevice);
    if (he == hipSuccess) he = hipMalloc(&bk->d_tiles, bk->tiles.size() * sizeof(BankTile));
    if (he == hipSuccess)
      he = hipMemcpy(bk->d_tiles, bk->tiles.data(), bk->tiles.size() * sizeof(BankTile),
                     hipMemcpyHostToDevice);
    if (he == hipSuccess) he = hipMalloc(&bk->d_tile_base, bk->tile_base.size() * sizeof(int));
    if (he == hipSuccess)
      he = hipMemcpy(bk->d_tile_base, bk->tile_base.data(), bk->tile_base.size() * sizeof(int),
                     hipMemcpyHostToDevice);
    if (he == hipSuccess) he = hipMalloc(&bk->d_rl, bk->rl.size() * sizeof(BankRefLevel));
    if (he == hipSuccess)
      he = hipMemcpy(bk->d_rl, bk->rl.data(), bk->rl.size() * sizeof(BankRefLevel),
                     hipMemcpyHostToDevice);
    if (he == hipSuccess) he = hipMalloc(&bk->d_lo, bk->lo_lb.size() * sizeof(int));
    if (he == hipSuccess)
      he = hipMemcpy(bk->d_lo, bk->lo_lb.data(), bk->lo_lb.size() * sizeof(int),
                     hipMemcpyHostToDevice);
    if (he == hipSuccess) he = hipMalloc(&bk->d_plan, sizeof(PlanDesc));
    if (he == hipSuccess)
      he = hipMemcpy(bk->d_plan, &bk->desc0, sizeof(PlanDesc), hipMemcpyHostToDevice);
    rc = map_err(he, "bank upload");
  }
  if (rc) {
    sidwt_bank_free(bk);
    return rc;
  }
  *out = bk;
  return SIDWT_OK;
}

void sidwt_bank_free(sidwt_bank *bk) {
  if (!bk) return;
  (void)hipDeviceSynchronize();
  for (sidwt_plan *p : bk->plans) sidwt_free(p);
  (void)hipFree(bk->d_w);
  (void)hipFree(bk->d_tiles);
  (void)hipFree(bk->d_tile_base);
  (void)hipFree(bk->d_rl);
  (void)hipFree(bk->d_lo);
  (void)hipFree(bk->d_plan);
  sidwt_bank_ws_free(bk->ws);
  delete bk;
}

int sidwt_bank_ws_create(const sidwt_bank *bk, sidwt_bank_ws **out) {
  if (!bk || !out) return SIDWT_E_INVAL;
  sidwt_bank_ws *w = new (std::nothrow) sidwt_bank_ws();
  if (!w) return SIDWT_E_NOMEM;
  *out = w;
  return SIDWT_OK;
}

void sidwt_bank_ws_free(sidwt_bank_ws *w) {
  if (!w) return;
  (void)hipDeviceSynchronize();
  if (w->h_stage) (void)hipHostFree(w->h_stage);
  if (w->up_done) (void)hipEventDestroy(w->up_done);
  (void)hipFree(w->d_segs);
  (void)hipFree(w->d_items);
  (void)hipFree(w->d_pulses);
  (void)hipFree(w->d_blocks);
  (void)hipFree(w->d_scratch);
  for (hipEvent_t e : w->ev)
    if (e) (void)hipEventDestroy(e);
  delete w;
}

int sidwt_bank_ws_timing(sidwt_bank_ws *ws, int on) {
  if (!ws) return SIDWT_E_INVAL;
  if (on)
    for (hipEvent_t &e : ws->ev)
      if (!e) {
        hipError_t he = hipEventCreate(&e);
        if (he != hipSuccess) {
          e = nullptr;
          return map_err(he, "hipEventCreate");
        }
      }
  ws->timing = on != 0;
  ws->timed = false;
  return SIDWT_OK;
}

int sidwt_bank_ws_times(sidwt_bank_ws *ws, float *lift_ms, float *gemm_ms) {
  if (!ws || !lift_ms || !gemm_ms) return SIDWT_E_INVAL;
  if (!ws->timed) return SIDWT_E_INVAL;
  hipError_t e = hipEventSynchronize(ws->ev[2]);
  if (e == hipSuccess) e = hipEventElapsedTime(lift_ms, ws->ev[0], ws->ev[1]);
  if (e == hipSuccess) e = hipEventElapsedTime(gemm_ms, ws->ev[1], ws->ev[2]);
  return map_err(e, "event timing");
}

int64_t sidwt_bank_scratch_bytes(const sidwt_bank *bk, int64_t n, int J) {
  if (!bk || n < 1 || J < 1 || J > bk->Jmax) return -1;
  const int64_t pyramid = 2 * transform_length(n, J) * (int64_t)sizeof(float2);
  // FP32: the one-shot batch may hold one pyramid per eligible reference
  return bk->precision == SIDWT_BANK_FP32 ? sidwt_bank_eligible(bk, n) * pyramid : pyramid;
}

int64_t sidwt_bank_eligible(const sidwt_bank *bk, int64_t n) {
  if (!bk || n < 1) return -1;
  return (int64_t)(std::upper_bound(bk->m.begin(), bk->m.end(), n) - bk->m.begin());
}

int64_t sidwt_bank_out_len(const sidwt_bank *bk, int64_t n, int J) {
  if (!bk || n < 1 || J < 1 || J > bk->Jmax) return -1;
  return sidwt_bank_eligible(bk, n) * J * transform_length(n, J);
}

const sidwt_plan *sidwt_bank_plan(const sidwt_bank *bk, int e) {
  if (!bk || e < 0 || e >= bk->E) return nullptr;
  return bk->plans[e];
}

int sidwt_bank_info(const sidwt_bank *bk, int64_t *v, int nv) {
  if (!bk || !v || nv < 1) return SIDWT_E_INVAL;
  const int64_t vals[] = {bk->E, bk->Jmax, bk->precision, bk->weight_words * 4, bk->Umax};
  const int k = (int)(sizeof(vals) / sizeof(vals[0]));
  for (int i = 0; i < nv; ++i) v[i] = i < k ? vals[i] : 0;
  return SIDWT_OK;
}

int sidwt_bank_correlate(sidwt_bank *bk, const void *const *rx, const int64_t *n, const int *J,
                         void *const *out, int count, void *hip_stream) {
  if (!bk || count < 0) return SIDWT_E_INVAL;
  if (count == 0) return SIDWT_OK;
  if (!bk->ws) {
    int rc = sidwt_bank_ws_create(bk, &bk->ws);
    if (rc) return rc;
  }
  return sidwt_bank_correlate_ws(bk, bk->ws, rx, n, J, out, count, hip_stream);
}

int sidwt_bank_correlate_ws(sidwt_bank *bk, sidwt_bank_ws *ws, const void *const *rx,
                            const int64_t *n, const int *J, void *const *out, int count,
                            void *hip_stream) {
  if (!bk || !ws || count < 0) return SIDWT_E_INVAL;
  if (count == 0) return SIDWT_OK;
  if (!rx || !n || !J || !out) return SIDWT_E_INVAL;
  if (bk->precision == SIDWT_BANK_FP32)
    return correlate_fp32(bk, rx, n, J, out, count, static_cast<hipStream_t>(hip_stream));
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  std::vector<BatchPulse> pulses(count);
  std::vector<BankSeg> segs;
  std::vector<long long> cost;       // per item of the segment
  std::vector<std::vector<LiftBlock>> per_pass(kMaxLevels + 1);
  std::vector<size_t> pass_lds(kMaxLevels + 1, 0);
  long long scratch = 0;
  for (int i = 0; i < count; ++i) {
    if (!rx[i] || n[i] < 1 || J[i] < 1 || J[i] > bk->Jmax) return SIDWT_E_INVAL;
    const int64_t N = transform_length(n[i], J[i]);
    if ((N >> J[i]) < 2) return SIDWT_E_INVAL;
    if (N > (int64_t(1) << 26)) return SIDWT_E_SIZE;
    const int E = (int)sidwt_bank_eligible(bk, n[i]);
    // (no eligible reference: an empty output, whose pointer may be NULL)
    if (E > 0 && (!out[i] || (reinterpret_cast<uintptr_t>(out[i]) & 15))) return SIDWT_E_INVAL;
    BatchPulse &p = pulses[i];
    p = BatchPulse{};
    p.rx = rx[i];
    p.n = n[i];
    p.N = (int)N;
    p.J = J[i];
    p.plan = 0;
    p.scratch = scratch;
    scratch += 2 * N;
    if (E == 0) continue;
    for (int k = 0; k * kBankLiftDepth < J[i]; ++k) {
      const int l0 = k * kBankLiftDepth + 1, l1 = std::min(J[i], (k + 1) * kBankLiftDepth);
      const int nb = lift_block_count((int)N, l0, l1);
      for (int blk = 0; blk < nb; ++blk) per_pass[k].push_back(LiftBlock{i, l0, l1, blk});
      pass_lds[k] = std::max(pass_lds[k], (size_t)lift_block_lds((int)N, l0, l1) * sizeof(float2));
    }
    for (int l = 1; l <= J[i]; ++l) {
      const int L = (int)(N >> l), P = 1 << l;
      BankSeg sg{};
      sg.out = out[i];
      sg.scratch = scratch - 2 * N;
      sg.N = (int)N;
      sg.J = J[i];
      sg.E = E;
      sg.level = l;
      sg.L = L;
      sg.ntiles = (E * P + kBankTilePairs - 1) / kBankTilePairs;
      sg.nblocks = (L + 255) / 256;
      const int last = L - 256 * (sg.nblocks - 1);
      const int per_last = bank_tiles_per_item(last);
      // Levels 1 and 2 have the longest panels: their full blocks take the
      // wave shape with half the panel loads per MFMA.
      sg.wide = l <= 2;
      // Short panels (high levels): several tile groups per item, so that
      // an item runs about kBankItemSteps panel steps per tile column over
      // one data window (its load, max reduction and hi/lo split).
      const long long *pre = bk->steps_pre.data() + bk->tile_base[l] + (l - 1);
      const long long st = pre[sg.ntiles];   // steps (both bands) of the segment's tiles
      const double per_tile = (double)st / std::max(1, sg.ntiles);
      int gm = 1;
      while (gm < kBankMaxGroups && 4.0 * gm * per_tile < kBankItemSteps) gm *= 2;
      sg.gmul = gm;
      sg.g_full = ((sg.ntiles + 3) / 4 + gm - 1) / gm;
      sg.g_last = ((sg.ntiles + per_last - 1) / per_last + gm - 1) / gm;
      segs.push_back(sg);
      // cost of one item: rows x steps of its tiles (mean over the level's tiles)
      cost.push_back(std::min(L, 256) * st / std::max(1, sg.nblocks > 1 ? sg.g_full : sg.g_last) +
                     std::min(L, 256) * 8);
    }
  }
  // Segments with the costliest items first (longest-processing-time order).
  std::vector<int> order(segs.size());
  for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<BankSeg> sorted(segs.size());
  long long nitems = 0;
  for (size_t k = 0; k < order.size(); ++k) {
    sorted[k] = segs[order[k]];
    sorted[k].item0 = nitems;
    nitems += (long long)(sorted[k].nblocks - 1) * sorted[k].g_full + sorted[k].g_last;
  }
  if (nitems > (1LL << 31) - 1) return SIDWT_E_SIZE;
  // Items (segment, index within it): classes of half an octave of the
  // item's own cost (rows x panel steps of its tiles), costliest first;
  // within a class by level, then tile group, then segment, then row block,
  // so the items of one level and tile group of different requests are
  // neighbours.  Workgroups go to the eight XCDs round-robin (position p to
  // XCD p mod 8), so each class is then laid out in runs of kBankXcdRun
  // consecutive list items, run r going to the XCD of the class's (r mod
  // 8)-th position (the class's last 8 kBankXcdRun - 1 items or fewer keep
  // their order): the items of a run
  // mostly share a tile group's weight panels (a deep level's panels are
  // read by every request, whose few rows reuse them little) and find them
  // in that XCD's L2, while every XCD still draws from the whole class.
  // When the call is split, the items of levels below kBankDeepLevel and
  // those from it on form two such lists, one per launch (the general
  // kernel, then the deep one); otherwise one list for the general kernel.
  std::vector<std::vector<int>> seg_of_level(kMaxLevels + 1);
  for (size_t k = 0; k < sorted.size(); ++k) seg_of_level[sorted[k].level].push_back((int)k);
  // The items of levels [l_lo, l_hi], ordered and placed as described above.
  auto order_levels = [&](int l_lo, int l_hi, std::vector<int2> &items) {
    std::vector<std::vector<int2>> bucket(130);
    for (int l = l_lo; l <= l_hi; ++l) {
      if (seg_of_level[l].empty()) continue;
      const long long *pre = bk->steps_pre.data() + bk->tile_base[l] + (l - 1);
      int gmax = 0;
      for (int k : seg_of_level[l]) gmax = std::max(gmax, std::max(sorted[k].g_full, sorted[k].g_last));
      for (int grp = 0; grp < gmax; ++grp)
        for (int k : seg_of_level[l]) {
          const BankSeg &q = sorted[k];
          for (int rb = 0; rb < q.nblocks; ++rb) {
            const bool lastb = rb == q.nblocks - 1;
            if (grp >= (lastb ? q.g_last : q.g_full)) continue;
            const int rows = lastb ? q.L - 256 * (q.nblocks - 1) : 256;
            const int span = bank_tiles_per_item(rows) * q.gmul;
            const int t0 = grp * span, t1 = std::min(q.ntiles, t0 + span);
            const double c = (double)rows * (double)(pre[t1] - pre[t0] + 8);
            const int cls = std::min(129, std::max(0, (int)std::floor(2.0 * std::log2(c))));
            bucket[cls].push_back(make_int2(k, lastb ? (q.nblocks - 1) * q.g_full + grp
                                                     : rb * q.g_full + grp));
          }
        }
    }
    const size_t first = items.size();
    std::vector<size_t> cls_end;
    for (int c = 129; c >= 0; --c) {
      if (bucket[c].empty()) continue;
      items.insert(items.end(), bucket[c].begin(), bucket[c].end());
      cls_end.push_back(items.size());
    }
    std::vector<int2> placed(items.begin() + first, items.end());
    size_t c0 = first;
    for (size_t c1 : cls_end) {
      const size_t R = kBankXcdRun, full = (c1 - c0) / (8 * R) * (8 * R);
      for (size_t j = 0; j < full; ++j) {
        // the class's j-th position takes element k mod R of run
        // 8 (k / R) + j mod 8 (k = j / 8): a run's items sit at positions
        // of one residue mod 8 from the class start, so they go to one XCD
        // whatever the class's offset in its launch
        const size_t x = j % 8, k = j / 8;
        placed[c0 - first + j] = items[c0 + (8 * (k / R) + x) * R + k % R];
      }
      c0 = c1;
    }
    std::copy(placed.begin(), placed.end(), items.begin() + first);
  };
  long long n_shallow = 0;
  for (const BankSeg &q : sorted)
    if (q.level < kBankDeepLevel) n_shallow += (long long)(q.nblocks - 1) * q.g_full + q.g_last;
  const bool split = n_shallow >= kBankSplitItems;
  std::vector<int2> items;
  items.reserve((size_t)nitems);
  order_levels(1, split ? kBankDeepLevel - 1 : kMaxLevels, items);
  const long long n_main = (long long)items.size();
  if (split) order_levels(kBankDeepLevel, kMaxLevels, items);
  if ((long long)items.size() != nitems) return SIDWT_E_INVAL;  // (cannot happen)
  std::vector<LiftBlock> blocks;
  int boff[kMaxLevels + 1] = {0}, nblk[kMaxLevels + 1] = {0}, npass = 0;
  for (int k = 0; k <= kMaxLevels; ++k) {
    boff[k] = (int)blocks.size();
    nblk[k] = (int)per_pass[k].size();
    blocks.insert(blocks.end(), per_pass[k].begin(), per_pass[k].end());
    if (nblk[k]) npass = k + 1;
  }
  int rc = grow(&ws->d_segs, &ws->c_segs, sorted.size());
  if (!rc) rc = grow(&ws->d_items, &ws->c_items, items.size());
  if (!rc) rc = grow(&ws->d_pulses, &ws->c_pulses, pulses.size());
  if (!rc) rc = grow(&ws->d_blocks, &ws->c_blocks, blocks.size());
  if (!rc) rc = grow(&ws->d_scratch, &ws->c_scratch, (size_t)scratch);
  if (rc) return rc;
  // Descriptor uploads through the workspace's pinned staging buffer.
  const size_t nb[4] = {sorted.size() * sizeof(BankSeg), items.size() * sizeof(int2),
                        pulses.size() * sizeof(BatchPulse), blocks.size() * sizeof(LiftBlock)};
  const void *src[4] = {sorted.data(), items.data(), pulses.data(), blocks.data()};
  void *dst[4] = {ws->d_segs, ws->d_items, ws->d_pulses, ws->d_blocks};
  size_t at[5] = {0};
  for (int k = 0; k < 4; ++k) at[k + 1] = at[k] + ((nb[k] + 255) & ~size_t(255));
  hipError_t e = hipSuccess;
  if (!ws->up_done) e = hipEventCreateWithFlags(&ws->up_done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventSynchronize(ws->up_done);  // staging free again
  if (e == hipSuccess && ws->c_stage < at[4]) {
    if (ws->h_stage) (void)hipHostFree(ws->h_stage);
    ws->h_stage = nullptr;
    ws->c_stage = 0;
    e = hipHostMalloc((void **)&ws->h_stage, at[4], hipHostMallocDefault);
    if (e == hipSuccess) ws->c_stage = at[4];
  }
  for (int k = 0; k < 4 && e == hipSuccess; ++k) {
    if (!nb[k]) continue;
    std::memcpy(ws->h_stage + at[k], src[k], nb[k]);
    e = hipMemcpyAsync(dst[k], ws->h_stage + at[k], nb[k], hipMemcpyHostToDevice, st);
  }
  if (e == hipSuccess) e = hipEventRecord(ws->up_done, st);
  if (e != hipSuccess) return map_err(e, "descriptor upload");
  const LiftBlock *bp[kMaxLevels + 1];
  for (int k = 0; k <= kMaxLevels; ++k) bp[k] = ws->d_blocks + boff[k];
  ws->timed = false;
  if (ws->timing) e = hipEventRecord(ws->ev[0], st);
  if (e == hipSuccess)
    e = launch_lift_passes(bk->d_plan, ws->d_pulses, bp, nblk, pass_lds.data(), npass,
                           ws->d_scratch, st);
  if (e != hipSuccess) return map_err(e, "lifting");
  if (ws->timing) e = hipEventRecord(ws->ev[1], st);
  if (e != hipSuccess) return map_err(e, "event");
  e = launch_bank(bk->precision == SIDWT_BANK_BF16, false, ws->d_segs, ws->d_items,
                  (int)n_main, bk->d_tiles, bk->d_tile_base, bk->d_rl, bk->Jmax, bk->d_lo,
                  bk->d_w, ws->d_scratch, 256 + bk->Umax, st);
  if (e == hipSuccess)
    e = launch_bank(bk->precision == SIDWT_BANK_BF16, true, ws->d_segs, ws->d_items + n_main,
                    (int)(nitems - n_main), bk->d_tiles, bk->d_tile_base, bk->d_rl, bk->Jmax,
                    bk->d_lo, bk->d_w, ws->d_scratch, 256 + bk->UmaxDeep, st);
  if (e == hipSuccess && ws->timing) {
    e = hipEventRecord(ws->ev[2], st);
    ws->timed = e == hipSuccess;
  }
  return map_err(e, "bank kernel");
}

}  // extern "C"
