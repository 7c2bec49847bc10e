// Host side of libsidwt: argument checks, plan lifecycle, LDS layout and
// launches.  The C ABI is declared in include/sidwt.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/sidwt.h"
#include "sidwt_host.hpp"
#include "sidwt_swap.hpp"
#include "sidwt_factor.hpp"

namespace sidwt {
bool generic_steps_fit(const LiftingDesc &d);
hipError_t launch_generic(const LiftingDesc &d, int J, int N, const void *rx, long long n,
                          long long count, long long rx_stride, void *pyr, hipStream_t st);
hipError_t noalloc_scratch(void **out);
hipError_t launch_detect(const void *planes, long long pulse_stride, int J, int N, long long count,
                         float rel, int max_peaks, int *lags, float *db, int *found,
                         hipStream_t st);
}

namespace sidwt {
hipError_t launch_tree(int filter, const void *in, int in_lo, int in_len, int level, int k0,
                       int np, void *outA, int loA, int lenA, void *outB, int loB, int lenB,
                       hipStream_t st);
hipError_t launch_fused(const PlanDesc &plan, const FusedLayout &lay, const void *rx, long long n,
                        long long count, long long rx_stride, void *out, long long out_stride,
                        unsigned planes, hipStream_t st);
hipError_t launch_lift(int filter, int J, int N, const void *rx, long long n, long long count,
                       long long rx_stride, void *pyr, hipStream_t st);
hipError_t launch_synth(int filter, int J, int to, int N, const void *pyr, long long count,
                        void *out, hipStream_t st);
hipError_t launch_fused_i8(const I8Layout &lay, const I8Tile *tiles, const signed char *panels,
                           const void *rx, long long n, long long count, long long rx_stride,
                           void *out, long long out_stride, unsigned planes, const I8Ptrs *ptrs,
                           hipStream_t st);
hipError_t launch_i8_blocks(const I8TilePlan &tp, const I8Tile *tiles, const signed char *panels,
                            const void *rx, long long n, long long count, long long rx_stride,
                            void *pyr, void *out, long long out_stride, const I8Ptrs *ptrs,
                            hipStream_t st);
size_t synth_lds_bytes(int filter, int N, int to);
}  // namespace sidwt

using sidwt::FusedLayout;
using sidwt::PlanDesc;

struct sidwt_plan {
  int filter;
  int J;
  int64_t m;
  int device;
  hipStream_t stream;
  PlanDesc desc;
  void *coef;
  size_t coef_bytes;
  // The reference as complex64 (float filters): plane 0's weights of the
  // roles-exchanged correlation.
  void *ref_dev = nullptr;
  // Integer plans: digit panels of the phases for the int8 matrix-core
  // path (i8_wl digits per entry; 0 when the path does not apply).
  int i8_wl = 0;
  std::vector<sidwt::I8Tile> i8_tiles;
  std::vector<int> i8_tile_base;
  sidwt::I8Tile *d_i8_tiles = nullptr;
  signed char *d_i8_panels = nullptr;
  // Pulses too long for the whole-pulse LDS layout go through the tiled
  // batch path; its buffers are kept for the last (n, count) seen.
  mutable sidwt_batch *tiled = nullptr;
  mutable int64_t tiled_n = 0, tiled_count = 0;
};

namespace {

using namespace sidwt::host;

bool valid_filter(int f) { return f >= SIDWT_LEGALL53 && f <= SIDWT_LEGALL53_INT; }

int map_err(hipError_t e) {
  if (e == hipSuccess) return SIDWT_OK;
  if (e == hipErrorOutOfMemory) return SIDWT_E_NOMEM;
  return SIDWT_E_DEVICE;
}

int check_pulse(const sidwt_plan *p, int64_t n, int64_t *N_out) {
  if (n < 1) return SIDWT_E_INVAL;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return SIDWT_E_DEVICE;
  if (dev != p->device) return SIDWT_E_INVAL;  // the plan's memory lives on its own device
  const int64_t N = transform_length(n, p->J);
  if (N > kMaxN) return SIDWT_E_SIZE;
  if ((N >> p->J) < 2) return SIDWT_E_INVAL;
  if (p->m > N) return SIDWT_E_SIZE;
  if (p->filter == SIDWT_LEGALL53_INT && !int_support_fits(p->desc, N)) return SIDWT_E_SIZE;
  *N_out = N;
  return SIDWT_OK;
}

}  // namespace

namespace {

// Digit panels of an integer plan for the int8 path (see build_i8_panels):
// the phases come back from the device, the fewest digits that hold every
// entry are chosen, and the path is kept only while every shift-class sum
// of a tile (at most min(3, WL) digit pairs, 32 products of at most 2^14
// per chunk of 16 offsets) stays below 2^31.  Leaves i8_wl = 0 when the
// path does not apply.
hipError_t build_i8(sidwt_plan *p) {
  const PlanDesc &d = p->desc;
  std::vector<int32_t> coef(p->coef_bytes / 4);
  hipError_t e = hipMemcpy(coef.data(), p->coef, p->coef_bytes, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return e;
  long long maxabs = 0;
  for (int32_t v : coef) maxabs = std::max(maxabs, std::llabs((long long)v));
  const int wl = i8_weight_limbs(maxabs);
  if (!wl) return hipSuccess;
  std::vector<signed char> panels;
  build_i8_panels(d, coef.data(), wl, &p->i8_tiles, &p->i8_tile_base, &panels);
  const long long pairs = std::min(sidwt::kI8DataLimbs, wl);
  for (const sidwt::I8Tile &t : p->i8_tiles)
    if (pairs * 32LL * (t.nch[0] + t.nch[1]) * 16384LL >= (1LL << 31)) return hipSuccess;
  e = hipMalloc(&p->d_i8_tiles, p->i8_tiles.size() * sizeof(sidwt::I8Tile));
  if (e == hipSuccess)
    e = hipMemcpy(p->d_i8_tiles, p->i8_tiles.data(), p->i8_tiles.size() * sizeof(sidwt::I8Tile),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&p->d_i8_panels, std::max<size_t>(panels.size(), 16));
  if (e == hipSuccess)
    e = hipMemcpy(p->d_i8_panels, panels.data(), panels.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (p->d_i8_tiles) (void)hipFree(p->d_i8_tiles);
    if (p->d_i8_panels) (void)hipFree(p->d_i8_panels);
    p->d_i8_tiles = nullptr;
    p->d_i8_panels = nullptr;
    return e;
  }
  p->i8_wl = wl;
  return hipSuccess;
}

}  // namespace

// Descriptor of a plan for the batch module (C++ linkage, not exported in
// the header).
const sidwt::PlanDesc *sidwt_plan_desc(const sidwt_plan *p) { return p ? &p->desc : nullptr; }

// ---------------------------------------------------------------------------
// Integer batches (C++ linkage; sidwt_batch.cpp holds the handle when every
// plan of a batch is integer).  Pulses are grouped by (plan, n); a group on
// the int8 path is one launch of the whole-pulse kernel, or one lifting pass
// per level plus one block launch, over the group's per-pulse pointers
// (uploaded only when they change).  FP64 plans (J >= 8) run one whole-pulse
// launch per pulse.  Groups go out in order on the call's stream, so the
// block path's pyramid is shared by all groups (largest group's size).
// ---------------------------------------------------------------------------
struct sidwt_int_batch {
  struct Group {
    const sidwt_plan *p;
    int64_t n, N;
    int path;                 // 0: int8 whole pulse, 1: int8 blocks, 2: FP64 per pulse
    std::vector<int> pulses;  // batch indices
    int ptr0;                 // first entry in the pointer array
    sidwt::I8Layout lay;
    sidwt::I8TilePlan tp;
    FusedLayout flay;
  };
  int count = 0;
  std::vector<Group> groups;
  std::vector<sidwt::I8Ptrs> ptrs;     // group order
  sidwt::I8Ptrs *d_ptrs = nullptr;
  sidwt::I8Ptrs *h_stage = nullptr;    // pinned staging of ptrs
  hipEvent_t up_done = nullptr;
  bool uploaded = false;
  void *pyr = nullptr;
  size_t pyr_bytes = 0;
  int64_t n_whole = 0, n_blocks = 0, n_fp64 = 0;
};

void sidwt_int_batch_free(sidwt_int_batch *ib) {
  if (!ib) return;
  (void)hipDeviceSynchronize();
  (void)hipFree(ib->d_ptrs);
  (void)hipFree(ib->pyr);
  if (ib->h_stage) (void)hipHostFree(ib->h_stage);
  if (ib->up_done) (void)hipEventDestroy(ib->up_done);
  delete ib;
}

int sidwt_int_batch_create(const sidwt_plan *const *plans, const int64_t *n, int count,
                           sidwt_int_batch **out) {
  if (!plans || !n || !out || count < 1) return SIDWT_E_INVAL;
  sidwt_int_batch *ib = new (std::nothrow) sidwt_int_batch();
  if (!ib) return SIDWT_E_NOMEM;
  ib->count = count;
  int rc = SIDWT_OK;
  for (int i = 0; i < count && !rc; ++i) {
    const sidwt_plan *p = plans[i];
    if (!p || p->filter != SIDWT_LEGALL53_INT) {
      rc = SIDWT_E_INVAL;
      break;
    }
    int64_t N = 0;
    rc = check_pulse(p, n[i], &N);
    if (rc) break;
    size_t g = 0;
    while (g < ib->groups.size() && !(ib->groups[g].p == p && ib->groups[g].n == n[i])) ++g;
    if (g == ib->groups.size()) {
      sidwt_int_batch::Group G{};
      G.p = p;
      G.n = n[i];
      G.N = N;
      if (p->i8_wl && make_i8_layout(p->desc, p->i8_wl, p->i8_tiles.data(),
                                     p->i8_tile_base.data(), N, &G.lay) == 0)
        G.path = 0;
      else if (p->i8_wl && make_i8_tile_plan(p->desc, p->i8_wl, p->i8_tiles.data(),
                                             p->i8_tile_base.data(), N, &G.tp) == 0)
        G.path = 1;
      else if (make_layout(p->desc, N, &G.flay) == 0)
        G.path = 2;
      else
        rc = SIDWT_E_UNSUPPORTED;
      ib->groups.push_back(G);
    }
    ib->groups[g].pulses.push_back(i);
  }
  if (!rc) {
    int at = 0;
    for (auto &G : ib->groups) {
      G.ptr0 = at;
      at += (int)G.pulses.size();
      const int64_t c = (int64_t)G.pulses.size();
      (G.path == 0 ? ib->n_whole : G.path == 1 ? ib->n_blocks : ib->n_fp64) += c;
      if (G.path == 1)
        ib->pyr_bytes = std::max(ib->pyr_bytes, (size_t)c * 2 * (size_t)G.N * sizeof(int2));
    }
    ib->ptrs.assign((size_t)count, sidwt::I8Ptrs{nullptr, nullptr});
    hipError_t e = hipMalloc(&ib->d_ptrs, (size_t)count * sizeof(sidwt::I8Ptrs));
    if (e == hipSuccess && ib->pyr_bytes) e = hipMalloc(&ib->pyr, ib->pyr_bytes);
    if (e == hipSuccess)
      e = hipHostMalloc((void **)&ib->h_stage, (size_t)count * sizeof(sidwt::I8Ptrs),
                        hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ib->up_done, hipEventDisableTiming);
    rc = map_err(e);
  }
  if (rc) {
    sidwt_int_batch_free(ib);
    return rc;
  }
  *out = ib;
  return SIDWT_OK;
}

int sidwt_int_batch_run(sidwt_int_batch *ib, const void *const *rx, void *const *out,
                        hipStream_t st) {
  if (!ib || !rx || !out) return SIDWT_E_INVAL;
  bool same = ib->uploaded;
  for (const auto &G : ib->groups)
    for (size_t k = 0; k < G.pulses.size(); ++k) {
      const int i = G.pulses[k];
      if (!rx[i] || !out[i]) return SIDWT_E_INVAL;
      sidwt::I8Ptrs &q = ib->ptrs[(size_t)G.ptr0 + k];
      same = same && q.rx == rx[i] && q.out == out[i];
      q.rx = static_cast<const short2 *>(rx[i]);
      q.out = static_cast<long long *>(out[i]);
    }
  hipError_t e = hipSuccess;
  if (!same) {
    const size_t bytes = ib->ptrs.size() * sizeof(sidwt::I8Ptrs);
    e = hipEventSynchronize(ib->up_done);  // the staging buffer is free again
    if (e == hipSuccess) {
      std::memcpy(ib->h_stage, ib->ptrs.data(), bytes);
      e = hipMemcpyAsync(ib->d_ptrs, ib->h_stage, bytes, hipMemcpyHostToDevice, st);
    }
    if (e == hipSuccess) e = hipEventRecord(ib->up_done, st);
    if (e != hipSuccess) return map_err(e);
    ib->uploaded = true;
  }
  for (const auto &G : ib->groups) {
    const sidwt_plan *p = G.p;
    const long long c = (long long)G.pulses.size();
    const sidwt::I8Ptrs *dp = ib->d_ptrs + G.ptr0;
    if (G.path == 0) {
      e = sidwt::launch_fused_i8(G.lay, p->d_i8_tiles, p->d_i8_panels, nullptr, G.n, c, 0,
                                 nullptr, 0, (1u << p->J) - 1u, dp, st);
    } else if (G.path == 1) {
      e = sidwt::launch_i8_blocks(G.tp, p->d_i8_tiles, p->d_i8_panels, nullptr, G.n, c, 0,
                                  ib->pyr, nullptr, 0, dp, st);
    } else {
      for (long long k = 0; k < c && e == hipSuccess; ++k) {
        const int i = G.pulses[(size_t)k];
        e = sidwt::launch_fused(p->desc, G.flay, rx[i], G.n, 1, G.n, out[i],
                                (long long)p->J * G.N, (1u << p->J) - 1u, st);
      }
    }
    if (e != hipSuccess) return map_err(e);
  }
  return SIDWT_OK;
}

void sidwt_int_batch_counts(const sidwt_int_batch *ib, int64_t *whole, int64_t *blocks,
                            int64_t *fp64, int64_t *scratch_bytes) {
  *whole = ib->n_whole;
  *blocks = ib->n_blocks;
  *fp64 = ib->n_fp64;
  *scratch_bytes = (int64_t)ib->pyr_bytes;
}

extern "C" {

const char *sidwt_strerror(int code) {
  switch (code) {
    case SIDWT_OK: return "ok";
    case SIDWT_E_INVAL: return "invalid argument";
    case SIDWT_E_SIZE: return "size out of range for this plan";
    case SIDWT_E_NOMEM: return "device allocation failed";
    case SIDWT_E_DEVICE: return "HIP runtime error";
    case SIDWT_E_UNSUPPORTED: return "request not supported by the library";
    case SIDWT_E_SCRATCH: return "request needs more than the library's static scratch";
    default: return "unknown error";
  }
}

const char *sidwt_version(void) { return "sidwt 0.1 gfx950"; }

int sidwt_plan_create(int filter, int J, const void *ref, int64_t m, sidwt_plan **out) {
  if (!out || !ref || !valid_filter(filter) || J < 1 || J > SIDWT_MAX_LEVELS || m < 1)
    return SIDWT_E_INVAL;
  if (m > kMaxRef) return SIDWT_E_SIZE;
  if (filter == SIDWT_LEGALL53_INT) {
    // Exactness of the FP64 accumulation, checked on the host before any
    // device work (for a full-scale int16 pulse and this reference's peak).
    PlanDesc probe;
    std::memset(&probe, 0, sizeof(probe));
    probe.J = J;
    probe.m = (int)m;
    plan_windows(filter, J, (int)m, &probe);
    const int16_t *r16 = static_cast<const int16_t *>(ref);
    int peak = 0;
    for (int64_t i = 0; i < 2 * m; ++i) peak = std::max(peak, std::abs((int)r16[i]));
    if (!int_sums_exact(probe, peak)) return SIDWT_E_SIZE;
  }
  sidwt_plan *p = new (std::nothrow) sidwt_plan();
  if (!p) return SIDWT_E_NOMEM;
  p->filter = filter;
  p->J = J;
  p->m = m;
  p->stream = nullptr;
  p->coef = nullptr;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return SIDWT_E_DEVICE;
  }
  PlanDesc &d = p->desc;
  std::memset(&d, 0, sizeof(d));
  d.filter = filter;
  d.J = J;
  d.m = (int)m;
  const long long off = plan_windows(filter, J, (int)m, &d);
  const size_t elem = 8;  // float2 or int2
  p->coef_bytes = (size_t)off * elem;
  hipError_t e = hipMalloc(&p->coef, p->coef_bytes);
  if (e != hipSuccess) {
    delete p;
    return map_err(e);
  }
  d.coef = p->coef;
  // Reference on the device as 8-byte complex elements.
  std::vector<int32_t> host(2 * (size_t)m);
  if (filter == SIDWT_LEGALL53_INT) {
    const int16_t *r16 = static_cast<const int16_t *>(ref);
    for (int64_t i = 0; i < 2 * m; ++i) host[i] = r16[i];
  } else {
    std::memcpy(host.data(), ref, 8 * (size_t)m);
  }
  void *ref_dev = nullptr;
  e = hipMalloc(&ref_dev, 8 * (size_t)m);
  if (e == hipSuccess) e = hipMemcpy(ref_dev, host.data(), 8 * (size_t)m, hipMemcpyHostToDevice);
  int in_lo = 0;
  int in_len = (int)m;
  const char *base = static_cast<const char *>(p->coef);
  for (int l = 1; l <= J && e == hipSuccess; ++l) {
    const sidwt::LevelDesc &lv = d.lv[l];
    int k0 = std::min({lv.lo[0], lv.lo[1], sidwt::floor_div(in_lo, 2)}) - 4;
    int k1 = std::max({lv.lo[0] + lv.len[0], lv.lo[1] + lv.len[1],
                       sidwt::floor_div(in_lo + in_len + 1, 2) + 1}) + 4;
    const void *in = (l == 1) ? ref_dev : (const void *)(base + d.lv[l - 1].off[0] * elem);
    e = sidwt::launch_tree(filter, in, in_lo, in_len, l, k0, k1 - k0,
                           (void *)(base + lv.off[0] * elem), lv.lo[0], lv.len[0],
                           (void *)(base + lv.off[1] * elem), lv.lo[1], lv.len[1], nullptr);
    in_lo = lv.lo[0];
    in_len = lv.len[0];
  }
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e == hipSuccess && filter == SIDWT_LEGALL53_INT && i8_data_fits(d)) e = build_i8(p);
  if (e != hipSuccess || filter == SIDWT_LEGALL53_INT) {
    if (ref_dev) (void)hipFree(ref_dev);
    ref_dev = nullptr;
  }
  if (e != hipSuccess) {
    (void)hipFree(p->coef);
    delete p;
    return map_err(e);
  }
  p->ref_dev = ref_dev;
  *out = p;
  return SIDWT_OK;
}

void sidwt_free(sidwt_plan *p) {
  if (!p) return;
  sidwt_batch_free(p->tiled);
  if (p->coef || p->ref_dev || p->d_i8_panels) (void)hipDeviceSynchronize();
  if (p->d_i8_tiles) (void)hipFree(p->d_i8_tiles);
  if (p->d_i8_panels) (void)hipFree(p->d_i8_panels);
  if (p->coef) (void)hipFree(p->coef);
  if (p->ref_dev) (void)hipFree(p->ref_dev);
  delete p;
}

int64_t sidwt_out_len(const sidwt_plan *p, int64_t n) {
  if (!p || n < 1) return -1;
  return (int64_t)p->J * transform_length(n, p->J);
}

int sidwt_set_stream(sidwt_plan *p, void *hip_stream) {
  if (!p) return SIDWT_E_INVAL;
  p->stream = static_cast<hipStream_t>(hip_stream);
  return SIDWT_OK;
}

// Uniform batch, the planes of `planes` (bit j: plane j) only, on stream
// `st`.  Pulses too long for one workgroup's LDS take the tiled path: with
// `cache` the plan keeps that path's batch for the last (n, count) (the
// plan-stream entry points), else a one-shot batch is built, run, the
// stream synchronised and the batch freed (the per-call-stream entry
// points, which leave the plan untouched).
static int correlate_many_planes(const sidwt_plan *p, const void *rx, int64_t n, int64_t count,
                                 int64_t rx_stride, void *out, int64_t out_stride,
                                 unsigned planes, hipStream_t st, bool cache) {
  if (!p || count < 0 || count > 0x7fffffff) return SIDWT_E_INVAL;
  const unsigned all = (1u << p->J) - 1u;
  planes &= all;
  if (!planes) return SIDWT_E_INVAL;
  int64_t N = 0;
  int rc = check_pulse(p, n, &N);
  if (rc) return rc;
  if (rx_stride < n || out_stride < (int64_t)p->J * N) return SIDWT_E_INVAL;
  if (count == 0) return SIDWT_OK;
  if (!rx || !out) return SIDWT_E_INVAL;
  if (p->i8_wl) {
    sidwt::I8Layout il;
    if (make_i8_layout(p->desc, p->i8_wl, p->i8_tiles.data(), p->i8_tile_base.data(), N, &il) == 0)
      return map_err(sidwt::launch_fused_i8(il, p->d_i8_tiles, p->d_i8_panels, rx, n, count,
                                            rx_stride, out, out_stride, planes, nullptr, st));
    // Too long for one workgroup: levels lifted into a temporary HBM
    // pyramid, then blocks of lag-block rows (the stream is synchronised
    // before the pyramid is released).
    sidwt::I8TilePlan tp;
    if (make_i8_tile_plan(p->desc, p->i8_wl, p->i8_tiles.data(), p->i8_tile_base.data(), N,
                          &tp) == 0) {
      if (planes != all) return SIDWT_E_UNSUPPORTED;
      void *pyr = nullptr;
      hipError_t e = hipMalloc(&pyr, (size_t)count * 2 * (size_t)N * sizeof(int2));
      if (e != hipSuccess) return map_err(e);
      e = sidwt::launch_i8_blocks(tp, p->d_i8_tiles, p->d_i8_panels, rx, n, count, rx_stride,
                                  pyr, out, out_stride, nullptr, st);
      const hipError_t es = hipStreamSynchronize(st);
      (void)hipFree(pyr);
      return map_err(e != hipSuccess ? e : es);
    }
  }
  FusedLayout lay;
  if (make_layout(p->desc, N, &lay) == 0)
    return map_err(sidwt::launch_fused(p->desc, lay, rx, n, count, rx_stride, out, out_stride,
                                       planes, st));
  // Too long for one workgroup's LDS: levels lifted into an HBM scratch
  // pyramid, then lag tiles (the uneven-batch machinery, one plan).
  if (p->filter == SIDWT_LEGALL53_INT || planes != all) return SIDWT_E_UNSUPPORTED;
  std::vector<const void *> rxp((size_t)count);
  std::vector<void *> outp((size_t)count);
  for (int64_t i = 0; i < count; ++i) {
    rxp[i] = static_cast<const char *>(rx) + i * rx_stride * 8;
    outp[i] = static_cast<char *>(out) + i * out_stride * 8;
  }
  std::vector<const sidwt_plan *> ps((size_t)count, p);
  std::vector<int64_t> ns((size_t)count, n);
  if (!cache)
    return sidwt_correlate_batch(ps.data(), rxp.data(), ns.data(), outp.data(), (int)count, st);
  if (!p->tiled || p->tiled_n != n || p->tiled_count != count) {
    sidwt_batch_free(p->tiled);
    p->tiled = nullptr;
    rc = sidwt_batch_create(ps.data(), ns.data(), (int)count, &p->tiled);
    if (rc) return rc;
    p->tiled_n = n;
    p->tiled_count = count;
  }
  return sidwt_batch_run(p->tiled, rxp.data(), outp.data(), st);
}

int sidwt_correlate_many(const sidwt_plan *p, const void *rx, int64_t n, int64_t count,
                         int64_t rx_stride, void *out, int64_t out_stride) {
  if (!p) return SIDWT_E_INVAL;
  return correlate_many_planes(p, rx, n, count, rx_stride, out, out_stride, ~0u, p->stream, true);
}

int sidwt_correlate_planes(const sidwt_plan *p, const void *rx, int64_t n, int64_t count,
                           int64_t rx_stride, void *out, int64_t out_stride,
                           unsigned plane_mask) {
  if (!p) return SIDWT_E_INVAL;
  return correlate_many_planes(p, rx, n, count, rx_stride, out, out_stride, plane_mask,
                               p->stream, true);
}

int sidwt_correlate(const sidwt_plan *p, const void *rx, int64_t n, void *out) {
  if (!p) return SIDWT_E_INVAL;
  return sidwt_correlate_many(p, rx, n, 1, n, out, sidwt_out_len(p, n));
}

int sidwt_correlate_many_on(const sidwt_plan *p, const void *rx, int64_t n, int64_t count,
                            int64_t rx_stride, void *out, int64_t out_stride,
                            unsigned plane_mask, void *hip_stream) {
  return correlate_many_planes(p, rx, n, count, rx_stride, out, out_stride, plane_mask,
                               static_cast<hipStream_t>(hip_stream), false);
}

int sidwt_correlate_on(const sidwt_plan *p, const void *rx, int64_t n, void *out,
                       void *hip_stream) {
  if (!p) return SIDWT_E_INVAL;
  return sidwt_correlate_many_on(p, rx, n, 1, n, out, sidwt_out_len(p, n), ~0u, hip_stream);
}

namespace {

// Workspace of the roles-exchanged correlation: levels 1 .. J-1 of the
// redundant tree, N complex64 elements per level and pulse; -1 when that
// does not fit in 63 bits.
int64_t swap_ws_bytes(int J, int64_t N, int64_t count) {
  const int64_t per_pulse = (int64_t)(J - 1) * N * 8;  // < 2^48 (N <= 2^30)
  if (per_pulse > 0 && count > INT64_MAX / per_pulse) return -1;
  return per_pulse * count;
}

}  // namespace

int64_t sidwt_swap_workspace_bytes(const sidwt_plan *p, int64_t n, int64_t count) {
  if (!p || n < 1 || count < 0) return -1;
  return swap_ws_bytes(p->J, transform_length(n, p->J), count);
}

static int correlate_swapped(const sidwt_plan *p, const void *rx, int64_t n, int64_t count,
                             int64_t rx_stride, void *out, int64_t out_stride, void *workspace,
                             int64_t workspace_bytes, hipStream_t st) {
  if (!p || count < 0 || (int64_t)count * p->J > 0x7fffffff) return SIDWT_E_INVAL;
  if (p->filter == SIDWT_LEGALL53_INT || !p->ref_dev) return SIDWT_E_UNSUPPORTED;
  // the deepest tree level launches one workgroup per (pulse, phase)
  if ((count << (p->J - 1)) > 0x7fffffff) return SIDWT_E_SIZE;
  int64_t N = 0;
  int rc = check_pulse(p, n, &N);
  if (rc) return rc;
  if (swap_ws_bytes(p->J, N, count) < 0) return SIDWT_E_SIZE;
  if (rx_stride < n || out_stride < (int64_t)p->J * N) return SIDWT_E_INVAL;
  sidwt::SwapDesc wd;
  std::memset(&wd, 0, sizeof(wd));
  size_t lds = 0, lds_chunk = 0;
  for (int j = 0; j < p->J; ++j) {
    const int K = j == 0 ? (int)p->m : p->desc.lv[j].len[0];
    lds = std::max(lds, sidwt::swap_lds_bytes((int)N, j, K, 0));
    lds_chunk = std::max(lds_chunk, sidwt::swap_lds_bytes((int)N, j, K, 1));
    wd.a[j] = j == 0 ? static_cast<const float2 *>(p->ref_dev)
                     : static_cast<const float2 *>(p->coef) + p->desc.lv[j].off[0];
    wd.lo[j] = j == 0 ? 0 : p->desc.lv[j].lo[0];
    wd.len[j] = K;
  }
  // whole planes per workgroup when they fit, else chunks of one phase
  const int chunked = lds > (size_t)kLdsWords * 4;
  if (chunked) lds = lds_chunk;
  if (lds > (size_t)kLdsWords * 4) return SIDWT_E_UNSUPPORTED;
  if (chunked) {  // one workgroup per (pulse, plane, phase, chunk of 8192 lags)
    int64_t items = 0;
    for (int j = 0; j < p->J; ++j) items += count * ((((N >> j) + 8191) / 8192) << j);
    if (items > 0x7fffffff) return SIDWT_E_SIZE;
  }
  if (count == 0) return SIDWT_OK;
  if (!rx || !out || (p->J > 1 && !workspace)) return SIDWT_E_INVAL;
  if (workspace_bytes < swap_ws_bytes(p->J, N, count)) return SIDWT_E_INVAL;
  return map_err(sidwt::launch_swap(p->filter, p->J, (int)N, rx, n, count, rx_stride, workspace,
                                    wd, lds, chunked, out, out_stride, st));
}

int sidwt_correlate_swapped(const sidwt_plan *p, const void *rx, int64_t n, int64_t count,
                            int64_t rx_stride, void *out, int64_t out_stride, void *workspace,
                            int64_t workspace_bytes) {
  if (!p) return SIDWT_E_INVAL;
  return correlate_swapped(p, rx, n, count, rx_stride, out, out_stride, workspace,
                           workspace_bytes, p->stream);
}

int sidwt_correlate_swapped_on(const sidwt_plan *p, const void *rx, int64_t n, int64_t count,
                               int64_t rx_stride, void *out, int64_t out_stride, void *workspace,
                               int64_t workspace_bytes, void *hip_stream) {
  return correlate_swapped(p, rx, n, count, rx_stride, out, out_stride, workspace,
                           workspace_bytes, static_cast<hipStream_t>(hip_stream));
}

int sidwt_correlate_swapped_noalloc(const sidwt_plan *p, const void *rx, int64_t n,
                                    int64_t count, int64_t rx_stride, void *out,
                                    int64_t out_stride, void *hip_stream) {
  if (!p || n < 1 || count < 0) return SIDWT_E_INVAL;
  const int64_t need = swap_ws_bytes(p->J, transform_length(n, p->J), count);
  if (need < 0 || need > (int64_t)SIDWT_NOALLOC_SCRATCH_BYTES) return SIDWT_E_SCRATCH;
  void *ws = nullptr;
  if (need > 0) {
    const hipError_t e = sidwt::noalloc_scratch(&ws);
    if (e != hipSuccess) return map_err(e);
  }
  return correlate_swapped(p, rx, n, count, rx_stride, out, out_stride, ws,
                           (int64_t)SIDWT_NOALLOC_SCRATCH_BYTES,
                           static_cast<hipStream_t>(hip_stream));
}

int sidwt_detect_peaks(const void *planes, int64_t count, int J, int64_t N, int64_t pulse_stride,
                       float rel_power, int max_peaks, int32_t *lags, float *db, int32_t *found,
                       void *hip_stream) {
  if (count < 0 || J < 1 || J > SIDWT_MAX_LEVELS || N < 1 || N > 0x7fffffff ||
      pulse_stride < (int64_t)J * N || count * J > 0x7fffffff || max_peaks < 0 ||
      !(rel_power >= 0.f) || rel_power > 3.0e38f)
    return SIDWT_E_INVAL;
  if (count == 0) return SIDWT_OK;
  if (!planes || !found || (max_peaks > 0 && (!lags || !db))) return SIDWT_E_INVAL;
  return map_err(sidwt::launch_detect(planes, pulse_stride, J, (int)N, count, rel_power,
                                      max_peaks, lags, db, found,
                                      static_cast<hipStream_t>(hip_stream)));
}

int sidwt_lift_generic(const sidwt_lifting *f, int J, const void *rx, int64_t n, int64_t count,
                       int64_t rx_stride, void *pyr, void *hip_stream) {
  const sidwt::LiftingDesc *d = sidwt::lifting_desc(f);
  if (!d || J < 1 || J > SIDWT_MAX_LEVELS || n < 1 || count < 0 || count > 0x7fffffff ||
      rx_stride < n)
    return SIDWT_E_INVAL;
  const int64_t N = transform_length(n, J);
  if ((N >> J) < 2) return SIDWT_E_INVAL;
  if (2 * (N / 2 + N / 4 + 1) > kLdsWords || !sidwt::generic_steps_fit(*d))
    return SIDWT_E_UNSUPPORTED;
  if (count == 0) return SIDWT_OK;
  if (!rx || !pyr) return SIDWT_E_INVAL;
  return map_err(sidwt::launch_generic(*d, J, (int)N, rx, n, count, rx_stride, pyr,
                                       static_cast<hipStream_t>(hip_stream)));
}

int sidwt_lift_many(int filter, int J, const void *rx, int64_t n, int64_t count,
                    int64_t rx_stride, void *pyr, void *hip_stream) {
  if (!valid_filter(filter) || J < 1 || J > SIDWT_MAX_LEVELS || n < 1 || count < 0 ||
      count > 0x7fffffff || rx_stride < n)
    return SIDWT_E_INVAL;
  const int64_t N = transform_length(n, J);
  if ((N >> J) < 2) return SIDWT_E_INVAL;
  if (2 * (N / 2 + N / 4 + 1) > kLdsWords) return SIDWT_E_UNSUPPORTED;
  if (count == 0) return SIDWT_OK;
  if (!rx || !pyr) return SIDWT_E_INVAL;
  return map_err(sidwt::launch_lift(filter, J, (int)N, rx, n, count, rx_stride, pyr,
                                    static_cast<hipStream_t>(hip_stream)));
}

int sidwt_synth_many(int filter, int J, int to, const void *pyr, int64_t N, int64_t count,
                     void *out, void *hip_stream) {
  if (!valid_filter(filter) || J < 1 || J > SIDWT_MAX_LEVELS || to < 0 || to >= J || N < 2 ||
      N > kMaxN || (N & ((int64_t(1) << J) - 1)) || (N >> J) < 2 || count < 0 ||
      count > 0x7fffffff)
    return SIDWT_E_INVAL;
  if (sidwt::synth_lds_bytes(filter, (int)N, to) > (size_t)kLdsWords * 4) return SIDWT_E_UNSUPPORTED;
  if (count == 0) return SIDWT_OK;
  if (!pyr || !out) return SIDWT_E_INVAL;
  return map_err(sidwt::launch_synth(filter, J, to, (int)N, pyr, count, out,
                                     static_cast<hipStream_t>(hip_stream)));
}

int sidwt_plan_info(const sidwt_plan *p, int64_t *v, int nv) {
  if (!p || !v || nv < 1) return SIDWT_E_INVAL;
  long long panel_bytes = 0;
  for (const sidwt::I8Tile &t : p->i8_tiles)
    panel_bytes += (long long)(t.nch[0] + t.nch[1]) * p->i8_wl * sidwt::kI8ChunkBytes;
  const int64_t vals[] = {p->filter, p->J, p->m, (int64_t)p->coef_bytes, p->i8_wl,
                          p->i8_wl ? panel_bytes : 0};
  const int k = (int)(sizeof(vals) / sizeof(vals[0]));
  for (int i = 0; i < nv; ++i) v[i] = i < k ? vals[i] : 0;
  return SIDWT_OK;
}

int sidwt_plan_phase(const sidwt_plan *p, int level, int band, int r, int32_t *lo, int32_t *len,
                     void *dst) {
  if (!p || !lo || !len || level < 1 || level > p->J || band < 0 || band > 1 || r < 0 ||
      r >= (1 << level))
    return SIDWT_E_INVAL;
  const sidwt::LevelDesc &lv = p->desc.lv[level];
  *lo = lv.lo[band];
  *len = lv.len[band];
  if (!dst) return SIDWT_OK;
  const char *src = static_cast<const char *>(p->coef) + (lv.off[band] + (long long)r * lv.len[band]) * 8;
  return map_err(hipMemcpy(dst, src, (size_t)lv.len[band] * 8, hipMemcpyDeviceToHost));
}

}  // extern "C"
