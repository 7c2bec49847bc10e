// Uneven batches of pulses through one persistent launch (C ABI part of
// libsidwt; declarations in include/sidwt.h).
//
// A batch object fixes the plans and pulse lengths.  Building it:
//   - short pulses (transform length N <= fused_max_N whose fused LDS
//     layout fits) become one "whole pulse" work item each (lifting and all
//     planes in LDS);
//   - long pulses are lifted into an HBM scratch pyramid, `lift_depth`
//     levels per pass (each pass reads its input level once, in blocks with
//     halos, and writes every level it lifts), and split into lag tiles
//     (rows of one level) whose band windows hold about `tile_window`
//     elements;
//   - items are ordered by estimated cost, largest first, and pulled by a
//     persistent kernel from an atomic counter.
// The launch sequence (counter reset, lifting passes, persistent kernels)
// is captured once in a HIP graph and replayed; each run only uploads the
// caller's pulse and output pointers.  sidwt_batch_tune times candidate
// tile windows, fused/tiled splits and lifting depths on the caller's
// buffers and keeps the best.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/sidwt.h"
#include "sidwt_host.hpp"

namespace sidwt {
hipError_t batch_set_lds(size_t bytes);
hipError_t batch_occupancy(bool tiles_only, size_t lds_bytes, int *blocks_per_cu);
hipError_t launch_lift_passes(const PlanDesc *plans, const BatchPulse *pulses,
                              const LiftBlock *const *blocks, const int *nblocks,
                              const size_t *lds, int npass, float2 *scratch, hipStream_t st);
hipError_t launch_batch_reset(int *counters, int n, hipStream_t st);
hipError_t launch_batch_items(bool tiles_only, const PlanDesc *plans, const FusedLayout *lays,
                              const BatchPulse *pulses, const BatchItem *items, int nitems,
                              int *counter, float2 *scratch, int grid, size_t lds_bytes,
                              hipStream_t st);
}  // namespace sidwt

// The plan object is defined in sidwt_api.cpp; the batch only needs its
// descriptor, which that file exposes through this accessor.
extern "C++" const sidwt::PlanDesc *sidwt_plan_desc(const sidwt_plan *p);

using namespace sidwt;
using namespace sidwt::host;

namespace {

int map_err(hipError_t e, const char *what = nullptr) {
  if (e == hipSuccess) return SIDWT_OK;
  if (what && std::getenv("SIDWT_DEBUG"))
    std::fprintf(stderr, "sidwt batch: %s: %s\n", what, hipGetErrorString(e));
  if (e == hipErrorOutOfMemory) return SIDWT_E_NOMEM;
  return SIDWT_E_DEVICE;
}

template <class T>
int upload(T **dptr, size_t *cap, const std::vector<T> &v) {
  const size_t need = std::max<size_t>(1, v.size());
  if (*cap < need) {
    if (*dptr) (void)hipFree(*dptr);
    *dptr = nullptr;
    *cap = 0;
    hipError_t e = hipMalloc(dptr, need * sizeof(T));
    if (e != hipSuccess) return map_err(e, "hipMalloc (descriptors)");
    *cap = need;
  }
  if (!v.empty()) {
    hipError_t e = hipMemcpy(*dptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return map_err(e, "hipMemcpy (descriptors)");
  }
  return SIDWT_OK;
}

}  // namespace

// Integer batches (sidwt_api.cpp): every plan of the batch integer.
struct sidwt_int_batch;
int sidwt_int_batch_create(const sidwt_plan *const *plans, const int64_t *n, int count,
                           sidwt_int_batch **out);
int sidwt_int_batch_run(sidwt_int_batch *ib, const void *const *rx, void *const *out,
                        hipStream_t st);
void sidwt_int_batch_free(sidwt_int_batch *ib);
void sidwt_int_batch_counts(const sidwt_int_batch *ib, int64_t *whole, int64_t *blocks,
                            int64_t *fp64, int64_t *scratch_bytes);

struct sidwt_batch {
  int count = 0;
  sidwt_int_batch *ib = nullptr;     // integer batch: every other field unused
  std::vector<PlanDesc> plans;       // distinct plans
  std::vector<int> pulse_plan;       // per pulse: index into plans
  std::vector<int64_t> n, N;
  std::vector<int> J;
  // configuration
  int fused_max_N = 8192;
  int tile_window = 3072;       // band-window budget of a tile, elements
  int lift_depth = 4;           // levels per lifting pass of the tiled pulses
  int tuned = 0;
  double tuned_us = 0;
  // derived
  std::vector<FusedLayout> lays;
  std::vector<BatchPulse> pulses;
  std::vector<BatchItem> items;
  // Lifting passes of the tiled pulses: pass k lifts levels
  // k*lift_depth + 1 .. (k+1)*lift_depth of every pulse that has them.
  std::vector<LiftBlock> blocks;     // grouped by pass
  int block_off[kMaxLevels + 1] = {0};
  int nblocks[kMaxLevels + 1] = {0};
  size_t pass_lds[kMaxLevels + 1] = {0};
  int npass = 0;
  int Jmax = 0, n_fused = 0, n_tiles = 0, grid = 0;
  size_t lds_bytes = 0;
  // Items run in up to three persistent launches, in this order: whole-pulse
  // items (general kernel), tile items whose layout needs more LDS than two
  // workgroups per CU allow, the remaining tile items (tile-only kernel, two
  // or more workgroups per CU).  cls_n / cls_grid / cls_lds per class.
  int cls_n[3] = {0, 0, 0}, cls_grid[3] = {0, 0, 0};
  size_t cls_lds[3] = {0, 0, 0};
  long long scratch_elems = 0;
  // device
  PlanDesc *d_plans = nullptr;
  size_t c_plans = 0;
  FusedLayout *d_lays = nullptr;
  size_t c_lays = 0;
  BatchPulse *d_pulses = nullptr;
  size_t c_pulses = 0;
  BatchItem *d_items = nullptr;
  size_t c_items = 0;
  LiftBlock *d_blocks = nullptr;
  size_t c_blocks = 0;
  int *d_counter = nullptr;          // one work counter per item class
  // Per-pulse device pointers: staged through pinned host memory (so the
  // copy is asynchronous) and uploaded only when they change; up_done marks
  // the end of the last copy out of h_pulses.
  BatchPulse *h_pulses = nullptr;
  hipEvent_t up_done = nullptr;
  bool uploaded = false;
  float2 *d_scratch = nullptr;
  long long scratch_cap = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap_stream = nullptr;
};

namespace {

void drop_graph(sidwt_batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// LDS words a tile item of level l needs: the level's band windows and its
// staged weights (the tile layout's total is the largest over its levels).
int tile_level_words(const FusedLayout &L, int l) {
  const int row = 2 * (L.V[l][0] + L.V[l][1]);
  return std::max(2 * L.band_size[l], L.w_at[l] + std::min(L.pc[l], 1 << l) * row);
}

double item_cost(const PlanDesc &d, const BatchItem &it, int N, const FusedLayout &lay) {
  if (it.kind == 0) {
    double c = 0;
    for (int l = 1; l <= d.J; ++l) c += 8.0 * N * (d.lv[l].len[0] + d.lv[l].len[1]);
    return c;
  }
  const int l = it.level;
  return 8.0 * it.rows * lay.T[l] * (1 << l) * (d.lv[l].len[0] + d.lv[l].len[1]);
}

// Rebuild work list, layouts and device descriptors for the current
// configuration.
int build(sidwt_batch *b) {
  drop_graph(b);
  b->lays.clear();
  b->pulses.assign(b->count, BatchPulse{});
  b->uploaded = false;
  b->items.clear();
  b->blocks.clear();
  std::vector<std::vector<LiftBlock>> per_pass(kMaxLevels + 1);
  std::vector<size_t> pass_lds(kMaxLevels + 1, 0);
  std::map<std::tuple<int, long long, int>, int> lay_index;  // (plan, N, kind)
  long long scratch = 0;
  size_t lds_words = 0;
  b->Jmax = 0;
  b->n_fused = b->n_tiles = 0;
  std::vector<std::pair<double, BatchItem>> costed;
  std::vector<char> costed_cls;
  std::vector<int> costed_words;   // LDS words the item needs
  for (int i = 0; i < b->count; ++i) {
    const int pi = b->pulse_plan[i];
    const PlanDesc &d = b->plans[pi];
    const long long N = b->N[i];
    BatchPulse &p = b->pulses[i];
    p.n = b->n[i];
    p.N = (int)N;
    p.J = d.J;
    p.plan = pi;
    p.scratch = 0;
    b->Jmax = std::max(b->Jmax, d.J);
    FusedLayout lay;
    bool fused = N <= b->fused_max_N && make_layout(d, N, &lay) == 0;
    const int kind = fused ? 0 : 1;
    auto key = std::make_tuple(pi, N, kind);
    auto itl = lay_index.find(key);
    if (itl == lay_index.end()) {
      if (!fused && make_tile_layout(d, N, b->tile_window, &lay) != 0) return SIDWT_E_UNSUPPORTED;
      lay_index[key] = (int)b->lays.size();
      b->lays.push_back(lay);
      lds_words = std::max<size_t>(lds_words, lay.total);
      itl = lay_index.find(key);
    }
    p.layout = itl->second;
    const FusedLayout &L = b->lays[p.layout];
    if (fused) {
      BatchItem it{};
      it.kind = 0;
      it.pulse = i;
      costed.push_back({item_cost(d, it, (int)N, L), it});
      costed_words.push_back(L.total);
      costed_cls.push_back(0);
      ++b->n_fused;
    } else {
      p.scratch = scratch;
      scratch += 2 * N;
      for (int l = 1; l <= d.J; ++l) {
        const int rows_l = (int)((N >> l) / L.T[l]);
        for (int r0 = 0; r0 < rows_l; r0 += L.rows[l]) {
          BatchItem it{};
          it.kind = 1;
          it.pulse = i;
          it.level = l;
          it.row0 = r0;
          it.rows = std::min(L.rows[l], rows_l - r0);
          costed.push_back({item_cost(d, it, (int)N, L), it});
          costed_words.push_back(tile_level_words(L, l));
          costed_cls.push_back(costed_words.back() > kLdsWordsTwoPerCu ? 1 : 2);
          ++b->n_tiles;
        }
      }
      for (int k = 0; k * b->lift_depth < d.J; ++k) {
        const int l0 = k * b->lift_depth + 1, l1 = std::min(d.J, (k + 1) * b->lift_depth);
        const int nb = lift_block_count((int)N, l0, l1);
        for (int blk = 0; blk < nb; ++blk) per_pass[k].push_back(LiftBlock{i, l0, l1, blk});
        pass_lds[k] = std::max(pass_lds[k], (size_t)lift_block_lds((int)N, l0, l1) * sizeof(float2));
      }
    }
  }
  // by class, each class longest first
  std::vector<int> order(costed.size());
  for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    if (costed_cls[x] != costed_cls[y]) return costed_cls[x] < costed_cls[y];
    return costed[x].first > costed[y].first;
  });
  size_t cls_words[3] = {0, 0, 0};
  for (int c = 0; c < 3; ++c) b->cls_n[c] = 0;
  for (int k : order) {
    const BatchItem &it = costed[k].second;
    const int c = costed_cls[k];
    ++b->cls_n[c];
    cls_words[c] = std::max<size_t>(cls_words[c], costed_words[k]);
    b->items.push_back(it);
  }
  b->npass = 0;
  for (int k = 0; k <= kMaxLevels; ++k) {
    b->block_off[k] = (int)b->blocks.size();
    b->nblocks[k] = (int)per_pass[k].size();
    b->pass_lds[k] = pass_lds[k];
    b->blocks.insert(b->blocks.end(), per_pass[k].begin(), per_pass[k].end());
    if (b->nblocks[k]) b->npass = k + 1;
  }
  b->scratch_elems = scratch;
  b->lds_bytes = std::max<size_t>(lds_words * 4, b->n_tiles ? kBalMinLdsBytes : 1024);
  // device side
  int rc = upload(&b->d_plans, &b->c_plans, b->plans);
  if (!rc) rc = upload(&b->d_lays, &b->c_lays, b->lays);
  if (!rc) rc = upload(&b->d_pulses, &b->c_pulses, b->pulses);
  if (!rc) rc = upload(&b->d_items, &b->c_items, b->items);
  if (!rc) rc = upload(&b->d_blocks, &b->c_blocks, b->blocks);
  if (rc) return rc;
  if (b->scratch_cap < std::max<long long>(1, scratch)) {
    if (b->d_scratch) (void)hipFree(b->d_scratch);
    b->d_scratch = nullptr;
    b->scratch_cap = 0;
    hipError_t e = hipMalloc(&b->d_scratch, (size_t)std::max<long long>(1, scratch) * sizeof(float2));
    if (e != hipSuccess) return map_err(e, "hipMalloc (scratch)");
    b->scratch_cap = std::max<long long>(1, scratch);
  }
  hipError_t e = batch_set_lds(b->lds_bytes);
  if (e != hipSuccess) return map_err(e, "hipFuncSetAttribute (LDS)");
  int cus = 0, dev = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return map_err(e, "device query");
  b->grid = 0;
  for (int c = 0; c < 3; ++c) {
    // tile classes: at least one partial-tile slot per wave (free below two
    // workgroups per CU, which the tile kernel's registers allow at most)
    b->cls_lds[c] = std::max<size_t>(cls_words[c] * 4, c > 0 ? kBalMinLdsBytes : 1024);
    b->cls_grid[c] = 0;
    if (b->cls_n[c] == 0) continue;
    int per_cu = 0;
    e = batch_occupancy(c > 0, b->cls_lds[c], &per_cu);
    if (e != hipSuccess) return map_err(e, "occupancy query");
    if (per_cu < 1) return SIDWT_E_UNSUPPORTED;
    b->cls_grid[c] = std::max(1, std::min<int>(per_cu * cus, b->cls_n[c]));
    b->grid = std::max(b->grid, b->cls_grid[c]);
  }
  return SIDWT_OK;
}

int enqueue(sidwt_batch *b, hipStream_t st) {
  const LiftBlock *block_ptr[kMaxLevels + 1];
  for (int k = 0; k <= kMaxLevels; ++k) block_ptr[k] = b->d_blocks + b->block_off[k];
  hipError_t e = launch_batch_reset(b->d_counter, 3, st);
  if (e == hipSuccess)
    e = launch_lift_passes(b->d_plans, b->d_pulses, block_ptr, b->nblocks, b->pass_lds, b->npass,
                           b->d_scratch, st);
  int first = 0;
  for (int c = 0; c < 3 && e == hipSuccess; ++c) {
    e = launch_batch_items(c > 0, b->d_plans, b->d_lays, b->d_pulses, b->d_items + first,
                           b->cls_n[c], b->d_counter + c, b->d_scratch, b->cls_grid[c],
                           b->cls_lds[c], st);
    first += b->cls_n[c];
  }
  return map_err(e, "kernel launch");
}

int ensure_graph(sidwt_batch *b) {
  if (b->exec) return SIDWT_OK;
  if (!b->cap_stream) {
    hipError_t e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return map_err(e);
  }
  hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return map_err(e, "hipStreamBeginCapture");
  int rc = enqueue(b, b->cap_stream);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(b->cap_stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return map_err(e, "hipStreamEndCapture");
  b->graph = g;
  e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    drop_graph(b);
    return map_err(e, "hipGraphInstantiate");
  }
  return SIDWT_OK;
}

int set_pointers(sidwt_batch *b, const void *const *rx, void *const *out, hipStream_t st) {
  bool same = b->uploaded;
  for (int i = 0; i < b->count; ++i) {
    if (!rx[i] || !out[i]) return SIDWT_E_INVAL;
    same = same && b->pulses[i].rx == rx[i] && b->pulses[i].out == out[i];
    b->pulses[i].rx = rx[i];
    b->pulses[i].out = out[i];
  }
  if (same) return SIDWT_OK;  // the device copy already holds these pointers
  const size_t bytes = b->pulses.size() * sizeof(BatchPulse);
  hipError_t e = hipSuccess;
  if (!b->h_pulses) e = hipHostMalloc((void **)&b->h_pulses, bytes, hipHostMallocDefault);
  if (e == hipSuccess && !b->up_done) e = hipEventCreateWithFlags(&b->up_done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventSynchronize(b->up_done);  // h_pulses is free again
  if (e != hipSuccess) return map_err(e, "pointer staging");
  std::memcpy(b->h_pulses, b->pulses.data(), bytes);
  e = hipMemcpyAsync(b->d_pulses, b->h_pulses, bytes, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipEventRecord(b->up_done, st);
  if (e != hipSuccess) return map_err(e, "hipMemcpyAsync (pointers)");
  b->uploaded = true;
  return SIDWT_OK;
}

int run(sidwt_batch *b, const void *const *rx, void *const *out, hipStream_t st, bool use_graph) {
  int rc = set_pointers(b, rx, out, st);
  if (rc) return rc;
  if (!use_graph) return enqueue(b, st);
  rc = ensure_graph(b);
  if (rc) return rc;
  return map_err(hipGraphLaunch(b->exec, st), "hipGraphLaunch");
}

// A batch over plan descriptors (equal pointers share one plan entry).
int create_from_descs(const PlanDesc *const *descs, const int64_t *n, int count,
                      sidwt_batch **out) {
  if (!descs || !n || !out || count < 1) return SIDWT_E_INVAL;
  sidwt_batch *b = new (std::nothrow) sidwt_batch();
  if (!b) return SIDWT_E_NOMEM;
  b->count = count;
  std::map<const PlanDesc *, int> idx;
  for (int i = 0; i < count; ++i) {
    const PlanDesc *d = descs[i];
    if (!d || n[i] < 1) {
      delete b;
      return SIDWT_E_INVAL;
    }
    if (is_int_filter(d->filter)) {
      delete b;
      return SIDWT_E_UNSUPPORTED;
    }
    const int64_t N = transform_length(n[i], d->J);
    if ((N >> d->J) < 2) {
      delete b;
      return SIDWT_E_INVAL;
    }
    if (d->m > N || N > (int64_t(1) << 26)) {
      delete b;
      return SIDWT_E_SIZE;
    }
    auto it = idx.find(d);
    if (it == idx.end()) {
      it = idx.emplace(d, (int)b->plans.size()).first;
      b->plans.push_back(*d);
    }
    b->pulse_plan.push_back(it->second);
    b->n.push_back(n[i]);
    b->N.push_back(N);
    b->J.push_back(d->J);
  }
  hipError_t e = hipMalloc(&b->d_counter, 3 * sizeof(int));
  int rc = map_err(e);
  if (!rc) rc = build(b);
  if (rc) {
    sidwt_batch_free(b);
    return rc;
  }
  *out = b;
  return SIDWT_OK;
}

}  // namespace

// One-shot batch over plan descriptors (C++ linkage, for the FP32 bank path
// of the same library): runs without graph capture on `st`, synchronises it
// and frees the batch.
int sidwt_batch_oneshot(const sidwt::PlanDesc *const *descs, const int64_t *n,
                        const void *const *rx, void *const *out, int count, hipStream_t st) {
  if (!rx || !out) return SIDWT_E_INVAL;
  sidwt_batch *b = nullptr;
  int rc = create_from_descs(descs, n, count, &b);
  if (rc) return rc;
  rc = run(b, rx, out, st, false);
  if (!rc) rc = map_err(hipStreamSynchronize(st));
  sidwt_batch_free(b);
  return rc;
}

extern "C" {

int sidwt_batch_create(const sidwt_plan *const *plans, const int64_t *n, int count,
                       sidwt_batch **out) {
  if (!plans || !n || !out || count < 1) return SIDWT_E_INVAL;
  std::vector<const PlanDesc *> descs((size_t)count);
  int n_int = 0;
  for (int i = 0; i < count; ++i) {
    descs[i] = plans[i] ? sidwt_plan_desc(plans[i]) : nullptr;
    if (!descs[i]) return SIDWT_E_INVAL;
    n_int += is_int_filter(descs[i]->filter) ? 1 : 0;
  }
  if (n_int == 0) return create_from_descs(descs.data(), n, count, out);
  if (n_int != count) return SIDWT_E_INVAL;  // integer and float plans in one batch
  sidwt_batch *b = new (std::nothrow) sidwt_batch();
  if (!b) return SIDWT_E_NOMEM;
  b->count = count;
  const int rc = sidwt_int_batch_create(plans, n, count, &b->ib);
  if (rc) {
    delete b;
    return rc;
  }
  *out = b;
  return SIDWT_OK;
}

void sidwt_batch_free(sidwt_batch *b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  sidwt_int_batch_free(b->ib);
  drop_graph(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  (void)hipFree(b->d_plans);
  (void)hipFree(b->d_lays);
  (void)hipFree(b->d_pulses);
  (void)hipFree(b->d_items);
  (void)hipFree(b->d_blocks);
  (void)hipFree(b->d_counter);
  (void)hipFree(b->d_scratch);
  if (b->h_pulses) (void)hipHostFree(b->h_pulses);
  if (b->up_done) (void)hipEventDestroy(b->up_done);
  delete b;
}

int sidwt_batch_config(sidwt_batch *b, int64_t fused_max_N, int tile_window) {
  if (!b || fused_max_N < 0 || tile_window < 64 || tile_window > 32768) return SIDWT_E_INVAL;
  if (b->ib) return SIDWT_OK;  // integer batches have no split or window
  (void)hipDeviceSynchronize();
  b->fused_max_N = (int)std::min<int64_t>(fused_max_N, 1 << 20);
  b->tile_window = tile_window;
  return build(b);
}

int sidwt_batch_configure(sidwt_batch *b, int64_t fused_max_N, int tile_window, int lift_depth) {
  if (!b || lift_depth < 1 || lift_depth > 8) return SIDWT_E_INVAL;
  if (fused_max_N < 0 || tile_window < 64 || tile_window > 32768) return SIDWT_E_INVAL;
  b->lift_depth = lift_depth;
  return sidwt_batch_config(b, fused_max_N, tile_window);
}

int sidwt_batch_run(sidwt_batch *b, const void *const *rx, void *const *out, void *hip_stream) {
  if (!b || !rx || !out) return SIDWT_E_INVAL;
  if (b->ib) return sidwt_int_batch_run(b->ib, rx, out, static_cast<hipStream_t>(hip_stream));
  return run(b, rx, out, static_cast<hipStream_t>(hip_stream), true);
}

int sidwt_batch_tune(sidwt_batch *b, const void *const *rx, void *const *out, void *hip_stream) {
  if (!b || !rx || !out) return SIDWT_E_INVAL;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (b->ib) {  // nothing to tune: one run, so the outputs hold a result
    const int rc = sidwt_int_batch_run(b->ib, rx, out, st);
    return rc ? rc : map_err(hipStreamSynchronize(st), "integer batch");
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return SIDWT_E_DEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return SIDWT_E_DEVICE;
  }
  auto time_cfg = [&](int fmax, int window, int depth, double *us) -> int {
    b->fused_max_N = fmax;
    b->tile_window = window;
    b->lift_depth = depth;
    int rc = build(b);
    if (rc) return rc;
    rc = run(b, rx, out, st, true);  // warm-up (also builds the graph)
    if (rc) return rc;
    if (hipEventRecord(e0, st) != hipSuccess) return SIDWT_E_DEVICE;
    for (int k = 0; k < 2 && !rc; ++k) rc = run(b, rx, out, st, true);
    if (rc) return rc;
    hipError_t er = hipEventRecord(e1, st);
    if (er == hipSuccess) er = hipEventSynchronize(e1);
    if (er != hipSuccess) return map_err(er, "tuning run");
    float ms = 0;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return SIDWT_E_DEVICE;
    *us = 1e3 * ms / 2;
    return SIDWT_OK;
  };
  // Tile window first (with the default split and lifting depth), then the
  // fused/tiled split, then the levels per lifting pass.
  const int win_c[] = {1024, 2048, 3072, 4096, 6144};
  const int fmax_c[] = {0, 2048, 4096, 8192, 16384};
  const int depth_c[] = {1, 2, 3, 4, 6};
  int best_win = b->tile_window, best_fmax = b->fused_max_N, best_depth = 4;
  double best = 1e300;
  int rc = SIDWT_OK;
  for (int win : win_c) {
    double us;
    int r = time_cfg(4096, win, best_depth, &us);
    if (r == SIDWT_E_UNSUPPORTED) continue;
    if (r) { rc = r; break; }
    if (us < best) { best = us; best_win = win; best_fmax = 4096; }
  }
  for (int fmax : fmax_c) {
    if (rc || fmax == 4096) continue;
    double us;
    int r = time_cfg(fmax, best_win, best_depth, &us);
    if (r == SIDWT_E_UNSUPPORTED) continue;
    if (r) { rc = r; break; }
    if (us < best) { best = us; best_fmax = fmax; }
  }
  for (int depth : depth_c) {
    if (rc || depth == 4) continue;
    double us;
    int r = time_cfg(best_fmax, best_win, depth, &us);
    if (r == SIDWT_E_UNSUPPORTED) continue;
    if (r) { rc = r; break; }
    if (us < best) { best = us; best_depth = depth; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  b->fused_max_N = best_fmax;
  b->tile_window = best_win;
  b->lift_depth = best_depth;
  b->tuned = 1;
  b->tuned_us = best;
  return build(b);
}

int sidwt_batch_info(const sidwt_batch *b, int64_t *v, int nv) {
  if (!b || !v || nv < 1) return SIDWT_E_INVAL;
  if (b->ib) {
    int64_t whole = 0, blocks = 0, fp64 = 0, scratch = 0;
    sidwt_int_batch_counts(b->ib, &whole, &blocks, &fp64, &scratch);
    const int64_t vals[] = {0, 0, b->count, whole + fp64, blocks, 0, 0, scratch, 0, 0, 1, 0};
    const int k = (int)(sizeof(vals) / sizeof(vals[0]));
    for (int i = 0; i < nv; ++i) v[i] = i < k ? vals[i] : 0;
    return SIDWT_OK;
  }
  const int64_t vals[] = {b->fused_max_N, b->tile_window, (int64_t)b->items.size(), b->n_fused,
                          b->n_tiles, (int64_t)b->lds_bytes, b->grid,
                          b->scratch_elems * (int64_t)sizeof(float2), b->tuned,
                          (int64_t)(b->tuned_us + 0.5), b->lift_depth, b->npass};
  const int k = (int)(sizeof(vals) / sizeof(vals[0]));
  for (int i = 0; i < nv; ++i) v[i] = i < k ? vals[i] : 0;
  return SIDWT_OK;
}

int sidwt_correlate_batch(const sidwt_plan *const *plans, const void *const *rx, const int64_t *n,
                          void *const *out, int count, void *hip_stream) {
  if (!rx || !out) return SIDWT_E_INVAL;
  sidwt_batch *b = nullptr;
  int rc = sidwt_batch_create(plans, n, count, &b);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  rc = b->ib ? sidwt_int_batch_run(b->ib, rx, out, st) : run(b, rx, out, st, false);
  if (!rc) rc = map_err(hipStreamSynchronize(st));
  sidwt_batch_free(b);
  return rc;
}

}  // extern "C"
