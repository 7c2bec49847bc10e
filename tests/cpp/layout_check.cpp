// CPU-side audit of the fused kernel's LDS layouts: for a sweep of filters,
// scale counts, reference and pulse lengths, every layout the library would
// use must pass the bounds audit.  Prints one summary line per workload of
// interest.  Exit status 0 when no violation is found.
#include <cstdio>
#include <cstdlib>

#include "../../paper_cs_0607001_amd/csrc/sidwt_host.hpp"

using namespace sidwt;
using namespace sidwt::host;

static int check(int filter, int J, int m, long long n, bool verbose, long long *n_ok) {
  PlanDesc d;
  std::memset(&d, 0, sizeof(d));
  d.filter = filter;
  d.J = J;
  d.m = m;
  plan_windows(filter, J, m, &d);
  const long long N = transform_length(n, J);
  if ((N >> J) < 2 || m > N) return 0;
  if (filter == F_LEGALL53_INT && !int_support_fits(d, N)) return 0;
  int bad = 0;
  if (filter != F_LEGALL53_INT) {
    for (int window : {100, 1024, 2048, 3072, 4096, 8192}) {
      FusedLayout tl;
      if (make_tile_layout(d, N, window, &tl) != 0) continue;
      const int v = tile_layout_violation(d, tl);
      if (v) {
        std::printf("TILE VIOLATION %d: filter=%d J=%d m=%d n=%lld window=%d\n", v, filter, J, m,
                    n, window);
        bad = 1;
      } else {
        ++*n_ok;
      }
    }
  }
  FusedLayout lay;
  if (make_layout(d, N, &lay) != 0) return bad;  // long pulse: tiles only
  const int v = layout_violation(d, lay);
  if (v) {
    std::printf("VIOLATION %d: filter=%d J=%d m=%d n=%lld\n", v, filter, J, m, n);
    return 1;
  }
  ++*n_ok;
  // Balanced correlation (float filters): the helpers of every cut tile get
  // distinct partial-sum slots below fused_bal_slots(lay).  The tile count
  // is formed here as the correlation loop forms it (column chunks of pc).
  const int slots = fused_bal_slots(lay);
  if (filter != F_LEGALL53_INT) {
    for (int l = 1; l <= J; ++l) {
      const int P = 1 << l, L = (int)(N >> l);
      const int mtiles = (L / lay.T[l] + 31) / 32, mpairs = (mtiles + 1) / 2;
      int pcc = P;
      for (int r0 = 0; r0 < P; r0 += lay.pc[l]) pcc = std::min(lay.pc[l], P - r0);
      const int ntiles = mpairs * (P < 16 ? 1 : pcc / 16);
      const int NW = kFusedThreads / 64, rem = ntiles % NW;
      if (rem < 1 || rem > NW / 2) continue;
      const int c = NW / rem;
      bool seen[64] = {};
      for (int w = 0; w < rem * c; ++w) {
        if (w % c == 0) continue;  // the tile's owner keeps its sum in registers
        const int idx = (w / c) * (c - 1) + w % c - 1;
        if (idx < 0 || idx >= slots || seen[idx]) {
          std::printf("SLOT VIOLATION: filter=%d J=%d m=%d n=%lld level %d wave %d\n", filter, J,
                      m, n, l, w);
          return 1;
        }
        seen[idx] = true;
      }
    }
  }
  if (verbose)
    std::printf("filter=%d J=%d m=%d n=%lld N=%lld: LDS %d bytes (%s per CU), balanced +%d slots\n",
                filter, J, m, n, N, lay.total * 4, lay.total <= kLdsWordsTwoPerCu ? "2" : "1",
                slots);
  return bad;
}

int main() {
  long long ok = 0;
  int bad = 0;
  // workloads of interest
  bad += check(F_LEGALL53, 3, 256, 1024, true, &ok);
  bad += check(F_CDF97, 5, 512, 8192, true, &ok);
  bad += check(F_LEGALL53_INT, 6, 512, 4096, true, &ok);
  bad += check(F_D4, 9, 2048, 8192, true, &ok);
  bad += check(F_CDF97, 10, 2048, 16384, true, &ok);
  bad += check(F_CDF97, 5, 512, 4096, true, &ok);
  bad += check(F_CDF97, 5, 512, 2048, true, &ok);
  // sweep
  const int filters[] = {F_LEGALL53, F_CDF97, F_D4, F_LEGALL53_INT};
  const int ms[] = {1, 2, 5, 16, 37, 64, 100, 255, 512, 1000, 2048, 4096};
  for (int f : filters)
    for (int J = 1; J <= 13; ++J)
      for (int m : ms)
        for (long long n = 2; n <= 70000; n = n * 5 / 4 + 7) bad += check(f, J, m, n, false, &ok);
  std::printf("layouts checked: %lld, violations: %d\n", ok, bad);
  return bad ? 1 : 0;
}
