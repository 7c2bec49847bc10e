// Prints the integer plan's exactness bounds as the library computes them
// (host planning code only): for J, the reference length m and its peak
// component, one line per level l = 1..J with the level l-1 approximation
// bounds of the pulse and the reference, the stored support lengths of both
// bands, the bound on the partial sums of that level's outputs, and whether
// the plan would be accepted.
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "../../paper_cs_0607001_amd/csrc/sidwt_host.hpp"

using namespace sidwt;
using namespace sidwt::host;

int main(int argc, char **argv) {
  if (argc != 4) {
    std::fprintf(stderr, "usage: %s J m peak\n", argv[0]);
    return 2;
  }
  const int J = std::atoi(argv[1]), m = std::atoi(argv[2]), peak = std::atoi(argv[3]);
  if (J < 1 || J > kMaxLevels || m < 1) return 2;
  PlanDesc d;
  std::memset(&d, 0, sizeof(d));
  d.filter = F_LEGALL53_INT;
  d.J = J;
  d.m = m;
  plan_windows(F_LEGALL53_INT, J, m, &d);
  double xp[kMaxLevels + 1], xr[kMaxLevels + 1];
  int_level_bounds(d, peak, xp, xr);
  for (int l = 1; l <= J; ++l)
    std::printf("%d %.17g %.17g %d %d %.17g\n", l, xp[l - 1], xr[l - 1], d.lv[l].len[0],
                d.lv[l].len[1], int_level_sum_bound(d, l, xp, xr));
  std::printf("exact %d\n", int_sums_exact(d, peak) ? 1 : 0);
  return 0;
}
