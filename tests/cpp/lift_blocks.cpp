// Prints the block geometry of the uneven batch's multi-level lifting
// passes (host-visible code of the library): for each transform length N,
// scale count J and depth given on stdin, every pass and block with its
// computed ranges [s, e) and own ranges [os, oe) per level, and the LDS
// elements the pass is given.  Also prints the lifting reach (HL, HR, odd
// member before) of each float filter.  Checked by tests/test_lift_blocks_cpu.py.
#include <cstdio>

#include "../../paper_cs_0607001_amd/csrc/sidwt_device.hpp"

using namespace sidwt;

int main() {
  std::printf("reach %d %d %d %d %d %d %d %d %d\n", YLift<F_LEGALL53>::HL, YLift<F_LEGALL53>::HR,
              (int)YLift<F_LEGALL53>::kOddBefore, YLift<F_CDF97>::HL, YLift<F_CDF97>::HR,
              (int)YLift<F_CDF97>::kOddBefore, YLift<F_D4>::HL, YLift<F_D4>::HR,
              (int)YLift<F_D4>::kOddBefore);
  int N, J, D;
  while (std::scanf("%d %d %d", &N, &J, &D) == 3) {
    for (int k = 0; k * D < J; ++k) {
      const int l0 = k * D + 1, l1 = (k + 1) * D < J ? (k + 1) * D : J;
      const int nb = lift_block_count(N, l0, l1);
      std::printf("pass %d %d %d %d %d %d\n", N, l0, l1, nb, lift_block_lds(N, l0, l1),
                  (int)lift_block_whole(N, l0));
      for (int blk = 0; blk < nb; ++blk) {
        int s[kMaxLevels + 1], e[kMaxLevels + 1], os[kMaxLevels + 1], oe[kMaxLevels + 1];
        lift_block_ranges(N, l0, l1, blk, s, e, os, oe);
        std::printf("block %d", blk);
        for (int l = l0 - 1; l <= l1; ++l) std::printf(" %d %d %d %d", s[l], e[l], os[l], oe[l]);
        std::printf("\n");
      }
    }
  }
  return 0;
}
