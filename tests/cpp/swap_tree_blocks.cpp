// Prints the block order of the roles-exchanged tree launches (host-visible
// code of the library): for each pulse count and level j given on stdin,
// every block index x of the count << j grid with the pulse and child phase
// it takes.  Checked by tests/test_swap_tree_blocks_cpu.py.
#include <cstdio>

#include "../../paper_cs_0607001_amd/csrc/sidwt_swap.hpp"

using namespace sidwt;

int main() {
  long long count;
  int j;
  while (std::scanf("%lld %d", &count, &j) == 2) {
    const long long G = count << j;
    std::printf("grid %lld %d\n", count, j);
    for (long long x = 0; x < G; ++x) {
      long long pulse;
      int p;
      swap_tree_block(x, G, j, pulse, p);
      std::printf("%lld %lld %d\n", x, pulse, p);
    }
  }
  return 0;
}
