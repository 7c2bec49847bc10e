// CPU emulation of the int8 matrix-core integer path, run against the
// oracle by tests/test_i8_emulation_cpu.py.  It uses the library's host
// planning code as it is (plan supports, digit panels, LDS layout) and
// mirrors the kernel's index arithmetic: the digit planes written from each
// level's bands, the units (32 rows x one column tile) of every level, the
// A rows read from the planes, the B lanes read from the panels, one int32
// sum per shift class, and the int64 output mapping.  Every plane and panel
// read is bounds-checked.  An MFMA is emulated as
//   D[row][col] += sum over lane group g and byte t of A(row, g)[t] B(col, g)[t].
//
// stdin: J N m, then the plan's pyramid (2 * elements int32, PlanDesc
// order), then for l = 1..J the pulse's bands c_l, d_l (2 * N/2^l int32
// each, (re, im) pairs).  stdout: "T l1 .. lJ", "WL w", then J*N*2 int64.
// Exit 3 on an out-of-bounds read.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../paper_cs_0607001_amd/csrc/sidwt_host.hpp"

using namespace sidwt;
using namespace sidwt::host;

static void fail(const char *what, long long a, long long b) {
  std::printf("OOB %s %lld %lld\n", what, a, b);
  std::exit(3);
}

int main(int argc, char **argv) {
  // "blocks": the long-pulse form (make_i8_tile_plan), every level's rows
  // in blocks whose digit windows start at their first row
  const bool blocks = argc > 1 && std::strcmp(argv[1], "blocks") == 0;
  int J, N, m;
  if (std::scanf("%d %d %d", &J, &N, &m) != 3) return 2;
  PlanDesc d;
  std::memset(&d, 0, sizeof(d));
  d.filter = F_LEGALL53_INT;
  d.J = J;
  d.m = m;
  const long long elems = plan_windows(F_LEGALL53_INT, J, m, &d);
  std::vector<int32_t> coef(2 * elems);
  for (auto &v : coef)
    if (std::scanf("%d", &v) != 1) return 2;
  long long maxabs = 0;
  for (int32_t v : coef) maxabs = std::max(maxabs, std::llabs((long long)v));
  const int WL = i8_weight_limbs(maxabs);
  if (!WL || !i8_data_fits(d)) return 4;
  std::vector<I8Tile> tiles;
  std::vector<int> tile_base;
  std::vector<signed char> panels;
  build_i8_panels(d, coef.data(), WL, &tiles, &tile_base, &panels);
  I8Layout lay;
  I8TilePlan tp;
  if (blocks) {
    if (make_i8_tile_plan(d, WL, tiles.data(), tile_base.data(), N, &tp) != 0) return 5;
    std::memset(&lay, 0, sizeof(lay));
    for (int l = 1; l <= J; ++l) {
      lay.T[l] = tp.T[l];
      lay.ntiles[l] = tp.ntiles[l];
      lay.tile_base[l] = tp.tile_base[l];
    }
    lay.plane_bytes = tp.plane_bytes;
  } else if (make_i8_layout(d, WL, tiles.data(), tile_base.data(), N, &lay) != 0) {
    return 5;
  }
  const int pb = lay.plane_bytes;
  std::vector<signed char> planes(2 * kI8DataLimbs * (size_t)pb, 0);
  std::vector<long long> out((size_t)J * N * 2, 0);
  std::printf("T");
  for (int l = 1; l <= J; ++l) std::printf(" %d", lay.T[l]);
  std::printf("\nWL %d\n", WL);
  for (int l = 1; l <= J; ++l) {
    const int L = N >> l, P = 1 << l, T = lay.T[l];
    std::vector<int32_t> band[2];
    for (int b = 0; b < 2; ++b) {
      band[b].resize(2 * (size_t)L);
      for (auto &v : band[b])
        if (std::scanf("%d", &v) != 1) return 2;
    }
    // row blocks of the level: one block of all rows in the fused form
    std::vector<I8Block> blist;
    if (blocks) {
      for (int q = 0; q < tp.nblocks; ++q)
        if (tp.blocks[q].level == l) blist.push_back(tp.blocks[q]);
    } else {
      blist.push_back(I8Block{l, 0, (L + T - 1) / T});
    }
    for (const I8Block &bk : blist) {
    std::fill(planes.begin(), planes.end(), 0);
    int ws[2], ext[2];
    for (int b = 0; b < 2; ++b) {
      if (blocks) {
        ws[b] = tp.ws[l][b] + T * bk.r0;   // window of the block, position 0 at row r0
        ext[b] = T * bk.rows + tp.K[l][b];
      } else {
        ws[b] = lay.ws[l][b];
        ext[b] = lay.ext[l][b];
      }
    }
    // digit planes, as put_digits writes them
    for (int b = 0; b < 2; ++b)
      for (int k = 0; k < L; ++k) {
        int xr = band[b][2 * k], xi = band[b][2 * k + 1];
        signed char dr[kI8DataLimbs], di[kI8DataLimbs];
        for (int a = 0; a < kI8DataLimbs; ++a) {
          const int r = ((xr + 128) & 255) - 128, i = ((xi + 128) & 255) - 128;
          xr = (xr - r) >> 8;
          xi = (xi - i) >> 8;
          dr[a] = (signed char)r;
          di[a] = (signed char)i;
        }
        if (xr || xi) fail("digits", band[b][2 * k], band[b][2 * k + 1]);
        for (int j = pos_mod(k - ws[b], L); j < ext[b]; j += L)
          for (int a = 0; a < kI8DataLimbs; ++a) {
            const size_t o = (size_t)(b * kI8DataLimbs + a) * pb + 2 * j;
            if (2 * j + 1 >= pb) fail("plane write", j, pb);
            planes[o] = dr[a];
            planes[o + 1] = di[a];
          }
      }
    // units, as correlate_i8_level runs them
    const int R = bk.rows, row0 = bk.r0, rtiles = (R + 31) >> 5, ctiles = lay.ntiles[l];
    const int NC = kI8DataLimbs + WL - 1;
    for (int unit = 0; unit < rtiles * ctiles; ++unit) {
      const int rt = unit % rtiles, ct = unit / rtiles;
      const I8Tile &t = tiles[lay.tile_base[l] + ct];
      std::vector<long long> acc((size_t)NC * 32 * 32, 0);
      for (int b = 0; b < 2; ++b)
        for (int c = 0; c < t.nch[b]; ++c)
          for (int a = 0; a < kI8DataLimbs; ++a)
            for (int w = 0; w < WL; ++w)
              for (int row = 0; row < 32; ++row)
                for (int col = 0; col < 32; ++col)
                  for (int g = 0; g < 2; ++g) {
                    const int p1 = std::min(rt * 32 + row, R - 1);
                    const long long pos = (long long)T * p1 + t.u0[b] + 8 * g + 16 * c;
                    if (pos < 0 || pos + 8 > ext[b]) fail("A position", pos, ext[b]);
                    const size_t ao = (size_t)(b * kI8DataLimbs + a) * pb + 2 * pos;
                    const int lane = 32 * g + col;
                    const long long bo = t.off[b] + (long long)(c * WL + w) * kI8ChunkBytes + 16 * lane;
                    if (bo < 0 || bo + 16 > (long long)panels.size()) fail("B", bo, panels.size());
                    long long sum = 0;
                    for (int q = 0; q < 16; ++q) sum += (long long)planes[ao + q] * panels[bo + q];
                    acc[((size_t)(a + w) * 32 + row) * 32 + col] += sum;
                  }
      for (int s = 0; s < NC; ++s)
        for (size_t q = 0; q < 32 * 32; ++q) {
          const long long v = acc[(size_t)s * 1024 + q];
          if (v >= (1LL << 31) || v < -(1LL << 31)) fail("int32 class sum", v, s);
        }
      for (int row = 0; row < 32; ++row) {
        const int pr = rt * 32 + row;
        if (pr >= R) continue;
        for (int col = 0; col < 32; ++col) {
          long long v = 0;
          for (int s = 0; s < NC; ++s) v += acc[((size_t)s * 32 + row) * 32 + col] << (8 * s);
          const long long si = (long long)T * P * (row0 + pr) + 16 * ct + (col >> 1);
          if (si < N) out[((size_t)(l - 1) * N + si) * 2 + (col & 1)] = v;
        }
      }
    }
    }  // blocks
  }
  for (long long v : out) std::printf("%lld\n", v);
  return 0;
}
