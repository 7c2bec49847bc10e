// Reference-bank device descriptors (shared by sidwt_bank.hip and
// sidwt_bank.cpp).
#pragma once

#include "sidwt_device.hpp"

namespace sidwt {

// A bank level's (reference, phase) pairs c = e * 2^l + r are cut into
// column tiles of kBankTilePairs consecutive pairs.  A tile's split weights
// sit in one panel per band, in the order the MFMA B operand is read: for
// every step of 8 lag offsets, hi then lo, lane by lane, 4 words (offsets
// 4g .. 4g+3 of the step for lane group g = lane / 32, pair (lane % 32) / 2,
// column variant lane % 2).  Offsets past a pair's window hold zeros.
constexpr int kBankTilePairs = 16;
constexpr int kBankStepWords = 512;   // one step of one tile: 2 x 64 lanes x 4 words

struct BankTile {
  long long off[2];     // panel start per band (4-byte units)
  int steps[2];         // panel length per band (steps of 8 offsets)
};

// Work of one request and level: its lags are cut into blocks of 256 (the
// last may be shorter) and its tiles [0, ntiles) into groups of
// bank_tiles_per_item(rows) tiles; one work item per (block, gmul
// consecutive groups), numbered block-major within the segment (item k:
// block k / g_full, group k mod g_full; the last block's items follow);
// the launch's item list gives each workgroup its (segment, k).  An item
// loads its data window once and runs its groups one after another.
__host__ __device__ inline int bank_tiles_per_item(int rows) {
  return rows > 128 ? 4 : rows > 64 ? 8 : 16;
}

struct BankSeg {
  void *out;            // the request's output, E x J x N complex64
  long long scratch;    // complex offset of the request's pyramid in scratch
  long long item0;      // first item's position in segment order (host bookkeeping)
  int N, J, E, level;   // E: eligible references (the first E of the bank)
  int L, ntiles;
  int nblocks;          // row blocks, the last holding L - 256 (nblocks - 1) lags
  int g_full, g_last;   // items per full block / in the last block
  int wide;             // full blocks run 128 rows x 2 tiles per wave (else 64 x 4)
  int gmul;             // tile groups per item
  int pad_;
};

// Per (reference e, level l): 1 / weight scale.
struct BankRefLevel {
  float inv_scale;
  int len[2];           // phase filter length per band
  int pad_;
};

}  // namespace sidwt
