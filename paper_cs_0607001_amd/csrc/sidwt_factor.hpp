// Lifting factorization of an analysis filter pair (eq. (16)): the step
// description shared by the host factorizer (sidwt_factor.cpp) and the
// generic lifting kernel (sidwt_generic.hip).
#pragma once

struct sidwt_lifting;

namespace sidwt {

constexpr int kMaxLiftSteps = 16;
constexpr int kMaxLiftTaps = 8;
constexpr int kPredict = 0;  // o += q(z) e
constexpr int kUpdate = 1;   // e += q(z) o

// Steps in the order they are applied; step s: q(z) = sum_t c[s][t]
// z^(lo[s] + t) (z advances: z v[k] = v[k + 1]).  Then c[k] = ke e[k + se],
// d[k] = ko o[k + so].
struct LiftingDesc {
  int n;
  int kind[kMaxLiftSteps];
  int lo[kMaxLiftSteps];
  int len[kMaxLiftSteps];
  double c[kMaxLiftSteps][kMaxLiftTaps];
  double ke, ko;
  int se, so;
};

int factorize(const double *lo, int lo_first, int lo_len, const double *hi, int hi_first,
              int hi_len, LiftingDesc *out);
const LiftingDesc *lifting_desc(const sidwt_lifting *f);

}  // namespace sidwt
