// Lifting factorization of a two-channel analysis filter pair (Sec. III-A,
// eq. (16): the Euclidean algorithm on the polyphase components of the
// lowpass, then one last step for the highpass).  Host code.
//
// Filters are given by taps: out[k] = sum_i c_i u[2k + i].  With e[k] =
// u[2k] and o[k] = u[2k + 1], the analysis is [c; d] = M(z) [e; o] where z
// advances a sequence (z e[k] = e[k + 1]) and
//   M = [[H_e, H_o], [G_e, G_o]],  H_e = sum_j c_{2j} z^j,  H_o = sum_j c_{2j+1} z^j.
// The factorization M = diag(K_e z^{s_e}, K_o z^{s_o}) T_m ... T_1 has
// elementary steps T = [[1, 0], [q, 1]] (predict: o += q(z) e) or
// [[1, q], [0, 1]] (update: e += q(z) o), applied T_1 first.  Each Euclid
// division a = q b + r is balanced: q cancels the lowest and highest terms
// of a in equal number, so symmetric filters give symmetric steps.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/sidwt.h"
#include "sidwt_factor.hpp"

namespace {

struct Poly {
  int lo = 0;                  // exponent of c[0]
  std::vector<double> c;       // coefficients of z^lo, z^(lo+1), ...
  bool zero() const { return c.empty(); }
  int width() const { return (int)c.size() - 1; }
};

double max_abs(const Poly &p) {
  double m = 0;
  for (double v : p.c) m = std::max(m, std::fabs(v));
  return m;
}

// Drop coefficients below tol at both ends.
void trim(Poly &p, double tol) {
  size_t b = 0, e = p.c.size();
  while (b < e && std::fabs(p.c[b]) <= tol) ++b;
  while (e > b && std::fabs(p.c[e - 1]) <= tol) --e;
  std::vector<double> c(p.c.begin() + b, p.c.begin() + e);
  p.lo += (int)b;
  p.c.swap(c);
  if (p.c.empty()) p.lo = 0;
}

Poly mul(const Poly &a, const Poly &b) {
  Poly r;
  if (a.zero() || b.zero()) return r;
  r.lo = a.lo + b.lo;
  r.c.assign(a.c.size() + b.c.size() - 1, 0.0);
  for (size_t i = 0; i < a.c.size(); ++i)
    for (size_t j = 0; j < b.c.size(); ++j) r.c[i + j] += a.c[i] * b.c[j];
  return r;
}

Poly sub(const Poly &a, const Poly &b) {
  if (b.zero()) return a;
  if (a.zero()) {
    Poly r = b;
    for (double &v : r.c) v = -v;
    return r;
  }
  Poly r;
  r.lo = std::min(a.lo, b.lo);
  const int hi = std::max(a.lo + a.width(), b.lo + b.width());
  r.c.assign(hi - r.lo + 1, 0.0);
  for (size_t i = 0; i < a.c.size(); ++i) r.c[a.lo - r.lo + i] += a.c[i];
  for (size_t i = 0; i < b.c.size(); ++i) r.c[b.lo - r.lo + i] -= b.c[i];
  return r;
}

// Balanced Laurent division: q such that a - q b keeps only a window of
// width(b) terms in the middle of a's span (width(a) >= width(b)).
Poly divide(const Poly &a, const Poly &b) {
  const int wa = a.width(), wb = b.width();
  const int nq = wa - wb + 1;
  const int k_low = nq / 2;
  Poly q;
  q.lo = a.lo - b.lo;
  q.c.assign(nq, 0.0);
  auto qb_at = [&](int p, int u_lo, int u_hi) {  // sum_u q[u] b[p - u] over u in [u_lo, u_hi]
    double s = 0;
    for (int u = u_lo; u <= u_hi; ++u) {
      const int bi = p - u;
      if (bi >= 0 && bi <= wb) s += q.c[u] * b.c[bi];
    }
    return s;
  };
  for (int t = 0; t < k_low; ++t)  // lowest k_low positions of a
    q.c[t] = (a.c[t] - qb_at(t, 0, t - 1)) / b.c[0];
  for (int t = 0; t < nq - k_low; ++t) {  // highest positions
    const int u = nq - 1 - t, p = wa - t;
    q.c[u] = (a.c[p] - qb_at(p, u + 1, nq - 1)) / b.c[wb];
  }
  return q;
}

}  // namespace

struct sidwt_lifting {
  sidwt::LiftingDesc d;
};

namespace sidwt {

int factorize(const double *lo, int lo_first, int lo_len, const double *hi, int hi_first,
              int hi_len, LiftingDesc *out) {
  std::memset(out, 0, sizeof(*out));
  auto split = [](const double *t, int first, int len, Poly &ev, Poly &od) {
    // tap i multiplies u[2k + i]: even i -> e[k + i/2], odd i -> o[k + (i-1)/2]
    int elo = 1 << 30, ehi = -(1 << 30), olo = 1 << 30, ohi = -(1 << 30);
    for (int n = 0; n < len; ++n) {
      const int i = first + n;
      const int j = (i - (i & 1)) / 2;
      if ((i & 1) == 0) elo = std::min(elo, j), ehi = std::max(ehi, j);
      else olo = std::min(olo, j), ohi = std::max(ohi, j);
    }
    if (elo <= ehi) ev.lo = elo, ev.c.assign(ehi - elo + 1, 0.0);
    if (olo <= ohi) od.lo = olo, od.c.assign(ohi - olo + 1, 0.0);
    for (int n = 0; n < len; ++n) {
      const int i = first + n;
      const int j = (i - (i & 1)) / 2;
      if ((i & 1) == 0) ev.c[j - ev.lo] += t[n];
      else od.c[j - od.lo] += t[n];
    }
  };
  Poly M[2][2];
  split(lo, lo_first, lo_len, M[0][0], M[0][1]);
  split(hi, hi_first, hi_len, M[1][0], M[1][1]);
  double scale = 0;
  for (auto &row : M)
    for (auto &p : row) scale = std::max(scale, max_abs(p));
  if (scale == 0) return SIDWT_E_INVAL;
  const double tol = 1e-11 * scale;
  for (auto &row : M)
    for (auto &p : row) trim(p, tol);
  // perfect reconstruction: the determinant must be a monomial
  Poly det = sub(mul(M[0][0], M[1][1]), mul(M[0][1], M[1][0]));
  trim(det, tol * scale);
  if (det.zero() || det.width() != 0) return SIDWT_E_INVAL;

  std::vector<std::pair<int, Poly>> steps;  // (kind, q)
  auto record = [&](int kind, Poly q) {
    trim(q, tol);
    if (!q.zero()) steps.emplace_back(kind, q);
  };
  for (int it = 0; it < 64 && !M[0][1].zero(); ++it) {
    Poly &a = M[0][0], &b = M[0][1];
    if (a.zero()) {
      // [0, b] -> [b, b] (col0 += col1) -> [b, 0] (col1 -= col0)
      Poly minus_one, one;
      minus_one.c = {-1.0};
      one.c = {1.0};
      for (int r = 0; r < 2; ++r) M[r][0] = sub(M[r][0], mul(minus_one, M[r][1]));
      record(kPredict, minus_one);
      for (int r = 0; r < 2; ++r) M[r][1] = sub(M[r][1], M[r][0]);
      record(kUpdate, one);
      for (auto &row : M)
        for (auto &p : row) trim(p, tol);
      continue;
    }
    if (a.width() >= b.width()) {
      Poly q = divide(a, b);  // col0 -= q col1; the step is o += q e
      for (int r = 0; r < 2; ++r) M[r][0] = sub(M[r][0], mul(q, M[r][1]));
      record(kPredict, q);
    } else {
      Poly q = divide(b, a);  // col1 -= q col0; the step is e += q o
      for (int r = 0; r < 2; ++r) M[r][1] = sub(M[r][1], mul(q, M[r][0]));
      record(kUpdate, q);
    }
    for (auto &row : M)
      for (auto &p : row) trim(p, tol);
  }
  if (!M[0][1].zero() || M[0][0].width() != 0 || M[1][1].width() != 0) return SIDWT_E_INVAL;
  // [[A, 0], [X, Y]] = diag(A, Y) [[1, 0], [X / Y, 1]]
  if (!M[1][0].zero()) {
    Poly t = M[1][0];
    t.lo -= M[1][1].lo;
    for (double &v : t.c) v /= M[1][1].c[0];
    record(kPredict, t);
  }
  if ((int)steps.size() > kMaxLiftSteps) return SIDWT_E_UNSUPPORTED;
  out->n = (int)steps.size();
  for (int s = 0; s < out->n; ++s) {
    const Poly &q = steps[s].second;
    if ((int)q.c.size() > kMaxLiftTaps) return SIDWT_E_UNSUPPORTED;
    out->kind[s] = steps[s].first;
    out->lo[s] = q.lo;
    out->len[s] = (int)q.c.size();
    for (size_t i = 0; i < q.c.size(); ++i) out->c[s][i] = q.c[i];
  }
  out->ke = M[0][0].c[0];
  out->se = M[0][0].lo;
  out->ko = M[1][1].c[0];
  out->so = M[1][1].lo;
  return SIDWT_OK;
}

}  // namespace sidwt

extern "C" {

int sidwt_lifting_factorize(const double *lo, int lo_first, int lo_len, const double *hi,
                            int hi_first, int hi_len, sidwt_lifting **out) {
  if (!out || !lo || !hi || lo_len < 1 || hi_len < 1 || lo_len > 64 || hi_len > 64 ||
      lo_first < -64 || lo_first > 64 || hi_first < -64 || hi_first > 64)
    return SIDWT_E_INVAL;
  *out = nullptr;
  sidwt_lifting *f = new (std::nothrow) sidwt_lifting();
  if (!f) return SIDWT_E_NOMEM;
  const int rc = sidwt::factorize(lo, lo_first, lo_len, hi, hi_first, hi_len, &f->d);
  if (rc) {
    delete f;
    return rc;
  }
  *out = f;
  return SIDWT_OK;
}

int sidwt_lifting_count(const sidwt_lifting *f) { return f ? f->d.n : SIDWT_E_INVAL; }

int sidwt_lifting_step(const sidwt_lifting *f, int i, int *kind, int *first, int *len,
                       double *coef) {
  if (!f || i < 0 || i >= f->d.n || !kind || !first || !len) return SIDWT_E_INVAL;
  *kind = f->d.kind[i];
  *first = f->d.lo[i];
  *len = f->d.len[i];
  if (coef)
    for (int t = 0; t < f->d.len[i]; ++t) coef[t] = f->d.c[i][t];
  return SIDWT_OK;
}

int sidwt_lifting_scaling(const sidwt_lifting *f, double *ke, int *se, double *ko, int *so) {
  if (!f || !ke || !se || !ko || !so) return SIDWT_E_INVAL;
  *ke = f->d.ke;
  *se = f->d.se;
  *ko = f->d.ko;
  *so = f->d.so;
  return SIDWT_OK;
}

void sidwt_lifting_free(sidwt_lifting *f) { delete f; }

}  // extern "C"

const sidwt::LiftingDesc *sidwt::lifting_desc(const sidwt_lifting *f) {
  return f ? &f->d : nullptr;
}
