// cp_saddle.hpp -- saddle probability on the 4-neighbour stencil (Eq. 2 in
// 1-D, Eq. 4 in 2-D).  Under independence (Sec. 3)
//   t1 = Pr[v < e, v > n, v < w, v > s] = int pdf_v S_e F_n S_w F_s dx
//   t2 = Pr[v > e, v < n, v > w, v < s] = int pdf_v F_e S_n F_w S_s dx
// and P_saddle = t1 + t2 (interior vertices; the alternating pattern needs
// all four neighbours).  Task 1 for a saddle term (Sec. 4.1.3): the range is
// [a_max^alt, b_min^alt] = [max(a_v, a of the F factors), min(b_v, b of the
// S factors)], cut at the start points of the S factors and the end points of
// the F factors.  With the four cut points sorted, every factor is a
// polynomial or a constant on each of the five pieces, so a clamped
// evaluation of all four factors with the exact Gauss-Legendre rule of the
// full product degree integrates exactly.
#pragma once

#include "cp_device.hpp"
#include "cp_hist.hpp"
#include "cp_tiles.hpp"

namespace cp {

// neighbour index 0..3 = e, n, w, s; F factors of t1: n, s; of t2: e, w
CP_HD bool saddle_is_cdf(int term, int i) { return term == 0 ? (i & 1) : !(i & 1); }

// ---------------------------------------------------------------------------
// uniform: local frame with origin at the vertex lower end, vertex [0, Lv]
// ---------------------------------------------------------------------------
template <typename T>
CP_HD T uni_saddle_term(int term, T Lv, T iLv, const T (&a)[4], const T (&b)[4], const T (&iL)[4]) {
  T lo = T(0), hi = Lv;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (saddle_is_cdf(term, i))
      lo = tmax(lo, a[i]);
    else
      hi = tmin(hi, b[i]);
  }
  if (!(hi > lo)) return T(0);
  T c[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) c[i] = tclamp(saddle_is_cdf(term, i) ? b[i] : a[i], lo, hi);
  int tag[4] = {0, 1, 2, 3};
  T pay[4][1] = {{T(0)}, {T(0)}, {T(0)}, {T(0)}};
  sort4<T, 1>(c, pay, tag);
  const T e[6] = {lo, c[0], c[1], c[2], c[3], hi};
  T acc = T(0);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const T mid = (e[k] + e[k + 1]) * T(0.5), hl = (e[k + 1] - e[k]) * T(0.5);
    T sum = T(0);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const T x = cfma(hl, T(GL<3>::x[j]), mid);
      T prod = T(1);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        // S = (b - x) / L, F = (x - a) / L, each clamped to [0, 1]
        const T u = saddle_is_cdf(term, i) ? (x - a[i]) * iL[i] : (b[i] - x) * iL[i];
        prod *= tclamp(u, T(0), T(1));
      }
      sum = cfma(T(GL<3>::w[j]), prod, sum);
    }
    acc = cfma(sum, hl, acc);
  }
  return acc * iLv;
}

// ---------------------------------------------------------------------------
// Epanechnikov: origin at the vertex centre, vertex [-wv, wv]
// ---------------------------------------------------------------------------
template <typename T>
CP_HD T epa_saddle_term(int term, T wv, T iwv, const T (&d)[4], const T (&w)[4], const T (&iw)[4]) {
  T lo = -wv, hi = wv;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (saddle_is_cdf(term, i))
      lo = tmax(lo, d[i] - w[i]);
    else
      hi = tmin(hi, d[i] + w[i]);
  }
  if (!(hi > lo)) return T(0);
  T c[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) c[i] = tclamp(saddle_is_cdf(term, i) ? d[i] + w[i] : d[i] - w[i], lo, hi);
  int tag[4] = {0, 1, 2, 3};
  T pay[4][1] = {{T(0)}, {T(0)}, {T(0)}, {T(0)}};
  sort4<T, 1>(c, pay, tag);
  const T e[6] = {lo, c[0], c[1], c[2], c[3], hi};
  // F factors use F(u) = S(-u): evaluate S at the reflected argument
  T sg[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) sg[i] = saddle_is_cdf(term, i) ? T(-1) : T(1);
  T acc = T(0);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const T mid = (e[k] + e[k + 1]) * T(0.5), hl = (e[k + 1] - e[k]) * T(0.5);
    const T av = mid * iwv, bv = hl * iwv;
    T au[4], bu[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      au[i] = sg[i] * (mid - d[i]) * iw[i];
      bu[i] = sg[i] * hl * iw[i];
    }
    T sum = T(0);
#pragma unroll
    for (int j = 0; j < 7; ++j) {
      const T x = T(GL<7>::x[j]);
      const T t = cfma(bv, x, av);
      T prod = cfma(-t, t, T(1));
#pragma unroll
      for (int i = 0; i < 4; ++i) prod *= epa_s4(tclamp(cfma(bu[i], x, au[i]), T(-1), T(1)));
      sum = cfma(T(GL<7>::w[j]), prod, sum);
    }
    // The integrand has degree 14 when no factor is clamped on the piece
    // (each unclamped factor a cubic in x with leading coefficient bu^3, the
    // vertex kernel a quadratic with -bv^2), below that otherwise (a clamped
    // factor is constant): the 7-point rule misses only the x^14 term, which
    // is added in closed form.  A factor is clamped on the whole piece or
    // nowhere inside it (its clamp point is a breakpoint), so the midpoint
    // decides.
    T lead = -bv * bv;
#pragma unroll
    for (int i = 0; i < 4; ++i) lead *= fabs(au[i]) < T(1) ? bu[i] * bu[i] * bu[i] : T(0);
    sum = cfma(T(GLRem<7>::e), lead, sum);
    acc = cfma(sum, hl, acc);
  }
  return acc * T(0.75) * iwv * T(0.00390625);
}

// ---------------------------------------------------------------------------
// per-vertex evaluation from LDS (e = centre, en = e/n/w/s LDS indices)
// ---------------------------------------------------------------------------
template <typename T, int MODEL>
CP_HD bool stencil_valid_ue(const T* L, int E, int e, const int (&en)[4], const bool (&pres)[4]) {
  bool ok = MODEL == CP_UNIFORM ? valid_range(L[e], L[E + e]) : valid_epa(L[e], L[E + e]);
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (pres[i]) ok = ok && (MODEL == CP_UNIFORM ? valid_range(L[en[i]], L[E + en[i]]) : valid_epa(L[en[i]], L[E + en[i]]));
  return ok;
}

// Saddle terms of an interior vertex whose five distributions are valid.
template <typename T, int MODEL>
CP_HD void vertex_saddle_ue(const T* L, int E, int e, const int (&en)[4], T& t1, T& t2) {
  const T p0 = L[e], p1 = L[E + e];
  if (MODEL == CP_UNIFORM) {
    const T Lv = p1 - p0, iLv = crcp(Lv);
    T a[4], b[4], iL[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const T q0 = L[en[i]], q1 = L[E + en[i]];
      a[i] = q0 - p0;
      b[i] = q1 - p0;
      iL[i] = crcp(q1 - q0);
    }
    t1 = uni_saddle_term(0, Lv, iLv, a, b, iL);
    t2 = uni_saddle_term(1, Lv, iLv, a, b, iL);
  } else {
    const T iwv = crcp(p1);
    T d[4], w[4], iw[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      d[i] = L[en[i]] - p0;
      w[i] = L[E + en[i]];
      iw[i] = crcp(w[i]);
    }
    t1 = epa_saddle_term(0, p1, iwv, d, w, iw);
    t2 = epa_saddle_term(1, p1, iwv, d, w, iw);
  }
}

}  // namespace cp
