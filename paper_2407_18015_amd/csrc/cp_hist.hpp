// cp_hist.hpp -- histogram model (Sec. 4.4.1): per-vertex sweep over the
// merged bin edges of the five stencil histograms.
//
// A histogram is a mixture of non-overlapping uniform kernels, so on every
// interval between consecutive edges of the five histograms the vertex pdf
// is constant and each neighbour's survival function is linear.  Eq. 5 sums
// the uniform-model probability over all h^5 kernel combinations; expanding
// that sum by linearity gives the same number as integrating
// pdf_v * prod S_n once over the merged edges, which costs O(5h) instead of
// O(h^5).  On each interval the product of four linear factors is integrated
// exactly from its end values (Bernstein form: the integral over [0,1] of
// t^k (1-t)^(4-k) is k!(4-k)!/5!), so every term is non-negative and no
// cancellation occurs.
//
// Staged per vertex in LDS (planes of the extended tile, E vertices each):
//   0 lo, 1 hi, 2..h+1 masses, h+2 zero.  An invalid histogram (lo >= hi,
// non-finite, negative mass) is marked by lo = NaN while staging.  The
// sweeps then replace the masses by their suffix sums U_j = m_j + ... +
// m_{h-1} (FP64 sums rounded once; U_h = 0 is the zero plane), so the
// survival at an edge is one read.
#pragma once

#include "cp_device.hpp"

namespace cp {

// staged planes per vertex: lo, hi, h masses (then suffix sums), one zero plane
__host__ __device__ constexpr int hist_planes(int h) { return h + 3; }

template <typename T>
struct HistLds {
  const T* base;
  int E;  // vertices per plane (extended tile)
  int h;
  T ih;   // 1 / h
  // mass j of vertex e; `rev` reads the histogram of -X (bins reversed)
  CP_HD T mass(int e, int j, bool rev) const {
    const int p = rev ? (1 + h - j) : (2 + j);
    return base[p * E + e];
  }
  CP_HD bool valid(int e) const { return base[e] == base[e]; }
};

// Validity marking of every staged histogram (lo := NaN when invalid).
template <typename T, int NT>
CP_HD void hist_stage_validity(T* lds, int E, int h, int tid) {
  for (int e = tid; e < E; e += NT) {
    const T lo = lds[e], hi = lds[E + e];
    const T d = hi - lo;
    bool ok = d > T(0) && d < T(3.0e38) && (lo - lo) == T(0);
    for (int j = 0; j < h; ++j) {
      const T m = lds[(2 + j) * E + e];
      ok = ok && m >= T(0) && m < T(3.0e38);
    }
    if (!ok) lds[e] = __builtin_nan("");
  }
}

// Integral over [0,1] of prod_{i<4} (f0_i (1-t) + f1_i t)
template <typename T>
CP_HD T bern4(const T (&f0)[4], const T (&f1)[4]) {
  T b0 = f0[0], b1 = f1[0];
  T c0 = b0 * f0[1], c1 = cfma(b0, f1[1], b1 * f0[1]), c2 = b1 * f1[1];
  T d0 = c0 * f0[2], d1 = cfma(c0, f1[2], c1 * f0[2]), d2 = cfma(c1, f1[2], c2 * f0[2]), d3 = c2 * f1[2];
  T e0 = d0 * f0[3], e1 = cfma(d0, f1[3], d1 * f0[3]), e2 = cfma(d1, f1[3], d2 * f0[3]),
    e3 = cfma(d2, f1[3], d3 * f0[3]), e4 = d3 * f1[3];
  return cfma(e2, T(1.0 / 30.0), cfma(e1 + e3, T(0.05), (e0 + e4) * T(0.2)));
}

}  // namespace cp

// ---------------------------------------------------------------------------
// Forward in one sweep: P_min and P_max of a vertex share the merged edges
// of the five histograms over the vertex range [0, hv], with F = T - S for
// every neighbour.  The staged masses are first replaced, per staged vertex,
// by their suffix sums U_j = m_j + ... + m_{h-1} (FP64 sums rounded once), so
// a neighbour's survival at an edge is one LDS read and crossing an edge
// costs one read, whatever the number of bins.
// ---------------------------------------------------------------------------
namespace cp {

// masses (planes 2..h+1) -> suffix sums U_0 .. U_{h-1}; U_0 = total mass;
// plane h+2 := 0 (U_h)
template <typename T, int NT>
CP_HD void hist_stage_suffix(T* lds, int E, int h, int tid) {
  for (int e = tid; e < E; e += NT) {
    double acc = 0.0;
    for (int j = h - 1; j >= 0; --j) {
      acc += (double)lds[(2 + j) * E + e];
      lds[(2 + j) * E + e] = (T)acc;
    }
    lds[(2 + h) * E + e] = T(0);
  }
}

template <typename T>
struct HistSuf {
  const T* base;
  int E, h;
  // U_j of vertex e, 0 <= j <= h (plane 2 + h is the staged zero plane, U_h)
  CP_HD T U(int e, int j) const { return base[(2 + j) * E + e]; }
};

// One neighbour in the vertex frame: survival S(x) = snx + slope (nxt - x)
// on the current bin; F = tot - S.  Its edges above the first are counted
// down from the last, hi - (h - k) Delta (k = h: hi itself), so the cursor
// keeps hi and not lo.
template <typename T>
struct SufCursor {
  int j;  // -1 below the range, h above it
  T hi, d, id, nxt, snx, slope, tot;
};

template <typename T>
CP_HD void suf_cursor_init(SufCursor<T>& c, const HistSuf<T>& L, int e, T lo, T hi, bool present, T big) {
  const int h = L.h;
  c.hi = hi;
  c.d = (hi - lo) * (T(1) / T(h));
  c.id = T(h) * crcp(hi - lo);
  if (!present) {  // constant factor 1 in both products
    c.j = h;
    c.nxt = big;
    c.snx = T(1);
    c.slope = T(0);
    c.tot = T(2);
    return;
  }
  c.tot = L.U(e, 0);
  if (!(lo < T(0))) {  // range starts at or after x = 0
    c.j = -1;
    c.nxt = lo;
    c.snx = c.tot;
    c.slope = T(0);
    return;
  }
  int j = (int)(-lo * c.id);
  j = j < 0 ? 0 : (j > h - 1 ? h - 1 : j);
  const auto edge = [&](int k) { return cfma(T(k - h), c.d, hi); };  // 1 <= k <= h
  if (j + 1 < h && !(edge(j + 1) > T(0))) ++j;
  if (j > 0 && edge(j) > T(0)) --j;
  c.j = j;
  c.nxt = edge(j + 1);
  const T uj = L.U(e, j);
  c.snx = L.U(e, j + 1);
  c.slope = (uj - c.snx) * c.id;
  if (!(hi > T(0))) {  // the whole range lies below x = 0
    c.j = h;
    c.nxt = big;
    c.snx = T(0);
    c.slope = T(0);
  }
}

// Cross the edge x1 if it is this cursor's next edge: one branch, and inside
// it no other (the next suffix sum is read from the zero plane once the
// cursor leaves the range, so survival and slope become 0 by themselves).
template <typename T>
CP_HD void suf_cursor_step(SufCursor<T>& c, const HistSuf<T>& L, int e, T x1, T big) {
  const int h = L.h;
  if (!(c.nxt == x1)) return;
  const int j1 = c.j + 1;  // the bin entered (h: past the range)
  const T prev = c.snx;
  c.snx = L.U(e, j1 + 1 < h ? j1 + 1 : h);
  c.slope = (prev - c.snx) * c.id;
  c.nxt = j1 >= h ? big : cfma(T(j1 + 1 - h), c.d, c.hi);
  c.j = j1;
}

// ---------------------------------------------------------------------------
// Branch-free cursor (the adjoint sweep): the same survival function as
// SufCursor, S(x) = snx + slope (nxt - x) on the current bin, F = tot - S, in
// a frame where the sweep runs from x = 0.  It holds the index m of its next
// edge (0 below the range, h + 1 past it); U_m is read from plane
// 2 + min(m, h) (the zero plane past the range), so no LDS index is kept; the
// edges are lo + m Delta for m < h and hi itself for m = h.  Every step is
// written with selects, so a wave whose lanes cross different edges runs one
// straight sequence of instructions.  The forward and saddle sweeps keep
// SufCursor: its branchy steps need fewer registers, and those sweeps gain
// more from occupancy than from fewer instructions.
// ---------------------------------------------------------------------------
template <typename T>
struct HistCursor {
  int m;   // index of the next edge (0 below the range, h + 1 past it)
  T nxt;   // next edge (big past the range)
  T snx;   // U_m: survival at the next edge
  T slope; // mass density of the current bin (0 outside the range)
  T tot, lo, hi, d, id;
  // inside the range (the current bin is a bin of this histogram)
  CP_HD bool in_range(int h) const { return (unsigned)(m - 1) < (unsigned)h; }
};

// `present` false: the constant factor 1 in both products (S = 1, F = 2 - 1)
template <typename T>
CP_HD void hist_cursor_init(HistCursor<T>& c, const T* base, int E, int h, int e, T lo, T hi, bool present, T big) {
  const T hf = T(h);
  c.lo = lo;
  c.hi = hi;
  c.d = (hi - lo) * (T(1) / hf);
  c.id = hf * crcp(hi - lo);
  c.slope = T(0);
  if (!present) {
    c.m = h + 1;
    c.nxt = big;
    c.snx = T(1);
    c.tot = T(2);
    return;
  }
  c.tot = base[2 * E + e];
  if (!(hi > T(0))) {  // the whole range lies at or below x = 0
    c.m = h + 1;
    c.nxt = big;
    c.snx = T(0);
    return;
  }
  if (!(lo < T(0))) {  // range starts at or after x = 0
    c.m = 0;
    c.nxt = lo;
    c.snx = c.tot;
    return;
  }
  int j = (int)(-lo * c.id);
  j = j < 0 ? 0 : (j > h - 1 ? h - 1 : j);
  const auto edge = [&](int k) { return k >= h ? hi : cfma(T(k), c.d, lo); };
  if (j + 1 < h && !(edge(j + 1) > T(0))) ++j;
  if (j > 0 && edge(j) > T(0)) --j;
  c.m = j + 1;
  c.nxt = edge(j + 1);
  c.snx = base[(3 + j) * E + e];
  c.slope = (base[(2 + j) * E + e] - c.snx) * c.id;
}

// Advance to the next edge if `adv` (selects, no branch); e is the
// histogram's LDS index in a plane.
template <typename T>
CP_HD void hist_cursor_step(HistCursor<T>& c, const T* base, int E, int e, int h, T big, bool adv) {
  const int m1 = c.m + 1;
  const T u1 = base[(2 + (m1 < h ? m1 : h)) * E + e];
  const T nx1 = m1 < h ? cfma(T(m1), c.d, c.lo) : (m1 == h ? c.hi : big);
  const T sl1 = (c.snx - u1) * c.id;
  c.m = adv ? m1 : c.m;
  c.snx = adv ? u1 : c.snx;
  c.slope = adv ? sl1 : c.slope;
  c.nxt = adv ? nx1 : c.nxt;
}

// The vertex's own bins over [0, hv]: bin jv, next edge nv (hv for the last
// bin, big past it), density pv, U above the bin uv; stepped with selects.
template <typename T>
struct VertexBins {
  int jv;
  T nv, pv, uv, dv, idv;
};

template <typename T>
CP_HD void vertex_bins_init(VertexBins<T>& b, const T* base, int E, int h, int ev, T hv) {
  b.dv = hv * (T(1) / T(h));
  b.idv = T(h) * crcp(hv);
  b.jv = 0;
  b.nv = h > 1 ? b.dv : hv;
  b.uv = base[3 * E + ev];
  b.pv = (base[2 * E + ev] - b.uv) * b.idv;
}

template <typename T>
CP_HD void vertex_bins_step(VertexBins<T>& b, const T* base, int E, int h, int ev, T hv, T big, bool adv) {
  const int jn = b.jv + 1;
  const T un = base[(jn + 3 < h + 2 ? jn + 3 : h + 2) * E + ev];  // U_{jn+1}
  const T pn = (b.uv - un) * b.idv;
  const T nn = jn + 1 < h ? T(jn + 1) * b.dv : (jn + 1 == h ? hv : big);
  b.jv = adv ? jn : b.jv;
  b.uv = adv ? un : b.uv;
  b.pv = adv ? pn : b.pv;
  b.nv = adv ? nn : b.nv;
}

// P_min and P_max of vertex ev; neighbour ranges [lo_i, hi_i] in the vertex
// frame (origin at the vertex lower end), vertex range [0, hv].  SAD: also
// the saddle terms t1 = int pdf_v S_e F_n S_w F_s and t2 = int pdf_v F_e S_n
// F_w S_s (Eq. 4) in the same sweep: on every merged sub-interval the four
// survival and distribution functions are the ones P_min and P_max use, so
// the two mixed products are two more exact Bernstein integrals (the caller
// keeps them only for vertices with all four neighbours).
template <typename T, bool SAD = false>
__host__ __device__ void hist_vertex_sweep(const HistSuf<T>& L, int ev, const int (&en)[4], const bool (&pres)[4],
                                           T hv, const T (&lo)[4], const T (&hi)[4], T& pmin, T& pmax, T& t1,
                                           T& t2) {
  const int h = L.h;
  const T big = hv + hv + T(1);
  const T dv = hv * (T(1) / T(h)), idv = T(h) * crcp(hv);
  int jv = 0;
  T nv = h > 1 ? dv : hv;
  T uv = L.U(ev, 1);               // U_{jv+1}
  T pv = (L.U(ev, 0) - uv) * idv;  // density of the vertex's bin jv
  SufCursor<T> c[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) suf_cursor_init(c[i], L, en[i], lo[i], hi[i], pres[i], big);
  // survival / distribution values at the current left end (sa, fa) and at
  // the next edge (sb, fb); the loop body takes two intervals with the roles
  // swapped, so no values are copied between intervals
  T sa[4], fa[4], sb[4], fb[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    sa[i] = cfma(c[i].slope, c[i].nxt, c[i].snx);
    fa[i] = c[i].tot - sa[i];
  }
  T x0 = T(0), amin = T(0), amax = T(0), a1 = T(0), a2 = T(0);
  const auto interval = [&](const T(&s0)[4], const T(&f0)[4], T(&s1)[4], T(&f1)[4]) {
    T x1 = nv;
#pragma unroll
    for (int i = 0; i < 4; ++i) x1 = fmin_nn(x1, c[i].nxt);  // sweep edges: finite
    const T wgt = pv * (x1 - x0);
#pragma unroll
    for (int i = 0; i < 4; ++i) suf_cursor_step(c[i], L, en[i], x1, big);
    // end values from the cursors after their steps (a cursor that crossed
    // x1 gives S(x1) from its new bin): the state before the step is dead by
    // now, so the steps update it in place
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      s1[i] = cfma(c[i].slope, c[i].nxt - x1, c[i].snx);
      f1[i] = c[i].tot - s1[i];
    }
    amin = cfma(wgt, bern4(s0, s1), amin);
    amax = cfma(wgt, bern4(f0, f1), amax);
    if constexpr (SAD) {
      const T m0[4] = {s0[0], f0[1], s0[2], f0[3]}, m1[4] = {s1[0], f1[1], s1[2], f1[3]};
      const T n0[4] = {f0[0], s0[1], f0[2], s0[3]}, n1[4] = {f1[0], s1[1], f1[2], s1[3]};
      a1 = cfma(wgt, bern4(m0, m1), a1);
      a2 = cfma(wgt, bern4(n0, n1), a2);
    }
    if (nv == x1) {
      ++jv;
      const T un = L.U(ev, jv + 1 < h ? jv + 1 : h);
      pv = (uv - un) * idv;
      uv = un;
      nv = jv + 1 < h ? T(jv + 1) * dv : hv;
    }
    x0 = x1;
  };
  const int maxit = 5 * (h + 1) + 2;  // every step crosses at least one edge
  for (int it = 0; it < maxit; it += 2) {
    if (!(x0 < hv)) break;
    interval(sa, fa, sb, fb);
    if (!(x0 < hv) || it + 1 >= maxit) break;
    interval(sb, fb, sa, fa);
  }
  pmin = amin;
  pmax = amax;
  t1 = a1;
  t2 = a2;
}

template <typename T>
__host__ __device__ void hist_vertex_minmax(const HistSuf<T>& L, int ev, const int (&en)[4], const bool (&pres)[4],
                                            T hv, const T (&lo)[4], const T (&hi)[4], T& pmin, T& pmax) {
  T t1, t2;
  hist_vertex_sweep<T, false>(L, ev, en, pres, hv, lo, hi, pmin, pmax, t1, t2);
}

}  // namespace cp
