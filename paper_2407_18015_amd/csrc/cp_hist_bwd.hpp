// cp_hist_bwd.hpp -- adjoint of the histogram model with respect to the bin
// masses (free variables: P is multilinear in them, as in Eq. 5).
//
// One sweep over the vertex range integrates, for both P_min (prod S) and
// P_max (prod F = T - S), the leave-one-out products of every neighbour and
// their products with the survival function of the neighbour's current bin
// kernel, and emits each bin's weighted entry when the sweep leaves the bin.
// On every sub-interval all factors are linear, so the integrands are
// polynomials of degree <= 4: 2-point Gauss-Legendre plus the rule's
// remainder for the quartic terms, in closed form from the factors' slopes,
// integrates them exactly.  Entries of absent neighbours are not emitted.
//
// The sweep tile writes each stencil's entries to a workspace; a second
// kernel gathers every mass's five entries (no atomics).
#pragma once

#include "cp_hist.hpp"
#include "cp_tiles.hpp"

namespace cp {

// ---------------------------------------------------------------------------
// Both sides in one sweep over the vertex range [0, hv] (staged suffix sums):
//   dP_min/dm_j(v) = (1/Delta_v) int_{bin j of v} prod_n S_n
//   dP_max/dm_j(v) = (1/Delta_v) int_{bin j of v} prod_n F_n
//   dP_min/dm_j(n) = QS_n(e_j) + int_{bin j of n} pdf_v Kbar_j prod_{k!=n} S_k
//   dP_max/dm_j(n) = QF_n(hv) - QF_n(e_j) - int_{bin j of n} pdf_v Kbar_j prod_{k!=n} F_k
// with QS_n(y) = int_0^y pdf_v prod_{k!=n} S_k, QF_n likewise with F, and
// Kbar_j = (e_{j+1} - x)/Delta_n the survival function of bin j's kernel
// (dS_n/dm_j = Kbar_j, dF_n/dm_j = 1 - Kbar_j).  The upstream weights are
// folded into the accumulators (QS' = g_min QS, QF' = -g_max QF), so the
// entry of a neighbour bin is B + (1/Delta_n) int_{bin} (e_{j+1} - x)(lS + lF)
// with B = QS' + QF' at the bin's lower edge; it is emitted when the sweep
// leaves the bin, without the g_max QF_n(hv) term, which is known only at the
// end and belongs to every bin of the neighbour at or below the open one: it
// is stored once per neighbour (J.tail) and the gather adds it to all of the
// neighbour's bins, so the bins above the open one are emitted as
// QS_n(hv) - tail, those below the sweep as 0, and no entry is read back.  The node weights carry
// the vertex pdf and the half-length of the sub-interval, so the
// accumulators run over the whole sweep.
//
// Cursors as in the forward (HistCursor, VertexBins, staged layout of
// cp_hist.hpp); every sub-interval advances the cursors that end it with
// selects rather than branches.
//
// J must provide set(slot, k, value) and tail(i, value); slot 0 is the
// vertex's own histogram, slot 1 + i neighbour i (e, n, w, s).
// ---------------------------------------------------------------------------
template <typename T, typename JOut>
__host__ __device__ void hist_jac_both(const HistSuf<T>& L, int ev, const int (&en)[4], const bool (&pres)[4],
                                       T hv, const T (&lo)[4], const T (&hi)[4], T gmin, T gmax, JOut& J, T& pmin,
                                       T& pmax) {
  const int h = L.h, E = L.E;
  const T* base = L.base;
  const T hf = T(h);
  const T big = hv + hv + T(1);
  VertexBins<T> vb;
  vertex_bins_init(vb, base, E, h, ev, hv);
  HistCursor<T> c[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) hist_cursor_init(c[i], base, E, h, en[i], lo[i], hi[i], pres[i], big);
  // Y_n = B_n Delta_n + (kernel-weighted integral over the open bin so far):
  // the entry of a bin left is Y_n / Delta_n
  T QS[4], QF[4], Y[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) QS[i] = QF[i] = Y[i] = T(0);
  T vS = T(0), vF = T(0), amin = T(0), amax = T(0);
  T x0 = T(0);
  const int maxit = 5 * (h + 1) + 2;
  for (int it = 0; it < maxit; ++it) {
    if (!(x0 < hv)) break;
    T x1 = vb.nv;
#pragma unroll
    for (int i = 0; i < 4; ++i) x1 = fmin_nn(x1, c[i].nxt);  // sweep edges: finite
    const T mid = (x0 + x1) * T(0.5), hl = (x1 - x0) * T(0.5);
    const T php = vb.pv * hl, wS = php * gmin, wF = -php * gmax;
    // two-point Gauss-Legendre: exact for the leave-one-out products (degree
    // 3); the degree-4 integrands (full products, leave-one-out products times
    // the bin kernel) get the rule's remainder in closed form below.  One node
    // at a time (fewer registers live: the sweep needs occupancy).
    const T dx = hl * T(GL<2>::x[1]);
#pragma unroll 1
    for (int q = 0; q < 2; ++q) {
      const T x = q ? mid + dx : mid - dx;  // both weights 1
      T S[4], F[4], r[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        r[i] = c[i].nxt - x;
        S[i] = cfma(c[i].slope, r[i], c[i].snx);
        F[i] = c[i].tot - S[i];
      }
      const T s01 = S[0] * S[1], s23 = S[2] * S[3], f01 = F[0] * F[1], f23 = F[2] * F[3];
      vS = cfma(hl * s01, s23, vS);
      vF = cfma(hl * f01, f23, vF);
      const T ps01 = wS * s01, ps23 = wS * s23, pf01 = wF * f01, pf23 = wF * f23;
      const T ls[4] = {S[1] * ps23, S[0] * ps23, S[3] * ps01, S[2] * ps01};
      const T lf[4] = {F[1] * pf23, F[0] * pf23, F[3] * pf01, F[2] * pf01};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        QS[i] += ls[i];
        QF[i] += lf[i];
        Y[i] = cfma(ls[i] + lf[i], r[i], Y[i]);
      }
    }
    // The rule misses (8/45) hl^5 c4 of a quartic with leading coefficient
    // c4.  S_k has slope -s_k and F_k slope +s_k (s_k the cursor's density),
    // so c4 is s0 s1 s2 s3 for both full products, and pdf_v (g_min + g_max)
    // times the other three densities for an entry's kernel-weighted
    // integrand; in t_k = hl s_k (a change of S_k, bounded) no power of hl
    // or of a density is formed.
    {
      T t[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) t[i] = hl * c[i].slope;
      const T t01 = t[0] * t[1], t23 = t[2] * t[3];
      const T k45 = T(GLRem<2>::e) * hl;
      const T kv = k45 * (t01 * t23), ke = k45 * (wS - wF);
      vS += kv;
      vF += kv;
      const T lt[4] = {t[1] * t23, t[0] * t23, t[3] * t01, t[2] * t01};
#pragma unroll
      for (int i = 0; i < 4; ++i) Y[i] = cfma(ke, lt[i], Y[i]);
    }
    // vertex bin boundary: its entry is complete
    const bool advv = vb.nv == x1;
    if (advv && vb.jv < h) J.set(0, vb.jv, (gmin * vS + gmax * vF) * vb.idv);
    amin = advv ? cfma(vb.pv, vS, amin) : amin;
    amax = advv ? cfma(vb.pv, vF, amax) : amax;
    vS = advv ? T(0) : vS;
    vF = advv ? T(0) : vF;
    vertex_bins_step(vb, base, E, h, ev, hv, big, advv);
    // neighbour bin boundaries
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const bool adv = c[i].nxt == x1;
      // bin m - 1 is left; it is a bin of the range for 1 <= m <= h
      if (adv && c[i].in_range(h)) J.set(1 + i, c[i].m - 1, c[i].id * Y[i]);
      Y[i] = adv ? (QS[i] + QF[i]) * c[i].d : Y[i];
      hist_cursor_step(c[i], base, E, en[i], h, big, adv);
    }
    x0 = x1;
  }
  // remaining vertex bins (the sweep ended inside or past them): no range
  for (int k = vb.jv; k < h; ++k) J.set(0, k, (k == vb.jv) ? (gmin * vS + gmax * vF) * vb.idv : T(0));
  amin = cfma(vb.pv, vS, amin);
  amax = cfma(vb.pv, vF, amax);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (!pres[i]) continue;
    const int j = c[i].m - 1;  // open bin (-1: below the range, h: past it)
    const T tf = -QF[i];            // g_max QF_n(hv), added to every bin by the gather
    J.tail(i, tf);
    // first bin the sweep entered (the cursor's start, found again)
    HistCursor<T> c0;
    hist_cursor_init(c0, base, E, h, en[i], lo[i], hi[i], true, big);
    const int first = c0.m < 1 ? 0 : c0.m - 1;
    for (int k = 0; k < h; ++k) {
      if (k < first) {
        J.set(1 + i, k, T(0));  // entirely below the sweep: dF/dm = 1 there (the tail)
      } else if (k == j) {
        J.set(1 + i, k, c[i].id * Y[i]);  // the open bin: inside the range
      } else if (k > j) {
        J.set(1 + i, k, QS[i] - tf);  // entirely above the sweep: dS/dm = 1 there
      }  // first <= k < j: emitted when the sweep left the bin
    }
  }
  pmin = amin;
  pmax = amax;
}

// Entries of one stencil stored at J[(slot * h + k) * EJ + sj], its four
// tails at J[(5 h + i) * EJ + sj] (the workspace layout, [5 h + 4][H][W];
// also used by the host-side checks).  The plane size EJ (= H W) is below
// 2^30 (the descriptor check bounds the grid), so the plane offset is one
// 32 x 32 -> 64-bit product.
template <typename T>
struct JPlanes {
  T* J;
  uint32_t EJ;
  int64_t sj;
  int h;
  CP_HD int64_t at(int slot, int k) const { return (int64_t)((uint64_t)(uint32_t)(slot * h + k) * EJ) + sj; }
  CP_HD void set(int slot, int k, T v) const { J[at(slot, k)] = v; }
  CP_HD void tail(int i, T v) const { J[at(5, i)] = v; }  // plane 5 h + i
};


// Both sides of one stencil (centre e in the staged tile, grid position
// (gy, gx)) into J; returns the probabilities; an invalid stencil emits NaN
// for its own bins and those of its present neighbours.
template <typename T, typename JOut>
__host__ __device__ void hist_stencil_jac(const HistLds<T>& L, const HistSuf<T>& U, const T* par, int EP, int PX,
                                          int e, int gy, int gx, int H, int W, T gmin, T gmax, JOut& J, T& pmin,
                                          T& pmax) {
  const int h = L.h;
  const int en[4] = {e + 1, e - PX, e - 1, e + PX};
  const bool pres[4] = {gx + 1 < W, gy > 0, gx > 0, gy + 1 < H};
  bool ok = L.valid(e);
#pragma unroll
  for (int k = 0; k < 4; ++k) ok = ok && (!pres[k] || L.valid(en[k]));
  if (!ok) {
    for (int k = 0; k < h; ++k) J.set(0, k, qnan<T>());
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (pres[i]) {
        for (int k = 0; k < h; ++k) J.set(1 + i, k, qnan<T>());
        J.tail(i, T(0));
      }
    pmin = pmax = qnan<T>();
    return;
  }
  const T lov = par[e], hiv = par[EP + e];
  T lo[4], hi[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    lo[k] = par[en[k]] - lov;
    hi[k] = par[EP + en[k]] - lov;
  }
  hist_jac_both(U, e, en, pres, hiv - lov, lo, hi, gmin, gmax, J, pmin, pmax);
}

// Sweep tile of the adjoint: 64 x TY stencils (params staged with a
// one-vertex halo), entries written to the workspace J
// ([5 h + 4][H][W]: one plane per slot and bin, then the four tails, so the
// lanes of a wave that emit the same entry write consecutive words); a
// gather kernel then adds the five entries of every parameter.  If f.pmin is non-null the probabilities
// are written too (fused forward + adjoint).  NT threads; each takes the rows
// ly, ly + NT/64, ... of its column.
template <typename T, int TY, int NT = kFwdTX * TY>
__device__ __forceinline__ void tile_hist_sweep(const FieldPtrs<T>& f, int ty0, int tx0, T* lds, int tid, T* J) {
  constexpr int TX = kFwdTX, EX = TX + 2, EY = TY + 2, E = EX * EY;
  static_assert(NT % TX == 0 && TY % (NT / TX) == 0, "rows must split evenly over the threads");
  const int h = f.nb;
  stage<T, EY, EX, NT>(lds, f.params, 2 + h, f.ps, f.rs, f.H, f.W, ty0 - 1, tx0 - 1, tid);
  __syncthreads();
  hist_stage_validity<T, NT>(lds, E, h, tid);
  hist_stage_suffix<T, NT>(lds, E, h, tid);
  __syncthreads();
  const int lx = tid % TX, x = tx0 + lx;
  for (int ly = tid / TX; ly < TY; ly += NT / TX) {
    const int y = ty0 + ly;
    if (x < f.W && y < f.H) {
      const HistLds<T> L{lds, E, h, T(1) / T(h)};
      const HistSuf<T> U{lds, E, h};
      const int64_t at = (int64_t)y * f.rs + x;
      const int64_t sj = (int64_t)y * f.W + x;
      T pmin, pmax;
      JPlanes<T> Jo{J, (uint32_t)((int64_t)f.H * f.W), sj, h};
      hist_stencil_jac(L, U, lds, E, EX, (ly + 1) * EX + lx + 1, y, x, f.H, f.W, f.gmin[at], f.gmax[at], Jo, pmin,
                       pmax);
      if (f.pmin) {
        f.pmin[at] = pmin;
        f.pmax[at] = pmax;
      }
    }
  }
  __syncthreads();
}

// gather of the two-kernel adjoint: every mass of u adds its own stencil's
// entry and the entries of its four neighbours' stencils that refer to u
// (own, east's w slot, west's e slot, north's s slot, south's n slot)
template <typename T>
__device__ __forceinline__ void hist_gather_vertex(const FieldPtrs<T>& f, const T* __restrict__ J, int64_t id) {
  const int64_t plane = (int64_t)f.H * f.W;
  if (id >= plane) return;
  const int y = (int)(id / f.W), x = (int)(id - (int64_t)y * f.W);
  const int h = f.nb;
  const int64_t at = (int64_t)y * f.rs + x;
  f.grad[at] = T(0);
  f.grad[f.ps + at] = T(0);
  const auto e = [&](int64_t v, int slot, int k) { return J[(int64_t)(slot * h + k) * plane + v]; };
  // tails of the four stencils: u is the west (east, south, north) neighbour
  // of its east (west, north, south) neighbour
  const T te = x + 1 < f.W ? e(id + 1, 5, 2) : T(0), tw = x > 0 ? e(id - 1, 5, 0) : T(0);
  const T tn = y > 0 ? e(id - f.W, 5, 3) : T(0), ts = y + 1 < f.H ? e(id + f.W, 5, 1) : T(0);
  for (int k = 0; k < h; ++k) {
    T g = e(id, 0, k);
    if (x + 1 < f.W) g += e(id + 1, 3, k) + te;
    if (x > 0) g += e(id - 1, 1, k) + tw;
    if (y > 0) g += e(id - f.W, 4, k) + tn;
    if (y + 1 < f.H) g += e(id + f.W, 2, k) + ts;
    f.grad[(int64_t)(2 + k) * f.ps + at] = g;
  }
}

// The same gather for V = 16 / sizeof(T) vertices of one row per thread
// (W, the row stride and the plane stride multiples of V, grad 16-byte
// aligned): the own and north / south entries are aligned vector loads, the
// east / west ones the same vectors shifted by one vertex (4-byte aligned
// loads; at a row end the lane takes no entry, and every address stays
// inside the workspace: the shifted rows of slots 1 and 3, of the tail planes
// and the rows above / below of slots 4 and 2 lie between plane 1 and the
// last tail plane).  Terms are added in the scalar gather's order and absent
// ones skipped, so the sums are bit-identical to it.
template <typename T>
__device__ __forceinline__ void hist_gather_vec(const FieldPtrs<T>& f, const T* __restrict__ J, int64_t q) {
  constexpr int V = 16 / sizeof(T);
  typedef T Vec __attribute__((ext_vector_type(V)));
  const int64_t plane = (int64_t)f.H * f.W;
  const int64_t id = q * V;
  if (id >= plane) return;
  const int y = (int)(id / f.W), x = (int)(id - (int64_t)y * f.W);
  const int h = f.nb;
  const int64_t at = (int64_t)y * f.rs + x;
  const Vec z = Vec(T(0));
  *reinterpret_cast<Vec*>(f.grad + at) = z;
  *reinterpret_cast<Vec*>(f.grad + f.ps + at) = z;
  const bool hasn = y > 0, hass = y + 1 < f.H;
  const auto ld = [&](int slot, int k, int64_t v) {  // V entries from vertex v on (v 4-byte aligned)
    Vec r;
    __builtin_memcpy(&r, J + (int64_t)(slot * h + k) * plane + v, sizeof(Vec));
    return r;
  };
  const Vec te = ld(5, 2, id + 1), tw = ld(5, 0, id - 1);
  const Vec tn = ld(5, 3, hasn ? id - f.W : id), ts = ld(5, 1, hass ? id + f.W : id);
  for (int k = 0; k < h; ++k) {
    Vec g = *reinterpret_cast<const Vec*>(J + (int64_t)k * plane + id);
    const Vec e = ld(3, k, id + 1), w = ld(1, k, id - 1);
    const Vec n = ld(4, k, hasn ? id - f.W : id), s = ld(2, k, hass ? id + f.W : id);
#pragma unroll
    for (int j = 0; j < V; ++j) {
      T t = g[j];
      if (x + j + 1 < f.W) t += e[j] + te[j];
      if (x + j > 0) t += w[j] + tw[j];
      if (hasn) t += n[j] + tn[j];
      if (hass) t += s[j] + ts[j];
      g[j] = t;
    }
    *reinterpret_cast<Vec*>(f.grad + (int64_t)(2 + k) * f.ps + at) = g;
  }
}

}  // namespace cp
