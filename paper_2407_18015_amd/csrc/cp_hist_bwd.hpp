// cp_hist_bwd.hpp -- adjoint of the histogram model with respect to the bin
// masses (free variables: P is multilinear in them, as in Eq. 5).
//
// One sweep over the vertex range integrates, for both P_min (prod S) and
// P_max (prod F = T - S), the leave-one-out products of every neighbour and
// their products with the survival / CDF of the current bin's kernel, and
// writes each bin's weighted entry when the sweep leaves the bin.  Every
// sub-interval is integrated with 3-point Gauss-Legendre (integrands of
// degree <= 4).  Entries of absent neighbours are not written.
#pragma once

#include "cp_hist.hpp"
#include "cp_tiles.hpp"

namespace cp {

// ---------------------------------------------------------------------------
// Both sides in one sweep over the vertex range [0, hv] (staged suffix sums):
//   dP_min/dm_j(v) = (1/Delta_v) int_{bin j of v} prod_n S_n
//   dP_max/dm_j(v) = (1/Delta_v) int_{bin j of v} prod_n F_n
//   dP_min/dm_j(n) = QS_n(e_j) + int_{bin j of n} pdf_v Kbar_j prod_{k!=n} S_k
//   dP_max/dm_j(n) = QF_n(hv) - QF_n(e_{j+1}) + int_{bin j of n} pdf_v K_j prod_{k!=n} F_k
// with QS_n(y) = int_0^y pdf_v prod_{k!=n} S_k, QF_n likewise with F, and
// Kbar_j = (e_{j+1} - x)/Delta_n, K_j = 1 - Kbar_j the survival / CDF of bin
// j's kernel.  The sweep writes g_min dP_min + g_max dP_max for a bin when it
// leaves it, without the g_max QF_n(hv) term, which is known only at the end:
// then the bins already written receive it (read-modify-write), the open bin
// and the bins above and below the sweep are written once.
// ---------------------------------------------------------------------------
template <typename T>
__host__ __device__ void hist_jac_both(const HistSuf<T>& L, int ev, const int (&en)[4], const bool (&pres)[4],
                                       T hv, const T (&lo)[4], const T (&hi)[4], T gmin, T gmax, T* J, int64_t EJ,
                                       int64_t sj, T& pmin, T& pmax) {
  const int h = L.h;
  auto at = [&](int slot, int k) { return (int64_t)(slot * h + k) * EJ + sj; };
  const T big = hv + hv + T(1);
  const T dv = hv * (T(1) / T(h)), idv = T(h) * crcp(hv);
  int jv = 0;
  T nv = h > 1 ? dv : hv;
  T uv = L.U(ev, 1);
  T pv = (L.U(ev, 0) - uv) * idv;
  SufCursor<T> c[4];
  int first[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    suf_cursor_init(c[i], L, en[i], lo[i], hi[i], pres[i], big);
    first[i] = c[i].j < 0 ? 0 : c[i].j;  // first bin the sweep enters
  }
  T QS[4] = {T(0), T(0), T(0), T(0)}, QF[4] = {T(0), T(0), T(0), T(0)};
  T QSin[4] = {T(0), T(0), T(0), T(0)};  // QS at the lower edge of the current bin
  T cS[4] = {T(0), T(0), T(0), T(0)}, cF[4] = {T(0), T(0), T(0), T(0)};
  T vS = T(0), vF = T(0), amin = T(0), amax = T(0);
  T x0 = T(0);
  const int maxit = 5 * (h + 1) + 2;
  for (int it = 0; it < maxit; ++it) {
    if (!(x0 < hv)) break;
    T x1 = nv;
#pragma unroll
    for (int i = 0; i < 4; ++i) x1 = tmin(x1, c[i].nxt);
    const T mid = (x0 + x1) * T(0.5), hl = (x1 - x0) * T(0.5);
    T fs = T(0), ff = T(0), ls[4], lf[4], ks[4], kf[4];
    T kin[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      ls[i] = lf[i] = ks[i] = kf[i] = T(0);
      kin[i] = (c[i].j >= 0 && c[i].j < h) ? c[i].id : T(0);
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const T x = cfma(hl, T(GL<3>::x[q]), mid);
      const T w = T(GL<3>::w[q]);
      T S[4], F[4], K[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const T r = c[i].nxt - x;
        S[i] = cfma(c[i].slope, r, c[i].snx);
        F[i] = c[i].tot - S[i];
        K[i] = r * kin[i];  // Kbar inside the current bin, 0 outside
      }
      const T s01 = S[0] * S[1], s23 = S[2] * S[3], f01 = F[0] * F[1], f23 = F[2] * F[3];
      fs = cfma(w, s01 * s23, fs);
      ff = cfma(w, f01 * f23, ff);
      const T wls[4] = {w * (S[1] * s23), w * (S[0] * s23), w * (s01 * S[3]), w * (s01 * S[2])};
      const T wlf[4] = {w * (F[1] * f23), w * (F[0] * f23), w * (f01 * F[3]), w * (f01 * F[2])};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        ls[i] += wls[i];
        lf[i] += wlf[i];
        ks[i] = cfma(wls[i], K[i], ks[i]);
        // K = 1 - Kbar inside the bin: kf accumulates wlf (K) as (inbin ? wlf - wlf Kbar : 0)
        kf[i] = kin[i] != T(0) ? cfma(-wlf[i], K[i], kf[i] + wlf[i]) : kf[i];
      }
    }
    const T php = pv * hl;
    amin = cfma(php, fs, amin);
    amax = cfma(php, ff, amax);
    vS = cfma(hl, fs, vS);
    vF = cfma(hl, ff, vF);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      QS[i] = cfma(php, ls[i], QS[i]);
      QF[i] = cfma(php, lf[i], QF[i]);
      cS[i] = cfma(php, ks[i], cS[i]);
      cF[i] = cfma(php, kf[i], cF[i]);
    }
    if (nv == x1) {  // vertex bin boundary: its entry is complete
      if (jv < h) J[at(0, jv)] = (gmin * vS + gmax * vF) * idv;
      vS = vF = T(0);
      ++jv;
      const T un = L.U(ev, jv + 1);
      pv = (uv - un) * idv;
      uv = un;
      nv = jv + 1 < h ? T(jv + 1) * dv : (jv + 1 == h ? hv : big);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {  // neighbour bin boundaries
      if (!(c[i].nxt == x1)) continue;
      const int jo = c[i].j;
      if (jo >= 0 && jo < h) J[at(1 + i, jo)] = gmin * (QSin[i] + cS[i]) + gmax * (cF[i] - QF[i]);
      QSin[i] = QS[i];
      cS[i] = cF[i] = T(0);
      suf_cursor_step(c[i], L, en[i], hi[i], x1, big);
    }
    x0 = x1;
  }
  // remaining vertex bins (the sweep ended inside or past them): no range
  for (int k = jv; k < h; ++k) J[at(0, k)] = (k == jv) ? (gmin * vS + gmax * vF) * idv : T(0);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (!pres[i]) continue;
    const int j = c[i].j;  // open bin (h: past the range)
    const T tf = gmax * QF[i];
    for (int k = 0; k < h; ++k) {
      if (k < first[i]) {
        J[at(1 + i, k)] = tf;  // entirely below the sweep: F = 1 there
      } else if (k < j) {
        J[at(1 + i, k)] += tf;  // written when the sweep left it
      } else if (k == j) {
        J[at(1 + i, k)] = gmin * (QSin[i] + cS[i]) + gmax * cF[i];
      } else {
        J[at(1 + i, k)] = gmin * QS[i];  // entirely above the sweep: S = 1 there
      }
    }
  }
  pmin = amin;
  pmax = amax;
}

// Both sides of one stencil (centre e in the staged tile, grid position
// (gy, gx)) into J; returns the probabilities; an invalid stencil writes NaN.
template <typename T>
__host__ __device__ void hist_stencil_jac(const HistLds<T>& L, const HistSuf<T>& U, const T* par, int EP, int PX,
                                          int e, int gy, int gx, int H, int W, T gmin, T gmax, T* J, int64_t EJ,
                                          int64_t sj, T& pmin, T& pmax) {
  const int h = L.h;
  const int en[4] = {e + 1, e - PX, e - 1, e + PX};
  const bool pres[4] = {gx + 1 < W, gy > 0, gx > 0, gy + 1 < H};
  bool ok = L.valid(e);
#pragma unroll
  for (int k = 0; k < 4; ++k) ok = ok && (!pres[k] || L.valid(en[k]));
  if (!ok) {
    for (int k = 0; k < h; ++k) J[(int64_t)k * EJ + sj] = qnan<T>();
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (pres[i])
        for (int k = 0; k < h; ++k) J[(int64_t)((1 + i) * h + k) * EJ + sj] = qnan<T>();
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
  hist_jac_both(U, e, en, pres, hiv - lov, lo, hi, gmin, gmax, J, EJ, sj, pmin, pmax);
}

// Sweep tile for the per-field adjoint: 64 x TY stencils (params staged with a
// one-vertex halo), Jacobians written to the workspace J ([5][h][H][W]); a
// gather kernel then adds the five entries of every parameter.  If f.pmin is
// non-null the probabilities are written too (fused forward + adjoint).  NT
// threads; each takes the rows ly, ly + NT/64, ... of its column.
template <typename T, int TY, int NT = kFwdTX * TY>
__device__ __forceinline__ void tile_hist_sweep(const FieldPtrs<T>& f, int ty0, int tx0, T* lds, int tid, T* J) {
  constexpr int TX = kFwdTX, EX = TX + 2, EY = TY + 2, E = EX * EY;
  static_assert(NT % TX == 0 && TY % (NT / TX) == 0, "rows must split evenly over the threads");
  const int h = f.nb;
  stage<T, EY, EX, NT>(lds, f.params, 2 + h, f.ps, f.rs, f.H, f.W, ty0 - 1, tx0 - 1, tid);
  __syncthreads();
  // validity, then masses -> suffix sums (the same thread owns each staged vertex)
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
      const int64_t plane = (int64_t)f.H * f.W;
      T pmin, pmax;
      hist_stencil_jac(L, U, lds, E, EX, (ly + 1) * EX + lx + 1, y, x, f.H, f.W, f.gmin[at], f.gmax[at], J, plane,
                       (int64_t)y * f.W + x, pmin, pmax);
      if (f.pmin) {
        f.pmin[at] = pmin;
        f.pmax[at] = pmax;
      }
    }
  }
  __syncthreads();
}

}  // namespace cp
