// cp_hist_bwd.hpp -- adjoint of the histogram model with respect to the bin
// masses (free variables: P is multilinear in them, as in Eq. 5).
//
// For one side (the minimum; the maximum sweeps the reflected histograms):
//   dP/dm_j(v) = (1/Delta_v) int_{bin j of v} prod_n S_n
//   dP/dm_j(n) = Q_n(e_j) + int_{bin j of n} pdf_v Kbar_j prod_{k!=n} S_k
// where Q_n(y) = int_0^y pdf_v prod_{k!=n} S_k (the part where all of bin j
// lies above x, dS_n/dm_j = 1) and Kbar_j(x) = (e_{j+1} - x)/Delta_n is the
// survival of bin j's kernel (x inside bin j).  The sweep of cp_hist.hpp
// carries Q_n and the running value of the current bin; when it crosses an
// edge of histogram n it writes that bin's entry; bins above the end of the
// sweep receive Q_n at the end, bins below the start 0.  Every sub-interval
// is integrated with 3-point Gauss-Legendre (integrands of degree <= 4).
//
// Every Jacobian entry of a side is written exactly once: the minimum side
// assigns, the maximum side (ACC) adds, so the buffer needs no clearing.
#pragma once

#include "cp_hist.hpp"
#include "cp_tiles.hpp"

namespace cp {

// Weighted Jacobian of one stencil's side into J:
// J[(slot * h + k) * EJ + sj], slots 0 = v, 1..4 = e, n, w, s; entries of
// absent neighbours are not written.  `rev` (max side): sweep bin j is mass
// index h-1-j.  Returns the side probability.
template <typename T, bool ACC>
__host__ __device__ T hist_side_jac(const HistLds<T>& L, int ev, const int (&en)[4], const bool (&pres)[4],
                                    bool rev, T hv, const T (&lo)[4], const T (&hi)[4], T g, T* J, int64_t EJ,
                                    int64_t sj) {
  const int h = L.h;
  auto put = [&](int slot, int j, T v) {
    const int64_t a = (int64_t)(slot * h + (rev ? h - 1 - j : j)) * EJ + sj;
    if (ACC)
      J[a] = cfma(g, v, J[a]);
    else
      J[a] = g * v;
  };
  T bmin = hv;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (pres[i]) bmin = tmin(bmin, hi[i]);
  if (!(bmin > T(0))) {
    if (!ACC) {
      for (int k = 0; k < h; ++k) put(0, k, T(0));
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (pres[i])
          for (int k = 0; k < h; ++k) put(1 + i, k, T(0));
    }
    return T(0);
  }
  const T big = hv + hv + T(1);
  const T dv = hv * L.ih, idv = T(h) * crcp(hv);
  int jv = 0;
  T nv = h > 1 ? dv : hv;
  T pv = L.mass(ev, 0, rev) * idv;
  HistCursor<T> c[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) hist_cursor_init(c[i], L, en[i], rev, lo[i], hi[i], pres[i], big);
  if (!ACC) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (pres[i])
        for (int k = 0; k < c[i].j; ++k) put(1 + i, k, T(0));  // bins entirely below x = 0
  }
  T Q[4] = {T(0), T(0), T(0), T(0)};
  T cur[4] = {T(0), T(0), T(0), T(0)};
  T curv = T(0), value = T(0);
  T x0 = T(0);
  const int maxit = 5 * (h + 1) + 2;
  for (int it = 0; it < maxit; ++it) {
    if (!(x0 < bmin)) break;
    T x1 = tmin(nv, bmin);
#pragma unroll
    for (int i = 0; i < 4; ++i) x1 = tmin(x1, c[i].nxt);
    const T mid = (x0 + x1) * T(0.5), hl = (x1 - x0) * T(0.5);
    T full = T(0), loo[4] = {T(0), T(0), T(0), T(0)}, kb[4] = {T(0), T(0), T(0), T(0)};
    T kin[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) kin[i] = (c[i].j >= 0 && c[i].j < h) ? c[i].id : T(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const T x = cfma(hl, T(GL<3>::x[k]), mid);
      const T w = T(GL<3>::w[k]);
      T S[4], K[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const T r = c[i].nxt - x;
        S[i] = cfma(c[i].slope, r, c[i].snx);
        K[i] = r * kin[i];
      }
      const T p01 = S[0] * S[1], p23 = S[2] * S[3];
      full = cfma(w, p01 * p23, full);
      const T wl0 = w * (S[1] * p23), wl1 = w * (S[0] * p23), wl2 = w * (p01 * S[3]), wl3 = w * (p01 * S[2]);
      loo[0] += wl0;
      loo[1] += wl1;
      loo[2] += wl2;
      loo[3] += wl3;
      kb[0] = cfma(wl0, K[0], kb[0]);
      kb[1] = cfma(wl1, K[1], kb[1]);
      kb[2] = cfma(wl2, K[2], kb[2]);
      kb[3] = cfma(wl3, K[3], kb[3]);
    }
    const T php = pv * hl;
    value = cfma(php, full, value);
    curv = cfma(hl, full, curv);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      Q[i] = cfma(php, loo[i], Q[i]);
      cur[i] = cfma(php, kb[i], cur[i]);
    }
    if (nv == x1 && jv < h - 1) {  // vertex bin boundary
      put(0, jv, curv * idv);
      curv = T(0);
      ++jv;
      nv = jv + 1 < h ? T(jv + 1) * dv : hv;
      pv = L.mass(ev, jv, rev) * idv;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {  // neighbour bin boundaries
      const int jo = c[i].j;
      if (hist_cursor_step(c[i], L, en[i], rev, x1, big)) {
        if (jo >= 0 && jo < h) put(1 + i, jo, cur[i]);
        cur[i] = Q[i];
      }
    }
    x0 = x1;
  }
  // close the open bins; bins above the end see the whole range below them
  put(0, jv, curv * idv);
  if (!ACC)
    for (int k = jv + 1; k < h; ++k) put(0, k, T(0));
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (!pres[i]) continue;
    const int j = c[i].j;
    if (j >= 0 && j < h) put(1 + i, j, cur[i]);
    for (int k = (j < 0 ? 0 : j + 1); k < h; ++k) put(1 + i, k, Q[i]);
  }
  return value;
}

// Both sides of one stencil (centre e in the staged tile, grid position
// (gy, gx)) into J; returns the probabilities; an invalid stencil writes NaN.
template <typename T>
__host__ __device__ void hist_stencil_jac(const HistLds<T>& L, const T* par, int EP, int PX, int e, int gy, int gx,
                                          int H, int W, T gmin, T gmax, T* J, int64_t EJ, int64_t sj, T& pmin,
                                          T& pmax) {
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
  pmin = hist_side_jac<T, false>(L, e, en, pres, false, hiv - lov, lo, hi, gmin, J, EJ, sj);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    lo[k] = hiv - par[EP + en[k]];
    hi[k] = hiv - par[en[k]];
  }
  pmax = hist_side_jac<T, true>(L, e, en, pres, true, hiv - lov, lo, hi, gmax, J, EJ, sj);
}

// Sweep tile for the per-field adjoint: 64 x TY stencils (params staged with a
// one-vertex halo), Jacobians written to the workspace J ([5][h][H][W]); a
// gather kernel then adds the five entries of every parameter.  If f.pmin is
// non-null the probabilities are written too (fused forward + adjoint).
template <typename T, int TY>
__device__ __forceinline__ void tile_hist_sweep(const FieldPtrs<T>& f, int ty0, int tx0, T* lds, int tid, T* J) {
  constexpr int TX = kFwdTX, EX = TX + 2, EY = TY + 2, E = EX * EY, NT = TX * TY;
  const int h = f.nb;
  stage<T, EY, EX, NT>(lds, f.params, 2 + h, f.ps, f.rs, f.H, f.W, ty0 - 1, tx0 - 1, tid);
  __syncthreads();
  hist_stage_validity<T, NT>(lds, E, h, tid);
  __syncthreads();
  const int lx = tid % TX, ly = tid / TX;
  const int x = tx0 + lx, y = ty0 + ly;
  if (x < f.W && y < f.H) {
    const HistLds<T> L{lds, E, h, T(1) / T(h)};
    const int64_t at = (int64_t)y * f.rs + x;
    const int64_t plane = (int64_t)f.H * f.W;
    T pmin, pmax;
    hist_stencil_jac(L, lds, E, EX, (ly + 1) * EX + lx + 1, y, x, f.H, f.W, f.gmin[at], f.gmax[at], J, plane,
                     (int64_t)y * f.W + x, pmin, pmax);
    if (f.pmin) {
      f.pmin[at] = pmin;
      f.pmax[at] = pmax;
    }
  }
  __syncthreads();
}

template <int OX, int OY>
__host__ __device__ constexpr size_t hist_bwd_lds_elems(int h) {
  return (size_t)hist_planes(h) * (OX + 4) * (OY + 4) + (size_t)5 * h * (OX + 2) * (OY + 2);
}

// Self-contained adjoint tile (Jacobians in LDS, same two phases as the
// uniform / Epanechnikov tile); used by the batched persistent kernel, which
// cannot wait for a second pass.  Also writes zeros into the lo / hi planes of
// the gradient, which are not differentiated.
template <typename T, int OX, int OY, int NT>
__device__ __forceinline__ void tile_bwd_hist(const FieldPtrs<T>& f, int ty0, int tx0, T* lds, int tid) {
  using G = BwdGeom<OX, OY>;
  const int h = f.nb;
  T* par = lds;
  T* J = lds + (size_t)hist_planes(h) * G::EP;
  stage<T, G::PY, G::PX, NT>(par, f.params, 2 + h, f.ps, f.rs, f.H, f.W, ty0 - 2, tx0 - 2, tid);
  for (int i = tid; i < 5 * h * G::EJ; i += NT) J[i] = T(0);  // ring stencils outside the grid
  __syncthreads();
  hist_stage_validity<T, NT>(par, G::EP, h, tid);
  __syncthreads();
  const HistLds<T> L{par, G::EP, h, T(1) / T(h)};
  for (int i = tid; i < G::EJ; i += NT) {
    const int ey = i / G::EX, ex = i - ey * G::EX;
    const int gy = ty0 - 1 + ey, gx = tx0 - 1 + ex;
    if (!(gy >= 0 && gy < f.H && gx >= 0 && gx < f.W)) continue;
    const int64_t at = (int64_t)gy * f.rs + gx;
    T pmin, pmax;
    hist_stencil_jac(L, par, G::EP, G::PX, (ey + 1) * G::PX + ex + 1, gy, gx, f.H, f.W, f.gmin[at], f.gmax[at], J,
                     (int64_t)G::EJ, (int64_t)i, pmin, pmax);
    if (f.pmin && ey >= 1 && ey <= OY && ex >= 1 && ex <= OX) {
      f.pmin[at] = pmin;
      f.pmax[at] = pmax;
    }
  }
  __syncthreads();
  for (int i = tid; i < OX * OY; i += NT) {
    const int oy = i / OX, ox = i - oy * OX;
    const int gy = ty0 + oy, gx = tx0 + ox;
    if (gy < f.H && gx < f.W) {
      const int c = (oy + 1) * G::EX + ox + 1;
      const int64_t at = (int64_t)gy * f.rs + gx;
      f.grad[at] = T(0);
      f.grad[f.ps + at] = T(0);
      for (int k = 0; k < h; ++k) {
        // own (slot v), east's w slot, west's e slot, north's s slot, south's n slot
        const T g = J[(0 * h + k) * G::EJ + c] + J[(3 * h + k) * G::EJ + c + 1] +
                    J[(1 * h + k) * G::EJ + c - 1] + J[(4 * h + k) * G::EJ + c - G::EX] +
                    J[(2 * h + k) * G::EJ + c + G::EX];
        f.grad[(int64_t)(2 + k) * f.ps + at] = g;
      }
    }
  }
  __syncthreads();
}

}  // namespace cp
