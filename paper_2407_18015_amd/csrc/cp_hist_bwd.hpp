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
// sweep receive Q_n at the end.  Every sub-interval is integrated with
// 3-point Gauss-Legendre (integrands of degree <= 4).
#pragma once

#include "cp_hist.hpp"
#include "cp_tiles.hpp"

namespace cp {

// Weighted Jacobian of one stencil's side, added into J.
// J layout: J[(slot * h + k) * EJ + sj], slots 0 = v, 1..4 = e, n, w, s.
// `rev` (max side): sweep bin j is mass index h-1-j of the original field.
// Returns the side probability.
template <typename T>
__host__ __device__ T hist_side_jac(const HistLds<T>& L, int ev, const int (&en)[4], const bool (&pres)[4], bool rev,
                           T hv, const T (&lo)[4], const T (&hi)[4], T g, T* J, int EJ, int sj) {
  const int h = L.h;
  T bmin = hv;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (pres[i]) bmin = tmin(bmin, hi[i]);
  if (!(bmin > T(0))) return T(0);
  const T big = hv + hv + T(1);
  const T dv = hv / T(h), idv = T(h) / hv;
  int jv = 0;
  T nv = h > 1 ? dv : hv;
  T pv = L.mass(ev, 0, rev) * idv;
  HistCursor<T> c[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) hist_cursor_init(c[i], L, en[i], rev, lo[i], hi[i], pres[i], big);
  T Q[4] = {T(0), T(0), T(0), T(0)};
  T cur[4] = {T(0), T(0), T(0), T(0)};
  T curv = T(0), value = T(0);
  auto jidx = [&](int slot, int j) { return (slot * h + (rev ? h - 1 - j : j)) * EJ + sj; };
  T x0 = T(0);
  const int maxit = 5 * (h + 1) + 2;
  for (int it = 0; it < maxit; ++it) {
    if (!(x0 < bmin)) break;
    T x1 = tmin(nv, bmin);
#pragma unroll
    for (int i = 0; i < 4; ++i) x1 = tmin(x1, c[i].nxt);
    const T mid = (x0 + x1) * T(0.5), hl = (x1 - x0) * T(0.5);
    T full = T(0), loo[4] = {T(0), T(0), T(0), T(0)}, kb[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const T x = cfma(hl, T(GL<3>::x[k]), mid);
      const T w = T(GL<3>::w[k]);
      T S[4], K[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const T r = c[i].nxt - x;
        S[i] = cfma(c[i].slope, r, c[i].snx);
        K[i] = (c[i].j >= 0 && c[i].j < h) ? r * c[i].id : T(0);
      }
      const T p01 = S[0] * S[1], p23 = S[2] * S[3];
      const T lo0 = S[1] * p23, lo1 = S[0] * p23, lo2 = p01 * S[3], lo3 = p01 * S[2];
      full = cfma(w, p01 * p23, full);
      const T wl0 = w * lo0, wl1 = w * lo1, wl2 = w * lo2, wl3 = w * lo3;
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
    // vertex bin boundary
    if (nv == x1 && jv < h - 1) {
      const int a = jidx(0, jv);
      J[a] = cfma(g, curv * idv, J[a]);
      curv = T(0);
      ++jv;
      nv = jv + 1 < h ? T(jv + 1) * dv : hv;
      pv = L.mass(ev, jv, rev) * idv;
    }
    // neighbour bin boundaries
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int jo = c[i].j;
      if (hist_cursor_step(c[i], L, en[i], rev, x1, big)) {
        if (jo >= 0 && jo < h) {
          const int a = jidx(1 + i, jo);
          J[a] = cfma(g, cur[i], J[a]);
        }
        cur[i] = Q[i];
      }
    }
    x0 = x1;
  }
  // close the open bins; bins above the end see the whole range below them
  {
    const int a = jidx(0, jv);
    J[a] = cfma(g, curv * idv, J[a]);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (!pres[i]) continue;
    int j = c[i].j;
    if (j >= 0 && j < h) {
      const int a = jidx(1 + i, j);
      J[a] = cfma(g, cur[i], J[a]);
    }
    for (int k = (j < 0 ? 0 : j + 1); k < h; ++k) {
      const int a = jidx(1 + i, k);
      J[a] = cfma(g, Q[i], J[a]);
    }
  }
  return value;
}

template <int OX, int OY>
__host__ __device__ constexpr size_t hist_bwd_lds_elems(int h) {
  return (size_t)hist_planes(h) * (OX + 4) * (OY + 4) + (size_t)5 * h * (OX + 2) * (OY + 2);
}

// Adjoint tile for histograms (same two phases as the uniform/Epanechnikov
// tile).  Also writes zeros into the lo / hi planes of the gradient, which are
// not differentiated.  If pmin is non-null the probabilities of the output
// vertices are written too (fused forward + adjoint).
template <typename T, int OX, int OY, int NT>
__device__ __forceinline__ void tile_bwd_hist(const FieldPtrs<T>& f, int ty0, int tx0, T* lds, int tid) {
  using G = BwdGeom<OX, OY>;
  const int h = f.nb;
  T* par = lds;
  T* J = lds + (size_t)hist_planes(h) * G::EP;
  stage<T, G::PY, G::PX, NT>(par, f.params, 2 + h, f.ps, f.rs, f.H, f.W, ty0 - 2, tx0 - 2, tid);
  for (int i = tid; i < 5 * h * G::EJ; i += NT) J[i] = T(0);
  __syncthreads();
  hist_stage_sums<T, NT>(par, G::EP, h, tid);
  __syncthreads();
  const HistLds<T> L{par, G::EP, h};
  for (int i = tid; i < G::EJ; i += NT) {
    const int ey = i / G::EX, ex = i - ey * G::EX;
    const int gy = ty0 - 1 + ey, gx = tx0 - 1 + ex;
    if (!(gy >= 0 && gy < f.H && gx >= 0 && gx < f.W)) continue;
    const int e = (ey + 1) * G::PX + ex + 1;
    const int en[4] = {e + 1, e - G::PX, e - 1, e + G::PX};
    const bool pres[4] = {gx + 1 < f.W, gy > 0, gx > 0, gy + 1 < f.H};
    bool ok = L.valid(e);
#pragma unroll
    for (int k = 0; k < 4; ++k) ok = ok && (!pres[k] || L.valid(en[k]));
    const int64_t at = (int64_t)gy * f.rs + gx;
    const bool inner = ey >= 1 && ey <= OY && ex >= 1 && ex <= OX;
    if (!ok) {
      for (int k = 0; k < 5 * h; ++k) J[k * G::EJ + i] = qnan<T>();
      if (f.pmin && inner) {
        f.pmin[at] = qnan<T>();
        f.pmax[at] = qnan<T>();
      }
      continue;
    }
    const T gmin = f.gmin[at], gmax = f.gmax[at];
    const T lov = par[e], hiv = par[G::EP + e];
    T lo[4], hi[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      lo[k] = par[en[k]] - lov;
      hi[k] = par[G::EP + en[k]] - lov;
    }
    const T pmin = hist_side_jac(L, e, en, pres, false, hiv - lov, lo, hi, gmin, J, G::EJ, i);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      lo[k] = hiv - par[G::EP + en[k]];
      hi[k] = hiv - par[en[k]];
    }
    const T pmax = hist_side_jac(L, e, en, pres, true, hiv - lov, lo, hi, gmax, J, G::EJ, i);
    if (f.pmin && inner) {
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
