// cp_tiles.hpp -- tile-level routines shared by the per-field kernels and the
// batched persistent kernel.  A tile is a rectangle of output vertices; its
// parameters plus a halo are staged in LDS with coalesced row loads, then
// every thread evaluates its vertices from LDS.  All routines assume a 1-D
// block of NT threads and end with a barrier so the caller may reuse LDS.
#pragma once

#include "cp_device.hpp"
#include "cp_gauss.hpp"
#include "cp_hist.hpp"
#include "cpcrit.h"

namespace cp {

template <typename T>
struct FieldPtrs {
  const T* params;
  T* pmin;
  T* pmax;
  const T* gmin;
  const T* gmax;
  T* grad;
  int H, W, nb;
  int64_t rs, ps;  // row stride, plane stride (elements)
};

// Stage `np` planes of the rectangle [gy0, gy0+EY) x [gx0, gx0+EX) into LDS
// (plane-major, E = EY*EX per plane).  Cells outside the grid read as 0.
template <typename T, int EY, int EX, int NT>
__device__ __forceinline__ void stage(T* lds, const T* g, int np, int64_t ps, int64_t rs, int H, int W, int gy0,
                                      int gx0, int tid) {
  constexpr int E = EY * EX;
  for (int p = 0; p < np; ++p) {
    const T* gp = g + (int64_t)p * ps;
    for (int i = tid; i < E; i += NT) {
      const int ey = i / EX, ex = i - ey * EX;
      const int gy = gy0 + ey, gx = gx0 + ex;
      T v = T(0);
      if (gy >= 0 && gy < H && gx >= 0 && gx < W) v = gp[(int64_t)gy * rs + gx];
      lds[p * E + i] = v;
    }
  }
}

template <typename T>
CP_HD bool valid_range(T lo, T hi) {
  const T d = hi - lo;
  return d > T(0) && d < T(3.0e38) && (lo - lo) == T(0);
}
template <typename T>
CP_HD bool valid_epa(T m, T w) {
  return w > T(0) && w < T(3.0e38) && (m - m) == T(0);
}

// ---------------------------------------------------------------------------
// per-vertex evaluation from LDS (e = centre, en = e/n/w/s LDS indices)
// ---------------------------------------------------------------------------
template <typename T, int MODEL>
CP_HD void vertex_fwd_ue(const T* L, int E, int e, const int (&en)[4], const bool (&pres)[4],
                                              T& pmin, T& pmax) {
  const T p0 = L[e], p1 = L[E + e];
  T q0[4], q1[4];
  bool ok = MODEL == CP_UNIFORM ? valid_range(p0, p1) : valid_epa(p0, p1);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    q0[i] = L[en[i]];
    q1[i] = L[E + en[i]];
    if (pres[i]) ok = ok && (MODEL == CP_UNIFORM ? valid_range(q0[i], q1[i]) : valid_epa(q0[i], q1[i]));
  }
  if (!ok) {
    pmin = pmax = qnan<T>();
    return;
  }
  if (MODEL == CP_UNIFORM) {
    const T Lv = p1 - p0, iLv = crcp(Lv);
    T a[4], b[4], iL[4];
    UniSide<T> s;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a[i] = q0[i] - p0;
      b[i] = q1[i] - p0;
      iL[i] = crcp(q1[i] - q0[i]);
    }
    uni_setup(s, Lv, iLv, a, b, iL, pres);
    pmin = uni_side_value(s);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a[i] = p1 - q1[i];
      b[i] = p1 - q0[i];
    }
    uni_setup(s, Lv, iLv, a, b, iL, pres);
    pmax = uni_side_value(s);
  } else {
    T d[4], iw[4];
    const T iwv = crcp(p1);
    EpaSide<T> s;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      d[i] = q0[i] - p0;
      iw[i] = crcp(q1[i]);
    }
    epa_setup(s, p1, iwv, d, q1, iw, pres);
    pmin = epa_side_value(s);
#pragma unroll
    for (int i = 0; i < 4; ++i) d[i] = p0 - q0[i];
    epa_setup(s, p1, iwv, d, q1, iw, pres);
    pmax = epa_side_value(s);
  }
}

// Jacobian of one stencil, weighted by the upstream gradients:
// jac[slot*2 + q] = gmin dP_min/dtheta_q(slot) + gmax dP_max/dtheta_q(slot)
// WF: also return P_min, P_max (the Epanechnikov adjoint skips them otherwise).
// The stencil's parameters are passed by value: (p0, p1) of the vertex and
// (q0[i], q1[i]) of neighbour i (e, n, w, s), read only where pres[i].
template <typename T, int MODEL, bool WF = true>
CP_HD void vertex_jac_vals(T p0, T p1, const T (&q0)[4], const T (&q1)[4], const bool (&pres)[4], T gmin, T gmax,
                           T (&jac)[10], T& pmin, T& pmax) {
  bool ok = MODEL == CP_UNIFORM ? valid_range(p0, p1) : valid_epa(p0, p1);
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (pres[i]) ok = ok && (MODEL == CP_UNIFORM ? valid_range(q0[i], q1[i]) : valid_epa(q0[i], q1[i]));
  if (!ok) {
#pragma unroll
    for (int k = 0; k < 10; ++k) jac[k] = qnan<T>();
    pmin = pmax = qnan<T>();
    return;
  }
  if constexpr (MODEL == CP_GAUSSIAN) {
    gauss_vertex_jac<T>(p0, p1, q0, q1, pres, gmin, gmax, jac, pmin, pmax);
  } else if constexpr (MODEL == CP_UNIFORM) {
    const T Lv = p1 - p0, iLv = crcp(Lv);
    T a[4], b[4], iL[4];
    UniSide<T> s;
    UniGrad<T> g, r;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a[i] = q0[i] - p0;
      b[i] = q1[i] - p0;
      iL[i] = crcp(q1[i] - q0[i]);
    }
    uni_setup(s, Lv, iLv, a, b, iL, pres);
    uni_side_grad(s, g);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a[i] = p1 - q1[i];
      b[i] = p1 - q0[i];
    }
    uni_setup(s, Lv, iLv, a, b, iL, pres);
    uni_side_grad(s, r);
    T sg = T(0), sr = T(0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      sg += g.da[i] + g.db[i];
      sr += r.da[i] + r.db[i];
    }
    // min side, origin lo_v: a = lo_n - lo_v, b = hi_n - lo_v, Lv = hi_v - lo_v
    // max side, origin hi_v reflected: a = hi_v - hi_n, b = hi_v - lo_n
    pmin = g.f;
    pmax = r.f;
    jac[0] = gmin * (-g.dLv - sg) + gmax * (-r.dLv);
    jac[1] = gmin * g.dLv + gmax * (r.dLv + sr);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      jac[2 + 2 * i] = gmin * g.da[i] - gmax * r.db[i];
      jac[3 + 2 * i] = gmin * g.db[i] - gmax * r.da[i];
    }
  } else {
    T d[4], nd[4], iw[4];
    const T iwv = crcp(p1);
    EpaSide<T> s;
    EpaGrad<T> g, r;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      d[i] = q0[i] - p0;
      nd[i] = p0 - q0[i];
      iw[i] = crcp(q1[i]);
    }
    epa_setup<T>(s, p1, iwv, d, q1, iw, pres);
    epa_side_grad<T, WF>(s, g);
    epa_setup<T>(s, p1, iwv, nd, q1, iw, pres);
    epa_side_grad<T, WF>(s, r);
    // min side: d = m_n - m_v; max side: d = m_v - m_n; the vertex width
    // by scale invariance, summed in neighbour order (an absent neighbour's
    // derivatives are 0)
    T sg = T(0), sr = T(0), xg = T(0), xr = T(0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      sg += g.dd[i];
      sr += r.dd[i];
      xg = cfma(d[i], g.dd[i], cfma(q1[i], g.dw[i], xg));
      xr = cfma(nd[i], r.dd[i], cfma(q1[i], r.dw[i], xr));
    }
    pmin = g.f;
    pmax = r.f;
    jac[0] = -gmin * sg + gmax * sr;
    jac[1] = -(gmin * xg + gmax * xr) * iwv;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      jac[2 + 2 * i] = gmin * g.dd[i] - gmax * r.dd[i];
      jac[3 + 2 * i] = gmin * g.dw[i] + gmax * r.dw[i];
    }
  }
}

// ---------------------------------------------------------------------------
// forward tiles: 64 x TY outputs, halo 1; NT threads, each evaluating the
// rows ly, ly + NT/64, ... of its column (one row when NT = 64 TY)
// ---------------------------------------------------------------------------
constexpr int kFwdTX = 64;
// per-field forward / classification: 64 x 16 tiles (four rows per thread)
// once the grid gives at least this many of them (eight per CU), else 64 x 4
constexpr int kTallTileBlocks = 2048;

// evaluation of a tile whose parameters (two planes, halo included) are in
// LDS; also the second half of the fused fit + forward
template <typename T, int MODEL, int TY, int NT = kFwdTX * TY>
__device__ __forceinline__ void tile_fwd_ue_eval(const FieldPtrs<T>& f, int ty0, int tx0, const T* lds, int tid) {
  constexpr int TX = kFwdTX, EX = TX + 2, EY = TY + 2, E = EX * EY;
  static_assert(NT % TX == 0 && TY % (NT / TX) == 0, "rows must split evenly over the threads");
  const int lx = tid % TX, x = tx0 + lx;
  for (int ly = tid / TX; ly < TY; ly += NT / TX) {
    const int y = ty0 + ly;
    if (x < f.W && y < f.H) {
      const int e = (ly + 1) * EX + lx + 1;
      const int en[4] = {e + 1, e - EX, e - 1, e + EX};
      const bool pres[4] = {x + 1 < f.W, y > 0, x > 0, y + 1 < f.H};
      T pmin, pmax;
      vertex_fwd_ue<T, MODEL>(lds, E, e, en, pres, pmin, pmax);
      f.pmin[(int64_t)y * f.rs + x] = pmin;
      f.pmax[(int64_t)y * f.rs + x] = pmax;
    }
  }
}

template <typename T, int MODEL, int TY, int NT = kFwdTX * TY>
__device__ __forceinline__ void tile_fwd_ue(const FieldPtrs<T>& f, int ty0, int tx0, T* lds, int tid) {
  constexpr int EX = kFwdTX + 2, EY = TY + 2;
  stage<T, EY, EX, NT>(lds, f.params, 2, f.ps, f.rs, f.H, f.W, ty0 - 1, tx0 - 1, tid);
  __syncthreads();
  tile_fwd_ue_eval<T, MODEL, TY, NT>(f, ty0, tx0, lds, tid);
  __syncthreads();
}

template <typename T, int TY, int NT = kFwdTX * TY>
__device__ __forceinline__ void tile_fwd_hist(const FieldPtrs<T>& f, int ty0, int tx0, T* lds, int tid) {
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
      const int e = (ly + 1) * EX + lx + 1;
      const int en[4] = {e + 1, e - EX, e - 1, e + EX};
      const bool pres[4] = {x + 1 < f.W, y > 0, x > 0, y + 1 < f.H};
      bool ok = L.valid(e);
#pragma unroll
      for (int i = 0; i < 4; ++i) ok = ok && (!pres[i] || L.valid(en[i]));
      T pmin = qnan<T>(), pmax = qnan<T>();
      if (ok) {
        const T lov = lds[e], hiv = lds[E + e];
        T lo[4], hi[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          lo[i] = lds[en[i]] - lov;
          hi[i] = lds[E + en[i]] - lov;
        }
        hist_vertex_minmax(U, e, en, pres, hiv - lov, lo, hi, pmin, pmax);
      }
      f.pmin[(int64_t)y * f.rs + x] = pmin;
      f.pmax[(int64_t)y * f.rs + x] = pmax;
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// adjoint tiles (uniform / Epanechnikov): OX x OY outputs.  Phase 1 computes
// the weighted Jacobian of every stencil centred in the tile plus a one-vertex
// ring into LDS (parameters staged with a two-vertex halo); phase 2 gathers,
// for each output vertex, the five entries that refer to it.  No atomics.
// If f.pmin is non-null the probabilities are written as well (fused
// forward + adjoint).
// ---------------------------------------------------------------------------
template <int OX, int OY>
struct BwdGeom {
  static constexpr int EX = OX + 2, EY = OY + 2, EJ = EX * EY;  // stencils
  static constexpr int PX = OX + 4, PY = OY + 4, EP = PX * PY;  // parameters
};

// Stencils are dealt to threads as i = tid + k NT (k < KS).  Parameters are
// read from global memory (L1 / L2 hits: the tile and its two-vertex halo);
// the neighbour slots of each Jacobian (e, n, w, s: 8 planes) go to LDS, the
// vertex's own slot stays in registers, because the thread that evaluated a
// stencil also gathers the output at its centre.  Keeping LDS to 8 planes of
// the stencil grid fits five workgroups per CU.
template <typename T, int MODEL, int OX, int OY, int NT, bool WF>
__device__ __forceinline__ void tile_bwd_ue_impl(const FieldPtrs<T>& f, int ty0, int tx0, T* lds, int tid) {
  using G = BwdGeom<OX, OY>;
  constexpr int KS = (G::EJ + NT - 1) / NT;
  T* J = lds;  // [8][EJ]: (slot e, n, w, s) x (parameter 0, 1)
  T own[KS][2];
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    const int i = tid + k * NT;
    T jac[10];
#pragma unroll
    for (int q = 0; q < 10; ++q) jac[q] = T(0);
    if (i < G::EJ) {
      const int ey = i / G::EX, ex = i - ey * G::EX;
      const int gy = ty0 - 1 + ey, gx = tx0 - 1 + ex;
      if (gy >= 0 && gy < f.H && gx >= 0 && gx < f.W) {
        const bool pres[4] = {gx + 1 < f.W, gy > 0, gx > 0, gy + 1 < f.H};
        const int64_t at = (int64_t)gy * f.rs + gx;
        const int64_t an[4] = {at + 1, at - f.rs, at - 1, at + f.rs};
        const T p0 = f.params[at], p1 = f.params[f.ps + at];
        T q0[4], q1[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) {
          q0[n] = pres[n] ? f.params[an[n]] : T(0);
          q1[n] = pres[n] ? f.params[f.ps + an[n]] : T(1);
        }
        T pmin, pmax;
        vertex_jac_vals<T, MODEL, WF>(p0, p1, q0, q1, pres, f.gmin[at], f.gmax[at], jac, pmin, pmax);
        // fused forward: the adjoint evaluates the probabilities as well
        if (WF && ey >= 1 && ey <= OY && ex >= 1 && ex <= OX) {
          f.pmin[at] = pmin;
          f.pmax[at] = pmax;
        }
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) J[q * G::EJ + i] = jac[2 + q];
    }
    own[k][0] = jac[0];
    own[k][1] = jac[1];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    const int i = tid + k * NT;
    if (i >= G::EJ) continue;
    const int ey = i / G::EX, ex = i - ey * G::EX;
    if (ey < 1 || ey > OY || ex < 1 || ex > OX) continue;
    const int gy = ty0 - 1 + ey, gx = tx0 - 1 + ex;
    if (gy >= f.H || gx >= f.W) continue;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      // u is: slot v of its own stencil, w of its east neighbour's, e of
      // its west neighbour's, s of its north neighbour's, n of its south's
      const T g = own[k][q] + J[(4 + q) * G::EJ + i + 1] + J[(0 + q) * G::EJ + i - 1] +
                  J[(6 + q) * G::EJ + i - G::EX] + J[(2 + q) * G::EJ + i + G::EX];
      f.grad[(int64_t)q * f.ps + (int64_t)gy * f.rs + gx] = g;
    }
  }
  __syncthreads();
}

template <typename T, int MODEL, int OX, int OY, int NT>
__device__ __forceinline__ void tile_bwd_ue(const FieldPtrs<T>& f, int ty0, int tx0, T* lds, int tid) {
  if (f.pmin)
    tile_bwd_ue_impl<T, MODEL, OX, OY, NT, true>(f, ty0, tx0, lds, tid);
  else
    tile_bwd_ue_impl<T, MODEL, OX, OY, NT, false>(f, ty0, tx0, lds, tid);
}

template <int OX, int OY>
constexpr int bwd_ue_lds_elems() {
  return 8 * BwdGeom<OX, OY>::EJ;
}

// XCD-aware tile order: blocks are dealt to the 8 XCDs round-robin, so give
// each XCD a contiguous run of tiles (neighbouring tiles share halo lines in
// that XCD's L2).  A bijection on [0, n).
__device__ __forceinline__ int xcd_tile(int b, int n) {
  constexpr int X = 8;
  const int q = n / X, r = n - q * X, k = b % X, i = b / X;
  return k * q + (k < r ? k : r) + i;
}

}  // namespace cp
