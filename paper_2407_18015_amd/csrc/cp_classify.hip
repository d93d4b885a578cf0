// cp_classify.hip -- classification probabilities of every vertex: P_min,
// P_max (Eq. 3 and its negation), P_saddle = t1 + t2 (Eq. 4) and
// P_regular = 1 - P_min - P_max - P_saddle, in one pass over the parameters.
// Tiles of 64 x TY vertices stage their parameters plus a one-vertex halo in
// LDS, as the forward kernels do; every requested output is written from the
// same staged stencil.
#include <hip/hip_runtime.h>

#include "cp_gauss.hpp"
#include "cp_internal.hpp"
#include "cp_saddle.hpp"
#include "cp_tiles.hpp"

namespace cp {

template <typename T>
struct ClassPtrs {
  const T* params;
  T* pmin;
  T* pmax;
  T* psad;
  T* preg;
  T* terms;  // [2][H][rs]: t1, t2
  int H, W, nb;
  int64_t rs, ps;
};

template <typename T>
__device__ __forceinline__ void class_store(const ClassPtrs<T>& f, int y, int x, T pmin, T pmax, T t1, T t2) {
  const int64_t at = (int64_t)y * f.rs + x;
  const T ps = t1 + t2;
  if (f.pmin) f.pmin[at] = pmin;
  if (f.pmax) f.pmax[at] = pmax;
  if (f.psad) f.psad[at] = ps;
  if (f.terms) {
    f.terms[at] = t1;
    f.terms[f.ps + at] = t2;
  }
  if (f.preg) f.preg[at] = T(1) - pmin - pmax - ps;
}

// 64 x TY vertices per block of NT threads (TY / (NT / 64) rows per thread)
template <typename T, int MODEL, int TY, int NT>
__global__ __launch_bounds__(NT) void k_classify_ue(ClassPtrs<T> f, int tiles_x, int ntiles) {
  constexpr int TX = kFwdTX, EX = TX + 2, EY = TY + 2, E = EX * EY;
  static_assert(NT % TX == 0 && TY % (NT / TX) == 0, "rows must split evenly over the threads");
  __shared__ T lds[2 * E];
  const int t = xcd_tile(blockIdx.x, ntiles);
  const int ty0 = (t / tiles_x) * TY, tx0 = (t % tiles_x) * TX, tid = threadIdx.x;
  stage<T, EY, EX, NT>(lds, f.params, 2, f.ps, f.rs, f.H, f.W, ty0 - 1, tx0 - 1, tid);
  __syncthreads();
  const int lx = tid % TX, x = tx0 + lx;
  const bool mm = f.pmin || f.pmax || f.preg;
  const bool sad = f.psad || f.terms || f.preg;
  for (int ly = tid / TX; ly < TY; ly += NT / TX) {
    const int y = ty0 + ly;
    if (x >= f.W || y >= f.H) continue;
    const int e = (ly + 1) * EX + lx + 1;
    const int en[4] = {e + 1, e - EX, e - 1, e + EX};
    const bool pres[4] = {x + 1 < f.W, y > 0, x > 0, y + 1 < f.H};
    T pmin = T(0), pmax = T(0), t1 = T(0), t2 = T(0);
    if (!stencil_valid_ue<T, MODEL>(lds, E, e, en, pres)) {
      pmin = pmax = t1 = t2 = qnan<T>();
    } else if constexpr (MODEL == CP_GAUSSIAN) {
      T mn[4], sn[4], o[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        mn[i] = pres[i] ? lds[en[i]] : T(0);
        sn[i] = pres[i] ? lds[E + en[i]] : T(1);
      }
      gauss_vertex<T>(lds[e], lds[E + e], mn, sn, pres, o);
      pmin = o[0];
      pmax = o[1];
      t1 = o[2];
      t2 = o[3];
    } else {
      if (mm) vertex_fwd_ue<T, MODEL>(lds, E, e, en, pres, pmin, pmax);
      // the alternating pattern needs all four neighbours: 0 on the boundary
      if (sad && pres[0] && pres[1] && pres[2] && pres[3]) vertex_saddle_ue<T, MODEL>(lds, E, e, en, t1, t2);
    }
    class_store(f, y, x, pmin, pmax, t1, t2);
  }
}

template <typename T, int TY>
__global__ __launch_bounds__(kFwdTX* TY) void k_classify_hist(ClassPtrs<T> f, int tiles_x, int ntiles) {
  constexpr int TX = kFwdTX, EX = TX + 2, EY = TY + 2, E = EX * EY, NT = TX * TY;
  extern __shared__ __align__(16) unsigned char smem[];
  T* lds = reinterpret_cast<T*>(smem);
  const int t = xcd_tile(blockIdx.x, ntiles);
  const int ty0 = (t / tiles_x) * TY, tx0 = (t % tiles_x) * TX, tid = threadIdx.x;
  const int h = f.nb;
  stage<T, EY, EX, NT>(lds, f.params, 2 + h, f.ps, f.rs, f.H, f.W, ty0 - 1, tx0 - 1, tid);
  __syncthreads();
  hist_stage_validity<T, NT>(lds, E, h, tid);
  hist_stage_suffix<T, NT>(lds, E, h, tid);
  __syncthreads();
  const int lx = tid % TX, ly = tid / TX;
  const int x = tx0 + lx, y = ty0 + ly;
  if (x >= f.W || y >= f.H) return;
  const HistLds<T> L{lds, E, h, T(1) / T(h)};
  const HistSuf<T> U{lds, E, h};
  const int e = (ly + 1) * EX + lx + 1;
  const int en[4] = {e + 1, e - EX, e - 1, e + EX};
  const bool pres[4] = {x + 1 < f.W, y > 0, x > 0, y + 1 < f.H};
  bool ok = L.valid(e);
#pragma unroll
  for (int i = 0; i < 4; ++i) ok = ok && (!pres[i] || L.valid(en[i]));
  const bool mm = f.pmin || f.pmax || f.preg;
  const bool sad = f.psad || f.terms || f.preg;
  T pmin = T(0), pmax = T(0), t1 = T(0), t2 = T(0);
  if (!ok) {
    pmin = pmax = t1 = t2 = qnan<T>();
  } else {
    const T lov = lds[e], hiv = lds[E + e];
    T lo[4], hi[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      lo[i] = lds[en[i]] - lov;
      hi[i] = lds[E + en[i]] - lov;
    }
    // the saddle terms ride in the sweep of P_min / P_max (a vertex without
    // all four neighbours has none)
    if (sad) {
      hist_vertex_sweep<T, true>(U, e, en, pres, hiv - lov, lo, hi, pmin, pmax, t1, t2);
      if (!(pres[0] && pres[1] && pres[2] && pres[3])) t1 = t2 = T(0);
    } else if (mm) {
      hist_vertex_minmax(U, e, en, pres, hiv - lov, lo, hi, pmin, pmax);
    }
  }
  class_store(f, y, x, pmin, pmax, t1, t2);
}

// ---------------------------------------------------------------------------
// launcher
// ---------------------------------------------------------------------------
static int cdiv_c(int a, int b) { return (a + b - 1) / b; }

template <typename T, int TY>
static hipError_t launch_classify_hist(const ClassPtrs<T>& p, hipStream_t st) {
  const int tx = cdiv_c(p.W, kFwdTX), ty = cdiv_c(p.H, TY), n = tx * ty;
  const size_t lds = sizeof(T) * (size_t)hist_planes(p.nb) * (kFwdTX + 2) * (TY + 2);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_classify_hist<T, TY>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_classify_hist<T, TY>), dim3(n), dim3(kFwdTX * TY), lds, st, p, tx, n);
  return hipGetLastError();
}

template <typename T>
static hipError_t classify_typed(const Field& f, const void* params, void* pmin, void* pmax, void* psad,
                                 void* preg, void* terms, hipStream_t st) {
  ClassPtrs<T> p;
  p.params = static_cast<const T*>(params);
  p.pmin = static_cast<T*>(pmin);
  p.pmax = static_cast<T*>(pmax);
  p.psad = static_cast<T*>(psad);
  p.preg = static_cast<T*>(preg);
  p.terms = static_cast<T*>(terms);
  p.H = f.H;
  p.W = f.W;
  p.nb = f.nb;
  p.rs = f.rs;
  p.ps = f.plane();
  // uniform / Epanechnikov: 64 x 16 vertices per 256-thread block on grids
  // with at least eight such blocks per CU (as the forward), else 64 x 4;
  // the Gaussian quadrature keeps one row per thread (64 x 4)
  const int tx = cdiv_c(f.W, kFwdTX);
  const bool tall = (int64_t)tx * cdiv_c(f.H, 16) >= kTallTileBlocks;
  const int n4 = tx * cdiv_c(f.H, 4), n16 = tx * cdiv_c(f.H, 16);
  if (f.model == CP_UNIFORM) {
    if (tall)
      hipLaunchKernelGGL((k_classify_ue<T, CP_UNIFORM, 16, 256>), dim3(n16), dim3(256), 0, st, p, tx, n16);
    else
      hipLaunchKernelGGL((k_classify_ue<T, CP_UNIFORM, 4, 256>), dim3(n4), dim3(256), 0, st, p, tx, n4);
    return hipGetLastError();
  }
  if (f.model == CP_EPANECHNIKOV) {
    if (tall)
      hipLaunchKernelGGL((k_classify_ue<T, CP_EPANECHNIKOV, 16, 256>), dim3(n16), dim3(256), 0, st, p, tx, n16);
    else
      hipLaunchKernelGGL((k_classify_ue<T, CP_EPANECHNIKOV, 4, 256>), dim3(n4), dim3(256), 0, st, p, tx, n4);
    return hipGetLastError();
  }
  if (f.model == CP_GAUSSIAN) {
    hipLaunchKernelGGL((k_classify_ue<T, CP_GAUSSIAN, 4, 256>), dim3(n4), dim3(256), 0, st, p, tx, n4);
    return hipGetLastError();
  }
  const size_t per_row = sizeof(T) * (size_t)hist_planes(f.nb) * (kFwdTX + 2);
  if (per_row * 6 <= 64 * 1024) return launch_classify_hist<T, 4>(p, st);
  if (per_row * 4 <= 160 * 1024) return launch_classify_hist<T, 2>(p, st);
  return launch_classify_hist<T, 1>(p, st);
}

hipError_t cf_classify(const Field& f, const void* params, void* pmin, void* pmax, void* psad, void* preg,
                       void* terms, hipStream_t st) {
  if (f.dtype == CP_F64) return classify_typed<double>(f, params, pmin, pmax, psad, preg, terms, st);
  return classify_typed<float>(f, params, pmin, pmax, psad, preg, terms, st);
}

}  // namespace cp
