// cp_fit_forward.hip -- the fit and the forward of a uniform or Epanechnikov
// field in one launch.
//
// The fit (Sec. 5.1 and 5.2: uniform range = member min / max, Epanechnikov
// centre and half-width from the member mean and standard deviation) is
// HBM-bound and the forward (Eq. 3 and its negation, integrated exactly
// piece by piece) is VALU-bound.  Here a tile of 64 x TY output vertices fits
// its own vertices and the one-vertex halo around them straight from the
// members into LDS, writes the parameters of its own vertices, and evaluates
// P_min / P_max from LDS.  The parameters make no round trip through HBM
// before the forward, and the workgroups resident on a CU overlap: while some
// stream members, others integrate.
//
// Both halves are the routines of the separate calls (FitAcc fed the members
// in order 0..M-1, then tile_fwd_ue_eval), so parameters and probabilities
// equal those of the fit followed by the forward bit for bit.  Members are
// read in 16-byte groups of V = 16 / sizeof(T) vertices: a staged row of
// 64 + 2 vertices is 64 / V groups plus one on each side, of which only the
// vertex next to the tile is kept (its neighbours are fitted and dropped).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "cp_fit.hpp"
#include "cp_internal.hpp"
#include "cp_tiles.hpp"

namespace cp {

namespace {

template <typename T>
struct FitFwdArgs {
  const T* members;  // [M][H][rs], member plane stride f.ps
  int M;
  double wscale, eps;
  FieldPtrs<T> f;  // params written (interior vertices), pmin / pmax
};

// Fit the staged vertices of the tile at (ty0, tx0) into lds (two planes,
// (64 + 2) x (TY + 2) each) with NT threads; the parameters of the tile's own
// vertices also go to global memory.
template <typename T, int MODEL, int TY, int NT>
__device__ __forceinline__ void fit_tile(const FitFwdArgs<T>& a, int ty0, int tx0, T* lds, int tid) {
  constexpr int TX = kFwdTX, EX = TX + 2, EY = TY + 2, E = EX * EY;
  constexpr int V = 16 / sizeof(T);  // vertices per 16-byte group
  constexpr int GX = TX / V + 2;     // groups per staged row
  constexpr int NG = GX * EY;
  typedef T Vec __attribute__((ext_vector_type(V)));
  const FieldPtrs<T>& f = a.f;
  T* par = const_cast<T*>(f.params);
  for (int g = tid; g < NG; g += NT) {
    const int ey = g / GX, gi = g - ey * GX;
    const int gy = ty0 - 1 + ey, gx = tx0 + (gi - 1) * V;  // first column of the group
    T p0[V], p1[V];
    // W is a multiple of V, so a group lies wholly inside or outside the grid
    if (gy >= 0 && gy < f.H && gx >= 0 && gx < f.W) {
      const int64_t at = (int64_t)gy * f.rs + gx;
      FitAcc<T, MODEL> acc[V];
      {
        const Vec v = *reinterpret_cast<const Vec*>(a.members + at);
#pragma unroll
        for (int j = 0; j < V; ++j) acc[j].first(v[j]);
      }
#pragma unroll 4
      for (int k = 1; k < a.M; ++k) {
        const Vec v = *reinterpret_cast<const Vec*>(a.members + (int64_t)k * f.ps + at);
#pragma unroll
        for (int j = 0; j < V; ++j) acc[j].add(v[j]);
      }
#pragma unroll
      for (int j = 0; j < V; ++j) acc[j].finish(a.M, a.wscale, a.eps, p0[j], p1[j]);
      if (gi >= 1 && gi <= TX / V && ey >= 1 && ey <= TY) {  // the tile's own vertices
        Vec o0, o1;
#pragma unroll
        for (int j = 0; j < V; ++j) {
          o0[j] = p0[j];
          o1[j] = p1[j];
        }
        *reinterpret_cast<Vec*>(par + at) = o0;
        *reinterpret_cast<Vec*>(par + f.ps + at) = o1;
      }
    } else {
#pragma unroll
      for (int j = 0; j < V; ++j) p0[j] = p1[j] = T(0);  // outside the grid, as stage()
    }
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const int ex = (gi - 1) * V + j + 1;  // staged column of vertex gx + j
      if (ex >= 0 && ex < EX) {
        lds[ey * EX + ex] = p0[j];
        lds[E + ey * EX + ex] = p1[j];
      }
    }
  }
}

template <typename T, int MODEL, int TY>
__global__ __launch_bounds__(256) void k_fit_fwd_ue(FitFwdArgs<T> a, int tiles_x, int ntiles) {
  __shared__ T lds[2 * (kFwdTX + 2) * (TY + 2)];
  const int t = xcd_tile(blockIdx.x, ntiles);
  const int ty0 = (t / tiles_x) * TY, tx0 = (t % tiles_x) * kFwdTX;
  fit_tile<T, MODEL, TY, 256>(a, ty0, tx0, lds, threadIdx.x);
  __syncthreads();
  tile_fwd_ue_eval<T, MODEL, TY, 256>(a.f, ty0, tx0, lds, threadIdx.x);
}

template <typename T, int MODEL>
hipError_t launch(const FitFwdArgs<T>& a, hipStream_t st) {
  // 64 x 12 tiles: the 14 staged rows of 16-byte groups (252 in FP32) take
  // the 256 threads once (FP64's 476 twice); grids with fewer than eight
  // such tiles per CU use 64 x 4.  Measured at 2048^2 (Epanechnikov, 20 members): 64 x 12 128 us,
  // 64 x 16 (two passes of groups) 135 us, fit then forward 162 us.
  const int tx = (a.f.W + kFwdTX - 1) / kFwdTX;
  const bool tall = (int64_t)tx * ((a.f.H + 11) / 12) >= kTallTileBlocks;
  const int TYr = tall ? 12 : 4, n = tx * ((a.f.H + TYr - 1) / TYr);
  if (tall)
    hipLaunchKernelGGL((k_fit_fwd_ue<T, MODEL, 12>), dim3(n), dim3(256), 0, st, a, tx, n);
  else
    hipLaunchKernelGGL((k_fit_fwd_ue<T, MODEL, 4>), dim3(n), dim3(256), 0, st, a, tx, n);
  return hipGetLastError();
}

template <typename T>
hipError_t typed(const Field& f, const void* members, int M, double wscale, double eps, void* params, void* pmin,
                 void* pmax, hipStream_t st) {
  FitFwdArgs<T> a;
  a.members = static_cast<const T*>(members);
  a.M = M;
  a.wscale = wscale;
  a.eps = eps;
  a.f.params = static_cast<const T*>(params);
  a.f.pmin = static_cast<T*>(pmin);
  a.f.pmax = static_cast<T*>(pmax);
  a.f.gmin = a.f.gmax = nullptr;
  a.f.grad = nullptr;
  a.f.H = f.H;
  a.f.W = f.W;
  a.f.nb = f.nb;
  a.f.rs = f.rs;
  a.f.ps = f.plane();
  return f.model == CP_UNIFORM ? launch<T, CP_UNIFORM>(a, st) : launch<T, CP_EPANECHNIKOV>(a, st);
}

}  // namespace

bool fit_forward_fusable(const Field& f, const void* members, const void* params) {
  const int V = f.dtype == CP_F64 ? 2 : 4;
  return (f.model == CP_UNIFORM || f.model == CP_EPANECHNIKOV) && f.W % V == 0 && f.rs % V == 0 &&
         reinterpret_cast<uintptr_t>(members) % 16 == 0 && reinterpret_cast<uintptr_t>(params) % 16 == 0;
}

hipError_t fit_forward_ue(const Field& f, const void* members, int M, double wscale, double eps, void* params,
                          void* pmin, void* pmax, hipStream_t st) {
  if (f.dtype == CP_F64) return typed<double>(f, members, M, wscale, eps, params, pmin, pmax, st);
  return typed<float>(f, members, M, wscale, eps, params, pmin, pmax, st);
}

}  // namespace cp
