// cp_closed_form.hip -- per-field forward and adjoint kernels for the
// uniform, Epanechnikov and histogram models, and their launchers.
#include <hip/hip_runtime.h>

#include "cp_hist_bwd.hpp"
#include "cp_internal.hpp"
#include "cp_tiles.hpp"

namespace cp {

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
// 64 x TY outputs per block of NT threads (TY / (NT / 64) rows per thread)
template <typename T, int MODEL, int TY, int NT>
__global__ __launch_bounds__(NT) void k_fwd_ue(FieldPtrs<T> f, int tiles_x, int ntiles) {
  __shared__ T lds[2 * (kFwdTX + 2) * (TY + 2)];
  const int t = xcd_tile(blockIdx.x, ntiles);
  tile_fwd_ue<T, MODEL, TY, NT>(f, (t / tiles_x) * TY, (t % tiles_x) * kFwdTX, lds, threadIdx.x);
}

template <typename T, int TY>
__global__ __launch_bounds__(kFwdTX* TY) void k_fwd_hist(FieldPtrs<T> f, int tiles_x, int ntiles) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* lds = reinterpret_cast<T*>(smem);
  const int t = xcd_tile(blockIdx.x, ntiles);
  tile_fwd_hist<T, TY>(f, (t / tiles_x) * TY, (t % tiles_x) * kFwdTX, lds, threadIdx.x);
}

// ---------------------------------------------------------------------------
// adjoint
// ---------------------------------------------------------------------------
template <typename T, int MODEL, int OX, int OY>
__global__ __launch_bounds__(256) void k_bwd_ue(FieldPtrs<T> f, int tiles_x, int ntiles) {
  __shared__ T lds[bwd_ue_lds_elems<OX, OY>()];
  const int t = xcd_tile(blockIdx.x, ntiles);
  tile_bwd_ue<T, MODEL, OX, OY, 256>(f, (t / tiles_x) * OY, (t % tiles_x) * OX, lds, threadIdx.x);
}

// histogram adjoint, pass 1: per-stencil entries into the workspace
template <typename T, int TY>
__global__ __launch_bounds__(kFwdTX* TY) void k_hist_sweep(FieldPtrs<T> f, int tiles_x, int ntiles, T* J) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* lds = reinterpret_cast<T*>(smem);
  const int t = xcd_tile(blockIdx.x, ntiles);
  tile_hist_sweep<T, TY>(f, (t / tiles_x) * TY, (t % tiles_x) * kFwdTX, lds, threadIdx.x, J);
}

// histogram adjoint, pass 2: every mass of u gathers its own stencil's entry
// and the entries of its four neighbours' stencils that refer to u
template <typename T>
__global__ __launch_bounds__(256) void k_hist_gather(FieldPtrs<T> f, const T* __restrict__ J) {
  hist_gather_vertex<T>(f, J, (int64_t)blockIdx.x * 256 + threadIdx.x);
}

// the same, 16 bytes of vertices per thread (rows and planes in 16-byte units)
template <typename T>
__global__ __launch_bounds__(256) void k_hist_gather_vec(FieldPtrs<T> f, const T* __restrict__ J) {
  hist_gather_vec<T>(f, J, (int64_t)blockIdx.x * 256 + threadIdx.x);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static int cdiv(int a, int b) { return (a + b - 1) / b; }

constexpr size_t kMaxLds = 160 * 1024;  // LDS per workgroup on gfx950

template <typename T>
static FieldPtrs<T> make_ptrs(const Field& f, const void* params, void* pmin, void* pmax, const void* gmin,
                              const void* gmax, void* grad) {
  FieldPtrs<T> p;
  p.params = static_cast<const T*>(params);
  p.pmin = static_cast<T*>(pmin);
  p.pmax = static_cast<T*>(pmax);
  p.gmin = static_cast<const T*>(gmin);
  p.gmax = static_cast<const T*>(gmax);
  p.grad = static_cast<T*>(grad);
  p.H = f.H;
  p.W = f.W;
  p.nb = f.nb;
  p.rs = f.rs;
  p.ps = f.plane();
  return p;
}

// dynamic LDS above 64 KiB needs the per-kernel attribute
template <typename K>
static hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

template <typename T, int TY>
static hipError_t launch_fwd_hist(const FieldPtrs<T>& p, hipStream_t st) {
  const int tx = cdiv(p.W, kFwdTX), ty = cdiv(p.H, TY), n = tx * ty;
  const size_t lds = sizeof(T) * (size_t)hist_planes(p.nb) * (kFwdTX + 2) * (TY + 2);
  hipError_t e = allow_lds(k_fwd_hist<T, TY>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_fwd_hist<T, TY>), dim3(n), dim3(kFwdTX * TY), lds, st, p, tx, n);
  return hipGetLastError();
}

template <typename T>
static hipError_t fwd_typed(const Field& f, const void* params, void* pmin, void* pmax, hipStream_t st) {
  FieldPtrs<T> p = make_ptrs<T>(f, params, pmin, pmax, nullptr, nullptr, nullptr);
  if (f.model == CP_UNIFORM || f.model == CP_EPANECHNIKOV) {
    // 64 x 16 outputs per 256-thread block, four rows per thread: 79 us
    // against 87 us for 64 x 4 with one row per thread (Epanechnikov,
    // 2048^2); grids too small for eight such blocks per CU keep 64 x 4
    const int tx = cdiv(f.W, kFwdTX);
    const bool tall = (int64_t)tx * cdiv(f.H, 16) >= kTallTileBlocks;
    const int TYr = tall ? 16 : 4, n = tx * cdiv(f.H, TYr);
    if (f.model == CP_UNIFORM) {
      if (tall)
        hipLaunchKernelGGL((k_fwd_ue<T, CP_UNIFORM, 16, 256>), dim3(n), dim3(256), 0, st, p, tx, n);
      else
        hipLaunchKernelGGL((k_fwd_ue<T, CP_UNIFORM, 4, 256>), dim3(n), dim3(256), 0, st, p, tx, n);
    } else {
      if (tall)
        hipLaunchKernelGGL((k_fwd_ue<T, CP_EPANECHNIKOV, 16, 256>), dim3(n), dim3(256), 0, st, p, tx, n);
      else
        hipLaunchKernelGGL((k_fwd_ue<T, CP_EPANECHNIKOV, 4, 256>), dim3(n), dim3(256), 0, st, p, tx, n);
    }
    return hipGetLastError();
  }
  // histogram: pick the tile height that keeps the staged planes within LDS
  const size_t per_row = sizeof(T) * (size_t)hist_planes(f.nb) * (kFwdTX + 2);
  if (per_row * 6 <= 64 * 1024) return launch_fwd_hist<T, 4>(p, st);
  if (per_row * 4 <= kMaxLds) return launch_fwd_hist<T, 2>(p, st);
  return launch_fwd_hist<T, 1>(p, st);
}

hipError_t cf_forward(const Field& f, const void* params, void* pmin, void* pmax, hipStream_t st) {
  // the Gaussian sweep yields all four classification integrals at once
  if (f.model == CP_GAUSSIAN) return cf_classify(f, params, pmin, pmax, nullptr, nullptr, nullptr, st);
  if (f.dtype == CP_F64) return fwd_typed<double>(f, params, pmin, pmax, st);
  return fwd_typed<float>(f, params, pmin, pmax, st);
}

template <typename T, int OX, int OY>
static hipError_t launch_bwd_ue(const FieldPtrs<T>& p, int model, hipStream_t st) {
  const int tx = cdiv(p.W, OX), ty = cdiv(p.H, OY), n = tx * ty;
  if (model == CP_UNIFORM)
    hipLaunchKernelGGL((k_bwd_ue<T, CP_UNIFORM, OX, OY>), dim3(n), dim3(256), 0, st, p, tx, n);
  else
    hipLaunchKernelGGL((k_bwd_ue<T, CP_EPANECHNIKOV, OX, OY>), dim3(n), dim3(256), 0, st, p, tx, n);
  return hipGetLastError();
}

// independent Gaussian: FP32 30x30 outputs (32x32 stencils, four per
// thread), so the ring of halo stencils is 12% of the work against 24% for
// 14x14; FP64 keeps 14x14 (one stencil per thread: its 250 registers leave
// no room for a second)
template <typename T>
static hipError_t launch_bwd_gauss(const FieldPtrs<T>& p, hipStream_t st) {
  constexpr int O = sizeof(T) == 4 ? 30 : 14;
  const int tx = cdiv(p.W, O), ty = cdiv(p.H, O), n = tx * ty;
  hipLaunchKernelGGL((k_bwd_ue<T, CP_GAUSSIAN, O, O>), dim3(n), dim3(256), 0, st, p, tx, n);
  return hipGetLastError();
}

template <typename T, int TY>
static hipError_t launch_bwd_hist(const FieldPtrs<T>& p, hipStream_t st, const Scratch& scr) {
  const int tx = cdiv(p.W, kFwdTX), ty = cdiv(p.H, TY), n = tx * ty;
  const int64_t plane = (int64_t)p.H * p.W;
  void* ws = nullptr;
  hipError_t e = adjoint_scratch(sizeof(T) * (size_t)hist_ws_planes(p.nb) * plane, st, scr, &ws);
  if (e != hipSuccess) return e;
  T* J = static_cast<T*>(ws);
  const size_t lds = sizeof(T) * (size_t)hist_planes(p.nb) * (kFwdTX + 2) * (TY + 2);
  e = allow_lds(k_hist_sweep<T, TY>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_hist_sweep<T, TY>), dim3(n), dim3(kFwdTX * TY), lds, st, p, tx, n, J);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  constexpr int V = 16 / sizeof(T);
  if (p.W % V == 0 && p.rs % V == 0 && p.ps % V == 0 && reinterpret_cast<uintptr_t>(p.grad) % 16 == 0) {
    const int64_t groups = plane / V;
    hipLaunchKernelGGL(k_hist_gather_vec<T>, dim3((unsigned)((groups + 255) / 256)), dim3(256), 0, st, p,
                       static_cast<const T*>(J));
  } else {
    hipLaunchKernelGGL(k_hist_gather<T>, dim3((unsigned)((plane + 255) / 256)), dim3(256), 0, st, p,
                       static_cast<const T*>(J));
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t bwd_typed(const Field& f, const void* params, const void* gmin, const void* gmax, void* grad,
                            hipStream_t st, const Scratch& scr) {
  FieldPtrs<T> p = make_ptrs<T>(f, params, nullptr, nullptr, gmin, gmax, grad);
  if (f.model == CP_GAUSSIAN) return launch_bwd_gauss<T>(p, st);
  if (f.model != CP_HISTOGRAM) {
    // 30x30 outputs (32x32 stencils, 4 per thread) keep the FP32 tile under
    // 64 KiB of static LDS; FP64 uses 14x14 (16x16 stencils)
    if constexpr (sizeof(T) == 4)
      return launch_bwd_ue<T, 30, 30>(p, f.model, st);
    else
      return launch_bwd_ue<T, 14, 14>(p, f.model, st);
  }
  // sweep tiles as in the forward; the entries go through the workspace
  const size_t per_row = sizeof(T) * (size_t)hist_planes(f.nb) * (kFwdTX + 2);
  if (per_row * 6 <= 64 * 1024) return launch_bwd_hist<T, 4>(p, st, scr);
  if (per_row * 4 <= kMaxLds) return launch_bwd_hist<T, 2>(p, st, scr);
  return launch_bwd_hist<T, 1>(p, st, scr);
}

hipError_t cf_backward(const Field& f, const void* params, const void* gmin, const void* gmax, void* grad,
                       hipStream_t st, const Scratch& scr) {
  if (f.dtype == CP_F64) return bwd_typed<double>(f, params, gmin, gmax, grad, st, scr);
  return bwd_typed<float>(f, params, gmin, gmax, grad, st, scr);
}

bool gl_table(int n, double* x, double* w) {
  switch (n) {
#define CP_GL_CASE(N)                 \
  case N:                             \
    for (int i = 0; i < N; ++i) {     \
      x[i] = GL<N>::x[i];             \
      w[i] = GL<N>::w[i];             \
    }                                 \
    return true;
    CP_GL_CASE(1)
    CP_GL_CASE(2)
    CP_GL_CASE(3)
    CP_GL_CASE(4)
    CP_GL_CASE(5)
    CP_GL_CASE(6)
    CP_GL_CASE(7)
    CP_GL_CASE(8)
    CP_GL_CASE(10)
#undef CP_GL_CASE
    default:
      return false;
  }
}

}  // namespace cp
