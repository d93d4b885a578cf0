// cp_fit.hip -- per-vertex model fitting from ensemble members.
//
// Rules (Sec. 5.1 and 5.2 for the parametric ranges, Sec. 4.4 for
// histograms, Sec. 5.2/5.3 for the multivariate Gaussian):
//   uniform       lo = min, hi = max of the members
//   Epanechnikov  m = mean, w = bw * std(ddof) * M^(-1/5)
//   Gaussian      mu = mean, sigma = std(ddof) (independent per vertex)
//   histogram     lo = min, hi = max, nbins equal-width bins, mass = count/M;
//                 bin of x = floor(((x - lo) / (hi - lo)) * nbins), computed in
//                 the field's precision with every operation rounded once,
//                 the maximum in the last bin
//   degenerate    all members equal: lo/hi = x -/+ eps*max(1,|x|), Epanechnikov
//                 w (Gaussian sigma) = eps*max(1,|m|)
//   multivariate  mean plane; covariance of (e, n, w, s, v) over members with
//                 `ddof`, + jitter on the diagonal, FP64 Cholesky; absent
//                 neighbours get identity rows.
// The kernels are HBM-bound: every member value is read once (held in
// registers), statistics are accumulated in FP64.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "cp_fit.hpp"
#include "cp_internal.hpp"

namespace cp {

namespace {

constexpr int kFitTX = 64, kFitTY = 4, kMaxRegMembers = 32;

template <typename T>
__device__ __forceinline__ int bin_of(T x, T lo, T hi, int nb) {
  const T t = rn_div(rn_sub(x, lo), rn_sub(hi, lo));
  int j = (int)rn_mul(t, T(nb));
  return j < 0 ? 0 : (j > nb - 1 ? nb - 1 : j);
}

struct FitArgs {
  const void* members;
  void* params;
  int M, H, W, nb, ddof;
  int64_t rs, ps;
  double wscale;  // bw * M^(-1/5) / sqrt(M - ddof): Epanechnikov w = wscale * sqrt(sum of squares)
  double eps;
};

// Uniform / Epanechnikov / histogram.  MM (histogram): members held in
// registers (M <= MM); MM == 0 streams them twice from memory.
template <typename T, int MODEL, int MM>
__global__ __launch_bounds__(kFitTX* kFitTY) void k_fit(FitArgs a) {
  __shared__ int counts[MODEL == CP_HISTOGRAM ? kMaxBins * kFitTX * kFitTY : 1];
  const int tid = threadIdx.x;
  const int x = blockIdx.x * kFitTX + (tid % kFitTX);
  const int y = blockIdx.y * kFitTY + (tid / kFitTX);
  if (x >= a.W || y >= a.H) return;
  const T* mem = static_cast<const T*>(a.members);
  T* par = static_cast<T*>(a.params);
  const int64_t at = (int64_t)y * a.rs + x;
  const int M = a.M;
  if (MODEL != CP_HISTOGRAM) {
    T p0, p1;
    fit_ue_vertex<T, MODEL>(mem, M, a.ps, at, a.wscale, a.eps, p0, p1);
    par[at] = p0;
    par[a.ps + at] = p1;
    return;
  }
  T v[MM > 0 ? MM : 1];
  T mn, mx;
  if (MM > 0) {
#pragma unroll
    for (int k = 0; k < (MM > 0 ? MM : 1); ++k)
      if (k < M) v[k] = mem[(int64_t)k * a.ps + at];
    mn = mx = v[0];
#pragma unroll
    for (int k = 1; k < (MM > 0 ? MM : 1); ++k)
      if (k < M) {
        mn = v[k] < mn ? v[k] : mn;
        mx = v[k] > mx ? v[k] : mx;
      }
  } else {
    mn = mx = mem[at];
    for (int k = 1; k < M; ++k) {
      const T xk = mem[(int64_t)k * a.ps + at];
      mn = xk < mn ? xk : mn;
      mx = xk > mx ? xk : mx;
    }
  }
  T lo = mn, hi = mx;
  if (!(mn < mx)) {
    const T e = degenerate_half(T(a.eps), mn);
    lo = rn_sub(mn, e);
    hi = rn_add(mn, e);
  }
  // histogram: per-thread counters in LDS (dynamic bin index)
  int* cnt = counts + tid;
  constexpr int NT = kFitTX * kFitTY;
  for (int j = 0; j < a.nb; ++j) cnt[j * NT] = 0;
  if (MM > 0) {
#pragma unroll
    for (int k = 0; k < (MM > 0 ? MM : 1); ++k)
      if (k < M) cnt[bin_of(v[k], lo, hi, a.nb) * NT] += 1;
  } else {
    for (int k = 0; k < M; ++k) cnt[bin_of(mem[(int64_t)k * a.ps + at], lo, hi, a.nb) * NT] += 1;
  }
  par[at] = lo;
  par[a.ps + at] = hi;
  const T fm = T(M);
  for (int j = 0; j < a.nb; ++j) par[(int64_t)(2 + j) * a.ps + at] = rn_div(T(cnt[j * NT]), fm);
}

// Uniform / Epanechnikov with 16-byte loads: a thread fits V = 16 / sizeof(T)
// consecutive vertices of a row, reading each member plane as one vector
// (4 FP32 or 2 FP64 values).  On MI355X a stream of 16-byte loads reads HBM
// at ~6.7 TB/s against ~4 TB/s for 4-byte loads.  Needs W, the row stride and
// both base addresses multiples of V elements (the host checks).  The
// per-vertex operations are FitAcc's, as in k_fit.
// Members are read once and the parameters written once, so both go through
// non-temporal accesses (no cache allocation on the way): 5.7 against
// 5.0 TB/s for this access pattern at 2048^2 x 20.
template <typename T, int MODEL>
__global__ __launch_bounds__(256) void k_fit_vec(FitArgs a, int64_t nvec) {
  constexpr int V = 16 / sizeof(T);
  typedef T Vec __attribute__((ext_vector_type(V)));
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q >= nvec) return;
  const int wv = a.W / V;
  const int y = (int)(q / wv), x = (int)(q - (int64_t)y * wv) * V;
  const int64_t at = (int64_t)y * a.rs + x;
  const T* mem = static_cast<const T*>(a.members);
  T* par = static_cast<T*>(a.params);
  FitAcc<T, MODEL> acc[V];
  {
    const Vec v = __builtin_nontemporal_load(reinterpret_cast<const Vec*>(mem + at));
#pragma unroll
    for (int j = 0; j < V; ++j) acc[j].first(v[j]);
  }
#pragma unroll 4
  for (int k = 1; k < a.M; ++k) {
    const Vec v = __builtin_nontemporal_load(reinterpret_cast<const Vec*>(mem + (int64_t)k * a.ps + at));
#pragma unroll
    for (int j = 0; j < V; ++j) acc[j].add(v[j]);
  }
  T r0[V], r1[V];
#pragma unroll
  for (int j = 0; j < V; ++j) acc[j].finish(a.M, a.wscale, a.eps, r0[j], r1[j]);
  Vec o0, o1;
#pragma unroll
  for (int j = 0; j < V; ++j) {
    o0[j] = r0[j];
    o1[j] = r1[j];
  }
  __builtin_nontemporal_store(o0, reinterpret_cast<Vec*>(par + at));
  __builtin_nontemporal_store(o1, reinterpret_cast<Vec*>(par + a.ps + at));
}

// ---------------------------------------------------------------------------
// multivariate Gaussian: mean plane, then per-vertex covariance + Cholesky
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fit_mean(FitArgs a) {
  const int x = blockIdx.x * kFitTX + (threadIdx.x % kFitTX);
  const int y = blockIdx.y * kFitTY + (threadIdx.x / kFitTX);
  if (x >= a.W || y >= a.H) return;
  const float* mem = static_cast<const float*>(a.members);
  double* par = static_cast<double*>(a.params);
  const int64_t at = (int64_t)y * a.rs + x;
  double s = 0.0;
  for (int k = 0; k < a.M; ++k) s += (double)mem[(int64_t)k * a.ps + at];
  par[at] = s / (double)a.M;
}

__global__ __launch_bounds__(256) void k_fit_mvg(FitArgs a, double jitter) {
  const int x = blockIdx.x * kFitTX + (threadIdx.x % kFitTX);
  const int y = blockIdx.y * kFitTY + (threadIdx.x / kFitTX);
  if (x >= a.W || y >= a.H) return;
  const float* mem = static_cast<const float*>(a.members);
  double* par = static_cast<double*>(a.params);
  const int64_t at = (int64_t)y * a.rs + x;
  // variable order e, n, w, s, v
  const int dy[5] = {0, -1, 0, 1, 0}, dx[5] = {1, 0, -1, 0, 0};
  bool pres[5];
  int64_t off[5];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const int yy = y + dy[i], xx = x + dx[i];
    pres[i] = yy >= 0 && yy < a.H && xx >= 0 && xx < a.W;
    off[i] = pres[i] ? (int64_t)yy * a.rs + xx : at;
  }
  double k0[5], s1[5], s2[15];
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    k0[i] = (double)mem[off[i]];
    s1[i] = 0.0;
  }
#pragma unroll
  for (int i = 0; i < 15; ++i) s2[i] = 0.0;
  for (int k = 0; k < a.M; ++k) {
    double d[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      d[i] = (double)mem[(int64_t)k * a.ps + off[i]] - k0[i];
      s1[i] += d[i];
    }
    int t = 0;
#pragma unroll
    for (int r = 0; r < 5; ++r)
#pragma unroll
      for (int c = 0; c <= r; ++c, ++t) s2[t] = fma(d[r], d[c], s2[t]);
  }
  const double M = (double)a.M, den = (double)(a.M - a.ddof);
  double C[5][5];
  {
    int t = 0;
#pragma unroll
    for (int r = 0; r < 5; ++r)
#pragma unroll
      for (int c = 0; c <= r; ++c, ++t) {
        double v;
        if (pres[r] && pres[c])
          v = (s2[t] - s1[r] * s1[c] / M) / den + (r == c ? jitter : 0.0);
        else
          v = r == c ? 1.0 : 0.0;
        C[r][c] = v;
      }
  }
  double L[5][5];
  bool ok = true;
#pragma unroll
  for (int r = 0; r < 5; ++r)
#pragma unroll
    for (int c = 0; c <= r; ++c) {
      double s = C[r][c];
#pragma unroll
      for (int k = 0; k < c; ++k) s -= L[r][k] * L[c][k];
      if (r == c) {
        ok = ok && s > 0.0;
        L[r][c] = sqrt(s > 0.0 ? s : 1.0);
      } else {
        L[r][c] = s / L[c][c];
      }
    }
  int t = 0;
#pragma unroll
  for (int r = 0; r < 5; ++r)
#pragma unroll
    for (int c = 0; c <= r; ++c, ++t) par[(int64_t)(1 + t) * a.ps + at] = ok ? L[r][c] : __builtin_nan("");
}

template <typename T, int MODEL>
hipError_t launch_fit(const FitArgs& a, hipStream_t st) {
  constexpr int V = 16 / sizeof(T);
  if constexpr (MODEL != CP_HISTOGRAM) {
    if (a.W % V == 0 && a.rs % V == 0 && reinterpret_cast<uintptr_t>(a.members) % 16 == 0 &&
        reinterpret_cast<uintptr_t>(a.params) % 16 == 0) {
      const int64_t nvec = (int64_t)a.H * (a.W / V);
      hipLaunchKernelGGL((k_fit_vec<T, MODEL>), dim3((unsigned)((nvec + 255) / 256)), dim3(256), 0, st, a, nvec);
      return hipGetLastError();
    }
  }
  dim3 grid((a.W + kFitTX - 1) / kFitTX, (a.H + kFitTY - 1) / kFitTY);
  if (MODEL != CP_HISTOGRAM)
    hipLaunchKernelGGL((k_fit<T, MODEL, 0>), grid, dim3(kFitTX * kFitTY), 0, st, a);
  else if (a.M <= 8)
    hipLaunchKernelGGL((k_fit<T, MODEL, 8>), grid, dim3(kFitTX * kFitTY), 0, st, a);
  else if (a.M <= kMaxRegMembers)
    hipLaunchKernelGGL((k_fit<T, MODEL, kMaxRegMembers>), grid, dim3(kFitTX * kFitTY), 0, st, a);
  else
    hipLaunchKernelGGL((k_fit<T, MODEL, 0>), grid, dim3(kFitTX * kFitTY), 0, st, a);
  return hipGetLastError();
}

template <typename T>
hipError_t fit_typed(const FitArgs& a, int model, hipStream_t st) {
  if (model == CP_UNIFORM) return launch_fit<T, CP_UNIFORM>(a, st);
  if (model == CP_EPANECHNIKOV || model == CP_GAUSSIAN) return launch_fit<T, CP_EPANECHNIKOV>(a, st);
  return launch_fit<T, CP_HISTOGRAM>(a, st);
}

}  // namespace

// ---------------------------------------------------------------------------
// uniform model of an error-bounded reconstruction (Sec. 5.3, climate data):
// [d' - eb/2, d' + eb/2], each end rounded once in the field's precision
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_fit_error_bound(const T* __restrict__ d, T half, T* __restrict__ params,
                                                         int H, int W, int64_t rs, int64_t ps) {
  const int64_t n = (int64_t)H * W;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int y = (int)(i / W), x = (int)(i - (int64_t)y * W);
    const int64_t at = (int64_t)y * rs + x;
    const T v = d[at];
    params[at] = v - half;
    params[ps + at] = v + half;
  }
}

hipError_t fit_error_bound(const Field& f, const void* decompressed, double eb, void* params, hipStream_t st) {
  const int64_t n = (int64_t)f.H * f.W;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 256 * 16);
  if (f.dtype == CP_F64)
    hipLaunchKernelGGL(k_fit_error_bound<double>, dim3(blocks), dim3(256), 0, st,
                       static_cast<const double*>(decompressed), eb * 0.5, static_cast<double*>(params), f.H, f.W,
                       f.rs, f.plane());
  else
    hipLaunchKernelGGL(k_fit_error_bound<float>, dim3(blocks), dim3(256), 0, st,
                       static_cast<const float*>(decompressed), (float)(eb * 0.5), static_cast<float*>(params),
                       f.H, f.W, f.rs, f.plane());
  return hipGetLastError();
}

hipError_t fit_params(const Field& f, const void* members, int M, int ddof, double bw, double jitter, double eps,
                      void* params, hipStream_t st) {
  FitArgs a;
  a.members = members;
  a.params = params;
  a.M = M;
  a.H = f.H;
  a.W = f.W;
  a.nb = f.nb;
  a.ddof = ddof;
  a.rs = f.rs;
  a.ps = f.plane();
  a.wscale = fit_wscale(f.model, M, ddof, bw);
  a.eps = eps;
  if (f.model == CP_MVGAUSS) {
    dim3 grid((a.W + kFitTX - 1) / kFitTX, (a.H + kFitTY - 1) / kFitTY);
    hipLaunchKernelGGL(k_fit_mean, grid, dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fit_mvg, grid, dim3(256), 0, st, a, jitter);
    return hipGetLastError();
  }
  if (f.dtype == CP_F64) return fit_typed<double>(a, f.model, st);
  return fit_typed<float>(a, f.model, st);
}

}  // namespace cp
