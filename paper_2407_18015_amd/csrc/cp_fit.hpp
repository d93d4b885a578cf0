// cp_fit.hpp -- per-vertex fitting arithmetic of the range and
// location-scale models, and the correctly rounded helpers of the fits.
//
// Rules (Sec. 5.1 and 5.2):
//   uniform       lo = min, hi = max of the members
//   Epanechnikov  m = mean, w = bw * std(ddof) * M^(-1/5)
//   Gaussian      mu = mean, sigma = std(ddof)  (the Epanechnikov arithmetic
//                 with another scale)
//   degenerate    all members equal: lo/hi = x -/+ eps*max(1,|x|), Epanechnikov
//                 w (Gaussian sigma) = eps*max(1,|m|)
// Statistics are accumulated in FP64 about the first member (shifted sums).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "cpcrit.h"

namespace cp {

template <typename T>
__device__ __forceinline__ T rn_sub(T a, T b);
template <>
__device__ __forceinline__ float rn_sub(float a, float b) {
  return __fsub_rn(a, b);
}
template <>
__device__ __forceinline__ double rn_sub(double a, double b) {
  return __dsub_rn(a, b);
}
template <typename T>
__device__ __forceinline__ T rn_add(T a, T b);
template <>
__device__ __forceinline__ float rn_add(float a, float b) {
  return __fadd_rn(a, b);
}
template <>
__device__ __forceinline__ double rn_add(double a, double b) {
  return __dadd_rn(a, b);
}
template <typename T>
__device__ __forceinline__ T rn_mul(T a, T b);
template <>
__device__ __forceinline__ float rn_mul(float a, float b) {
  return __fmul_rn(a, b);
}
template <>
__device__ __forceinline__ double rn_mul(double a, double b) {
  return __dmul_rn(a, b);
}
template <typename T>
__device__ __forceinline__ T rn_div(T a, T b);
template <>
__device__ __forceinline__ float rn_div(float a, float b) {
  return __fdiv_rn(a, b);
}
template <>
__device__ __forceinline__ double rn_div(double a, double b) {
  return __ddiv_rn(a, b);
}

// degenerate half-width of the range model: eps * max(1, |x|), rounded once
template <typename T>
__device__ __forceinline__ T degenerate_half(T eps, T x) {
  return rn_mul(eps, x < T(0) ? (-x > T(1) ? -x : T(1)) : (x > T(1) ? x : T(1)));
}

// Running statistics of one vertex's members, then its parameters.
// Uniform: (lo, hi) = (min, max); Epanechnikov / Gaussian: (m, w) with
// w = wscale * sqrt(sum of squared deviations).  Every fit kernel feeds the
// members of a vertex in order k = 0, 1, ..., M-1 through these operations,
// so all of them give the same parameters bit for bit.
//
// The Epanechnikov branch detects "all members equal" without a min / max:
// with x0 the first member and d = x - x0 in FP64, some member differs from
// x0 exactly when some |d| > 0 (the difference of two distinct values of the
// field's type is never 0 in FP64).  A NaN member gives a NaN d, which the
// test ignores, as the min / max comparisons ignore it; a NaN first member
// makes every d NaN: degenerate, as !(min < max) is then.
template <typename T, int MODEL>
struct FitAcc {
  T mn, mx;
  double shift, s1, s2;
  bool spread;
  __device__ __forceinline__ void first(T x0) {
    if (MODEL == CP_UNIFORM) {
      mn = mx = x0;
    } else {
      shift = (double)x0;
      s1 = s2 = 0.0;
      spread = false;
    }
  }
  __device__ __forceinline__ void add(T xk) {
    if (MODEL == CP_UNIFORM) {
      mn = xk < mn ? xk : mn;
      mx = xk > mx ? xk : mx;
    } else {
      const double d = (double)xk - shift;
      spread = spread || fabs(d) > 0.0;
      s1 += d;
      s2 = fma(d, d, s2);
    }
  }
  __device__ __forceinline__ void finish(int M, double wscale, double eps, T& p0, T& p1) const {
    if (MODEL == CP_UNIFORM) {
      if (!(mn < mx)) {
        const T e = degenerate_half(T(eps), mn);
        p0 = rn_sub(mn, e);
        p1 = rn_add(mn, e);
      } else {
        p0 = mn;
        p1 = mx;
      }
      return;
    }
    const double mean = shift + s1 / (double)M;
    double w;
    if (!spread) {
      w = eps * fmax(1.0, fabs(mean));
    } else {
      const double ss = fmax(s2 - s1 * s1 / (double)M, 0.0);
      w = wscale * sqrt(ss);
    }
    p0 = (T)mean;
    p1 = (T)w;
  }
};

// Parameters (p0, p1) of one vertex from its M members, member k at
// mem[at + k*ps].
template <typename T, int MODEL>
__device__ __forceinline__ void fit_ue_vertex(const T* __restrict__ mem, int M, int64_t ps, int64_t at,
                                              double wscale, double eps, T& p0, T& p1) {
  FitAcc<T, MODEL> acc;
  acc.first(mem[at]);
#pragma unroll 4
  for (int k = 1; k < M; ++k) acc.add(mem[(int64_t)k * ps + at]);
  acc.finish(M, wscale, eps, p0, p1);
}

}  // namespace cp
