// cp_mc_math.hpp -- per-sample math of the Gaussian Monte Carlo estimators
// (normal deviates from uniforms, the normal CDF and density), on the
// hardware transcendental instructions of gfx950; erfc_pos and exp_neg also
// serve the FP32 independent-Gaussian quadrature.
//
// Measured against FP64 on the generator's uniforms: v_sin_f32 / v_cos_f32
// (argument in revolutions) 1.3e-7 absolute, v_sqrt_f32 9e-8, v_exp_f32
// 8e-8 and v_rcp_f32 9e-8 relative; v_log_f32 within one ulp of log2.
// The normal CDF uses the complementary error function of Numerical Recipes
// (Press et al., 2nd ed., Sec. 6.2, routine erfcc: a Chebyshev fit of
// log(erfc) with fractional error below 1.2e-7 everywhere), so one CDF costs
// a reciprocal, nine fused multiply-adds and one exponential.
#pragma once

#include <hip/hip_runtime.h>

namespace cp {

// Box-Muller: (u0, u1) in (0, 1] -> two independent N(0, 1) deviates
__device__ __forceinline__ void box_muller(float u0, float u1, float& z0, float& z1) {
  constexpr float kMinus2Ln2 = -1.3862943611198906f;  // -2 ln 2 (log2 -> ln)
  const float rad = __builtin_amdgcn_sqrtf(kMinus2Ln2 * __builtin_amdgcn_logf(u0));
  z0 = rad * __builtin_amdgcn_cosf(u1);  // cos(2 pi u1)
  z1 = rad * __builtin_amdgcn_sinf(u1);  // sin(2 pi u1)
}

// e^y for y <= 0 (the arguments here), through exp2
__device__ __forceinline__ float exp_neg(float y) { return __builtin_amdgcn_exp2f(y * 1.4426950408889634f); }

// erfc(x), x >= 0
__device__ __forceinline__ float erfc_pos(float x) {
  const float t = __builtin_amdgcn_rcpf(fmaf(0.5f, x, 1.0f));
  float p = 0.17087277f;
  p = fmaf(p, t, -0.82215223f);
  p = fmaf(p, t, 1.48851587f);
  p = fmaf(p, t, -1.13520398f);
  p = fmaf(p, t, 0.27886807f);
  p = fmaf(p, t, -0.18628806f);
  p = fmaf(p, t, 0.09678418f);
  p = fmaf(p, t, 0.37409196f);
  p = fmaf(p, t, 1.00002368f);
  p = fmaf(p, t, -1.26551223f);
  return t * exp_neg(fmaf(-x, x, p));
}

// standard normal CDF and density
__device__ __forceinline__ float phi_cdf(float r) {
  const float h = 0.5f * erfc_pos(fabsf(r) * 0.70710678118654752f);  // upper tail of |r|
  return r < 0.0f ? h : 1.0f - h;
}
__device__ __forceinline__ float phi_pdf(float r) { return 0.39894228040143268f * exp_neg(-0.5f * r * r); }

}  // namespace cp
