// cp_probes.hip -- measurement probes for the benchmark (libcpprobes.so, not
// part of the library's interface): the ceilings the hot-path kernels are
// compared with, measured on the same GPU in the same run.
//   cpb_mc_ceiling  the random-number and transcendental work of one sample of
//                   the conditional Monte Carlo estimator, with nothing else:
//                   one Philox4x32-10 block, two Box-Muller pairs, two normal
//                   CDFs (the adjoint: two normal densities), the same
//                   functions as the estimator (cp_mc_math.hpp), the
//                   FP64 accumulation, one wave64 per vertex and the wave
//                   reduction -- the estimator's launch shape without the
//                   stencil (mean, Cholesky product, min / max, gradients).
//   cpb_fma_peak    FP32 fused multiply-adds (plain, not packed), 1 to 16
//                   independent chains per lane: the vector FP32 ceiling.
//   cpb_copy        a 16-byte-per-lane copy: the reachable HBM bandwidth.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "cp_mc_math.hpp"
#include "cp_philox.hpp"

namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <bool PDF>
__global__ __launch_bounds__(256) void k_mc_ceiling(int nv, int ns, uint32_t k0, uint32_t k1, uint32_t fid,
                                                   double* out) {
  const int lane = threadIdx.x & 63;
  const int v = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (v >= nv) return;
  double a = 0.0, b = 0.0;
  for (int i = lane; i < ns; i += 64) {
    uint32_t c[4] = {(uint32_t)i, (uint32_t)v, fid, 0u};
    cp::philox(c, k0, k1);
    float z[4];
    cp::box_muller(cp::u24_of<float>(c[0]), cp::u24_of<float>(c[1]), z[0], z[1]);
    cp::box_muller(cp::u24_of<float>(c[2]), cp::u24_of<float>(c[3]), z[2], z[3]);
    const float r0 = z[1] - z[0], r1 = z[3] - z[2];
    if (PDF) {
      a += (double)cp::phi_pdf(r0);
      b += (double)cp::phi_pdf(r1);
    } else {
      a += (double)cp::phi_cdf(r0);
      b += (double)cp::phi_cdf(r1);
    }
  }
  a = wave_sum(a);
  b = wave_sum(b);
  if (lane == 0) {
    out[2 * (int64_t)v] = a / ns;
    out[2 * (int64_t)v + 1] = b / ns;
  }
}

template <int C>
__global__ __launch_bounds__(256) void k_fma_peak(int iters, float seed, float* out) {
  float x[C];
#pragma unroll
  for (int k = 0; k < C; ++k) x[k] = seed + (float)(threadIdx.x + k);
  const float m = 0.999999f, c = 1e-7f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < C; ++k) x[k] = fmaf(x[k], m, c);
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < C; ++k) s += x[k];
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

typedef float f4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_copy(int64_t n4, const f4* __restrict__ src, f4* __restrict__ dst) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

}  // namespace

extern "C" {

// pdf = 0: normal CDFs (the forward's per-sample work), 1: normal densities
// (the adjoint's).  out: [nv][2] doubles (means of the two columns, so
// nothing is dead code)
int cpb_mc_ceiling(int nv, int ns, uint64_t seed, uint32_t fid, int pdf, double* out, void* stream) {
  if (nv < 1 || ns < 1 || !out) return 1;
  const dim3 grid((unsigned)((nv + 3) / 4));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (pdf)
    hipLaunchKernelGGL(k_mc_ceiling<true>, grid, dim3(256), 0, st, nv, ns, (uint32_t)seed, (uint32_t)(seed >> 32),
                       fid, out);
  else
    hipLaunchKernelGGL(k_mc_ceiling<false>, grid, dim3(256), 0, st, nv, ns, (uint32_t)seed,
                       (uint32_t)(seed >> 32), fid, out);
  return hipGetLastError() == hipSuccess ? 0 : 2;
}

// blocks x 256 threads, each `chains` (1, 2, 4, 8 or 16) independent chains
// of iters FMAs; out: blocks * 256 floats
int cpb_fma_peak(int blocks, int iters, int chains, float* out, void* stream) {
  if (blocks < 1 || iters < 1 || !out) return 1;
  hipStream_t st = static_cast<hipStream_t>(stream);
  switch (chains) {
    case 1: hipLaunchKernelGGL(k_fma_peak<1>, dim3((unsigned)blocks), dim3(256), 0, st, iters, 1.0f, out); break;
    case 2: hipLaunchKernelGGL(k_fma_peak<2>, dim3((unsigned)blocks), dim3(256), 0, st, iters, 1.0f, out); break;
    case 4: hipLaunchKernelGGL(k_fma_peak<4>, dim3((unsigned)blocks), dim3(256), 0, st, iters, 1.0f, out); break;
    case 8: hipLaunchKernelGGL(k_fma_peak<8>, dim3((unsigned)blocks), dim3(256), 0, st, iters, 1.0f, out); break;
    case 16: hipLaunchKernelGGL(k_fma_peak<16>, dim3((unsigned)blocks), dim3(256), 0, st, iters, 1.0f, out); break;
    default: return 1;
  }
  return hipGetLastError() == hipSuccess ? 0 : 2;
}

// n4 float4 elements from src to dst (16-byte aligned)
int cpb_copy(int64_t n4, const void* src, void* dst, void* stream) {
  if (n4 < 1 || !src || !dst) return 1;
  hipLaunchKernelGGL(k_copy, dim3(256 * 16), dim3(256), 0, static_cast<hipStream_t>(stream), n4,
                     static_cast<const f4*>(src), static_cast<f4*>(dst));
  return hipGetLastError() == hipSuccess ? 0 : 2;
}

}  // extern "C"
