// cp_mvg.hip -- multivariate Gaussian over the 5-point stencil, Monte Carlo.
//
// The paper compares its closed forms with the correlated Gaussian model of
// prior work, sampled by Monte Carlo (Sec. 5.2: 1000 samples; Sec. 5.3: 2000
// samples).  Here each vertex owns one wave64; lane l takes samples l, l+64,
// ...; the stencil's mean and Cholesky factor are wave-uniform.
//
// Sample i of vertex (y, x): Philox4x32-10 with counter (i, y*W+x, field_id,
// b) and key (seed lo, seed hi); the four words of block b = 0 give uniforms
// u0..u3, words 0-1 of block 1 give u4, u5, each u = (r >> 8 + 1/2) 2^-24.
// Box-Muller pairs (u0,u1), (u2,u3), (u4,u5) give z0..z4, which drive
// (e, n, w, s, v): x = mu + L z.
//   hit estimator:         [x_v < min_n x_n]              (needs block 1)
//   conditional estimator: Phi((min_n x_n - c) / L44),   c = mu_v + sum_{j<4} L4j z_j
// The conditional estimator integrates the vertex given its neighbours in
// closed form (the paper's semianalytical idea of Sec. 4.4.2: sample part of
// the stencil, integrate the rest), has the same expectation, lower variance,
// needs one Philox block per sample, and is differentiable: the adjoint is
// its pathwise derivative.  Maxima use Phi((c - max_n x_n) / L44).
#include <hip/hip_runtime.h>

#include "cp_internal.hpp"
#include "cp_mc_math.hpp"
#include "cp_philox.hpp"

namespace cp {

namespace {

__device__ __forceinline__ float u24(uint32_t r) { return u24_of<float>(r); }


template <typename V>
__device__ __forceinline__ V wave_sum(V v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

struct MvgArgs {
  const double* par;
  float* pmin;
  float* pmax;
  const float* gmin;
  const float* gmax;
  double* grad;
  double* jmu;  // [5][H][W] workspace (adjoint)
  int H, W, ns, est;
  int64_t rs, ps;
  uint32_t k0, k1, fid;
};

// Wave-uniform stencil in the vertex's local frame (origin mu_v).
struct MvgStencil {
  float d[4];      // mu_n - mu_v
  float L[15];     // packed lower triangle over (e, n, w, s, v)
  bool pres[4];
  float iL44;
};

__device__ __forceinline__ void load_stencil(const MvgArgs& a, int y, int x, MvgStencil& s) {
  const int64_t at = (int64_t)y * a.rs + x;
  const double mv = a.par[at];
  const int dy[4] = {0, -1, 0, 1}, dx[4] = {1, 0, -1, 0};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int yy = y + dy[i], xx = x + dx[i];
    s.pres[i] = yy >= 0 && yy < a.H && xx >= 0 && xx < a.W;
    s.d[i] = s.pres[i] ? (float)(a.par[(int64_t)yy * a.rs + xx] - mv) : 0.0f;
  }
#pragma unroll
  for (int k = 0; k < 15; ++k) s.L[k] = (float)a.par[(int64_t)(1 + k) * a.ps + at];
  s.iL44 = 1.0f / s.L[14];
}

// x_n (local) for the four neighbours and the conditional mean c of v
__device__ __forceinline__ void stencil_values(const MvgStencil& s, const float z[4], float xn[4], float& c) {
  const float* L = s.L;
  xn[0] = s.d[0] + L[0] * z[0];
  xn[1] = s.d[1] + L[1] * z[0] + L[2] * z[1];
  xn[2] = s.d[2] + L[3] * z[0] + L[4] * z[1] + L[5] * z[2];
  xn[3] = s.d[3] + L[6] * z[0] + L[7] * z[1] + L[8] * z[2] + L[9] * z[3];
  c = L[10] * z[0] + L[11] * z[1] + L[12] * z[2] + L[13] * z[3];
}

__global__ __launch_bounds__(256) void k_mvg_fwd(MvgArgs a) {
  const int lane = threadIdx.x & 63;
  const int v = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (v >= a.H * a.W) return;
  const int y = v / a.W, x = v - y * a.W;
  MvgStencil s;
  load_stencil(a, y, x, s);
  double smin = 0.0, smax = 0.0;
  for (int i = lane; i < a.ns; i += 64) {
    uint32_t c0[4] = {(uint32_t)i, (uint32_t)v, a.fid, 0u};
    philox(c0, a.k0, a.k1);
    float z[4];
    box_muller(u24(c0[0]), u24(c0[1]), z[0], z[1]);
    box_muller(u24(c0[2]), u24(c0[3]), z[2], z[3]);
    float xn[4], cm;
    stencil_values(s, z, xn, cm);
    float lo = __builtin_inff(), hi = -__builtin_inff();
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (s.pres[k]) {
        lo = fminf(lo, xn[k]);
        hi = fmaxf(hi, xn[k]);
      }
    if (a.est == CP_MC_HIT) {
      uint32_t c1[4] = {(uint32_t)i, (uint32_t)v, a.fid, 1u};
      philox(c1, a.k0, a.k1);
      float z4, z5;
      box_muller(u24(c1[0]), u24(c1[1]), z4, z5);
      const float xv = cm + s.L[14] * z4;
      smin += xv < lo ? 1.0 : 0.0;
      smax += xv > hi ? 1.0 : 0.0;
    } else {
      smin += (double)phi_cdf((lo - cm) * s.iL44);
      smax += (double)phi_cdf((cm - hi) * s.iL44);
    }
  }
  smin = wave_sum(smin);
  smax = wave_sum(smax);
  if (lane == 0) {
    const int64_t at = (int64_t)y * a.rs + x;
    a.pmin[at] = (float)(smin / (double)a.ns);
    a.pmax[at] = (float)(smax / (double)a.ns);
  }
}

// Pathwise derivative of the conditional estimator.  With n* the argmin,
// r = (x_n* - c)/L44:  dr/dmu_n* = 1/L44, dr/dmu_v = -1/L44,
// dr/dL_n*j = z_j/L44, dr/dL_4j = -z_j/L44 (j<4), dr/dL44 = -r/L44; the
// maximum mirrors it.  L is local to the stencil (written directly); the
// mean plane is shared by five stencils, so its per-stencil partials go to a
// workspace and a second kernel gathers them.
__global__ __launch_bounds__(256) void k_mvg_bwd(MvgArgs a) {
  const int lane = threadIdx.x & 63;
  const int v = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (v >= a.H * a.W) return;
  const int y = v / a.W, x = v - y * a.W;
  MvgStencil s;
  load_stencil(a, y, x, s);
  const int64_t at = (int64_t)y * a.rs + x;
  const float gmn = a.gmin[at] * s.iL44, gmx = a.gmax[at] * s.iL44;
  float dmu[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
  float dl[15];
#pragma unroll
  for (int k = 0; k < 15; ++k) dl[k] = 0.f;
  for (int i = lane; i < a.ns; i += 64) {
    uint32_t c0[4] = {(uint32_t)i, (uint32_t)v, a.fid, 0u};
    philox(c0, a.k0, a.k1);
    float z[4];
    box_muller(u24(c0[0]), u24(c0[1]), z[0], z[1]);
    box_muller(u24(c0[2]), u24(c0[3]), z[2], z[3]);
    float xn[4], cm;
    stencil_values(s, z, xn, cm);
    float lo = __builtin_inff(), hi = -__builtin_inff();
    int amin = -1, amax = -1;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (s.pres[k]) {
        if (amin < 0 || xn[k] < lo) {
          lo = xn[k];
          amin = k;
        }
        if (amax < 0 || xn[k] > hi) {
          hi = xn[k];
          amax = k;
        }
      }
    if (amin < 0) continue;  // no neighbours: the estimate is the constant 1
    const float rmin = (lo - cm) * s.iL44, rmax = (cm - hi) * s.iL44;
    const float gm = gmn * phi_pdf(rmin), gx = gmx * phi_pdf(rmax);
    float cr[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) cr[r] = (amin == r ? gm : 0.f) - (amax == r ? gx : 0.f);
#pragma unroll
    for (int r = 0; r < 4; ++r) dmu[1 + r] += cr[r];
    dmu[0] += gx - gm;
    // rows 0..3 (packed offsets 0, 1, 3, 6)
    dl[0] = fmaf(cr[0], z[0], dl[0]);
    dl[1] = fmaf(cr[1], z[0], dl[1]);
    dl[2] = fmaf(cr[1], z[1], dl[2]);
    dl[3] = fmaf(cr[2], z[0], dl[3]);
    dl[4] = fmaf(cr[2], z[1], dl[4]);
    dl[5] = fmaf(cr[2], z[2], dl[5]);
    dl[6] = fmaf(cr[3], z[0], dl[6]);
    dl[7] = fmaf(cr[3], z[1], dl[7]);
    dl[8] = fmaf(cr[3], z[2], dl[8]);
    dl[9] = fmaf(cr[3], z[3], dl[9]);
    const float c4 = gx - gm;
#pragma unroll
    for (int j = 0; j < 4; ++j) dl[10 + j] = fmaf(c4, z[j], dl[10 + j]);
    dl[14] -= gm * rmin + gx * rmax;
  }
  const double inv = 1.0 / (double)a.ns;
  double out[20];
#pragma unroll
  for (int k = 0; k < 5; ++k) out[k] = wave_sum((double)dmu[k]);
#pragma unroll
  for (int k = 0; k < 15; ++k) out[5 + k] = wave_sum((double)dl[k]);
  if (lane == 0) {
    const int64_t plane = (int64_t)a.H * a.W, id = v;
#pragma unroll
    for (int k = 0; k < 5; ++k) a.jmu[k * plane + id] = out[k] * inv;
#pragma unroll
    for (int k = 0; k < 15; ++k) a.grad[(int64_t)(1 + k) * a.ps + at] = out[5 + k] * inv;
  }
}

// grad_mu(u) = J_v(u) + J_w(east) + J_e(west) + J_s(north) + J_n(south)
__global__ __launch_bounds__(256) void k_mvg_gather(MvgArgs a) {
  const int64_t id = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t plane = (int64_t)a.H * a.W;
  if (id >= plane) return;
  const int y = (int)(id / a.W), x = (int)(id - (int64_t)y * a.W);
  double g = a.jmu[id];
  if (x + 1 < a.W) g += a.jmu[3 * plane + id + 1];
  if (x > 0) g += a.jmu[1 * plane + id - 1];
  if (y > 0) g += a.jmu[4 * plane + id - a.W];
  if (y + 1 < a.H) g += a.jmu[2 * plane + id + a.W];
  a.grad[(int64_t)y * a.rs + x] = g;
}

__global__ __launch_bounds__(256) void k_philox_raw(int64_t n, const uint32_t* ctr, uint32_t k0, uint32_t k1,
                                                  uint32_t* out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  uint32_t c[4] = {ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
  philox(c, k0, k1);
#pragma unroll
  for (int k = 0; k < 4; ++k) out[4 * i + k] = c[k];
}

MvgArgs make_args(const Field& f, const double* params) {
  MvgArgs a{};
  a.par = params;
  a.H = f.H;
  a.W = f.W;
  a.ns = f.ns;
  a.est = f.est;
  a.rs = f.rs;
  a.ps = f.plane();
  a.k0 = (uint32_t)f.seed;
  a.k1 = (uint32_t)(f.seed >> 32);
  a.fid = f.fid;
  return a;
}

}  // namespace

hipError_t mvg_forward(const Field& f, const double* params, float* pmin, float* pmax, hipStream_t st) {
  MvgArgs a = make_args(f, params);
  a.pmin = pmin;
  a.pmax = pmax;
  const int64_t nv = (int64_t)f.H * f.W;
  hipLaunchKernelGGL(k_mvg_fwd, dim3((unsigned)((nv + 3) / 4)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t mvg_backward(const Field& f, const double* params, const float* gmin, const float* gmax, double* grad,
                        hipStream_t st, const Scratch& scr) {
  MvgArgs a = make_args(f, params);
  a.gmin = gmin;
  a.gmax = gmax;
  a.grad = grad;
  const int64_t nv = (int64_t)f.H * f.W;
  void* ws = nullptr;
  hipError_t e = adjoint_scratch(sizeof(double) * 5 * (size_t)nv, st, scr, &ws);
  if (e != hipSuccess) return e;
  a.jmu = static_cast<double*>(ws);
  hipLaunchKernelGGL(k_mvg_bwd, dim3((unsigned)((nv + 3) / 4)), dim3(256), 0, st, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mvg_gather, dim3((unsigned)((nv + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t philox_raw(int64_t n, const uint32_t* ctr, uint64_t seed, uint32_t* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_philox_raw, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, ctr, (uint32_t)seed,
                     (uint32_t)(seed >> 32), out);
  return hipGetLastError();
}

}  // namespace cp
