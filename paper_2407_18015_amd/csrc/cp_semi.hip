// cp_semi.hip -- semianalytical histogram estimator (Sec. 4.4.2).
//
// c samples are drawn from each vertex histogram; for each sample the
// probability that a neighbour lies above (below) it is closed-form: the
// neighbour's bin is found by one multiply, and the masses of the earlier
// bins come from cumulative sums prepared once per staged vertex (the paper's
// prefix-sum step), so the work per sample does not grow with the number of
// bins except for locating the sample's own bin.  The products are averaged:
//   P_min ~ T (1/c) sum_i prod_n S_n(x_i),   P_max ~ T (1/c) sum_i prod_n F_n(x_i),
//   t1 ~ T (1/c) sum_i S_e F_n S_w F_s(x_i), t2 with S and F exchanged,
// T = the vertex's total mass.  Sample i of vertex (y, x) uses word i mod 4 of
// Philox4x32-10 with counter (i / 4, y*W + x, field_id, 2) under key seed,
// u = ((word >> 8) + 1/2) 2^-24, r = u T, bin j = #{k in 1..h-1 : C_k <= r}
// (C_k = m_0 + ... + m_{k-1}), f = (r - C_j) / m_j clamped to [0, 1] (0 for an
// empty bin), x = lo + Delta (j + f): the inverse of the histogram CDF.
//
// Tiles of 64 x TY vertices stage lo, hi and the masses with a one-vertex
// halo (as the closed-form forward does) and replace the masses by the
// cumulative masses in place (FP64 running sums rounded once); a bin's mass
// is then the difference of its two cumulative values, which keeps the tile
// at 2 + h planes of LDS.  One thread per vertex loops over its samples.  Sample positions and neighbour tails are computed in FP64
// for both dtypes, in vertex-local coordinates: in FP32 a position carries
// an error of one unit in the last place of the distribution width, which
// is h units of a bin, and the neighbour's tail inherits it for every
// sample alike; FP64 arithmetic costs the same issue rate as FP32 here.
#include <hip/hip_runtime.h>

#include "cp_hist.hpp"
#include "cp_internal.hpp"
#include "cp_philox.hpp"
#include "cp_tiles.hpp"

namespace cp {

namespace {

template <typename T>
struct SemiArgs {
  const T* params;
  T* pmin;
  T* pmax;
  T* terms;  // [2][H][rs]: t1, t2
  int H, W, nb, ns;
  int64_t rs, ps;
  uint32_t k0, k1, fid;
};

template <typename T>
__device__ __forceinline__ T clamp01(T v) {
  return v < T(0) ? T(0) : (v > T(1) ? T(1) : v);
}

template <typename T, int TY>
__global__ __launch_bounds__(kFwdTX* TY) void k_semi(SemiArgs<T> a, int tiles_x, int ntiles) {
  constexpr int TX = kFwdTX, EX = TX + 2, EY = TY + 2, E = EX * EY, NT = TX * TY;
  extern __shared__ __align__(16) unsigned char smem[];
  T* lds = reinterpret_cast<T*>(smem);
  const int t = xcd_tile(blockIdx.x, ntiles);
  const int ty0 = (t / tiles_x) * TY, tx0 = (t % tiles_x) * TX, tid = threadIdx.x;
  const int h = a.nb;
  stage<T, EY, EX, NT>(lds, a.params, 2 + h, a.ps, a.rs, a.H, a.W, ty0 - 1, tx0 - 1, tid);
  __syncthreads();
  hist_stage_validity<T, NT>(lds, E, h, tid);
  // cumulative masses over the mass planes: plane k - 1 of `cum` holds C_k,
  // k = 1..h (C_h = T); the thread that checked a vertex sums it
  T* cum = lds + (size_t)2 * E;
  for (int e = tid; e < E; e += NT) {
    double c = 0.0;
    for (int k = 0; k < h; ++k) {
      c += (double)cum[k * E + e];
      cum[k * E + e] = (T)c;
    }
  }
  __syncthreads();
  const int lx = tid % TX, ly = tid / TX;
  const int x = tx0 + lx, y = ty0 + ly;
  if (x >= a.W || y >= a.H) return;
  const HistLds<T> L{lds, E, h, T(1) / T(h)};
  const int e = (ly + 1) * EX + lx + 1;
  const int en[4] = {e + 1, e - EX, e - 1, e + EX};
  const bool pres[4] = {x + 1 < a.W, y > 0, x > 0, y + 1 < a.H};
  bool ok = L.valid(e);
#pragma unroll
  for (int i = 0; i < 4; ++i) ok = ok && (!pres[i] || L.valid(en[i]));
  T out[4] = {qnan<T>(), qnan<T>(), qnan<T>(), qnan<T>()};
  if (ok) {
    using A = double;
    const A lov = (A)lds[e];
    const A dv = ((A)lds[E + e] - lov) / A(h);
    const T Tv = cum[(h - 1) * E + e];
    A lo[4], id[4], tot[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      lo[i] = (A)lds[en[i]] - lov;
      id[i] = A(h) / ((A)lds[E + en[i]] - (A)lds[en[i]]);
      tot[i] = (A)cum[(h - 1) * E + en[i]];
    }
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const uint32_t at = (uint32_t)((int64_t)y * a.W + x);
    uint32_t w[4] = {0u, 0u, 0u, 0u};
    for (int i = 0; i < a.ns; ++i) {
      if ((i & 3) == 0) {
        w[0] = (uint32_t)(i >> 2);
        w[1] = at;
        w[2] = a.fid;
        w[3] = 2u;
        philox(w, a.k0, a.k1);
      }
      const A r = u24_of<A>(w[i & 3]) * (A)Tv;
      int j = 0;
      for (int k = 1; k < h; ++k) j += (A)cum[(k - 1) * E + e] <= r ? 1 : 0;
      const A cj = j > 0 ? (A)cum[(j - 1) * E + e] : A(0);
      const A mj = (A)cum[j * E + e] - cj;
      const A f = mj > A(0) ? clamp01((r - cj) / mj) : A(0);
      const A xs = dv * (A(j) + f);
      A S[4], F[4];
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        S[n] = A(1);
        F[n] = A(1);
        if (!pres[n]) continue;
        const A z = (xs - lo[n]) * id[n];
        if (!(z > A(0))) {
          S[n] = tot[n];
          F[n] = A(0);
        } else if (!(z < A(h))) {
          S[n] = A(0);
          F[n] = tot[n];
        } else {
          const int k = min((int)z, h - 1);
          const A below = k > 0 ? (A)cum[(k - 1) * E + en[n]] : A(0);
          F[n] = fma((A)cum[k * E + en[n]] - below, z - A(k), below);
          S[n] = tot[n] - F[n];
        }
      }
      acc[0] += S[0] * S[1] * S[2] * S[3];
      acc[1] += F[0] * F[1] * F[2] * F[3];
      acc[2] += S[0] * F[1] * S[2] * F[3];
      acc[3] += F[0] * S[1] * F[2] * S[3];
    }
    const double sc = (double)Tv / (double)a.ns;
#pragma unroll
    for (int q = 0; q < 4; ++q) out[q] = (T)(acc[q] * sc);
    // the alternating pattern needs all four neighbours
    if (!(pres[0] && pres[1] && pres[2] && pres[3])) out[2] = out[3] = T(0);
  }
  const int64_t o = (int64_t)y * a.rs + x;
  if (a.pmin) a.pmin[o] = out[0];
  if (a.pmax) a.pmax[o] = out[1];
  if (a.terms) {
    a.terms[o] = out[2];
    a.terms[a.ps + o] = out[3];
  }
}

int cdiv_s(int p, int q) { return (p + q - 1) / q; }

template <typename T, int TY>
hipError_t launch_semi(const SemiArgs<T>& a, hipStream_t st) {
  const int tx = cdiv_s(a.W, kFwdTX), ty = cdiv_s(a.H, TY), n = tx * ty;
  const size_t lds = sizeof(T) * (size_t)(2 + a.nb) * (kFwdTX + 2) * (TY + 2);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_semi<T, TY>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_semi<T, TY>), dim3(n), dim3(kFwdTX * TY), lds, st, a, tx, n);
  return hipGetLastError();
}

template <typename T>
hipError_t semi_typed(const Field& f, const void* params, void* pmin, void* pmax, void* terms, hipStream_t st) {
  SemiArgs<T> a;
  a.params = static_cast<const T*>(params);
  a.pmin = static_cast<T*>(pmin);
  a.pmax = static_cast<T*>(pmax);
  a.terms = static_cast<T*>(terms);
  a.H = f.H;
  a.W = f.W;
  a.nb = f.nb;
  a.ns = f.ns;
  a.rs = f.rs;
  a.ps = f.plane();
  a.k0 = (uint32_t)f.seed;
  a.k1 = (uint32_t)(f.seed >> 32);
  a.fid = f.fid;
  // tile height: the staged planes (the masses overwritten by their
  // cumulative sums) must fit the LDS
  const size_t per_row = sizeof(T) * (size_t)(2 + f.nb) * (kFwdTX + 2);
  if (per_row * 6 <= 64 * 1024) return launch_semi<T, 4>(a, st);
  if (per_row * 4 <= 160 * 1024) return launch_semi<T, 2>(a, st);
  return launch_semi<T, 1>(a, st);
}

}  // namespace

hipError_t semi_forward(const Field& f, const void* params, void* pmin, void* pmax, void* terms, hipStream_t st) {
  if (f.dtype == CP_F64) return semi_typed<double>(f, params, pmin, pmax, terms, st);
  return semi_typed<float>(f, params, pmin, pmax, terms, st);
}

}  // namespace cp
