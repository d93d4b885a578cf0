// cp_gauss.hpp -- independent Gaussian model (the parametric comparison
// model of Sec. 5.2: per-vertex N(mu, sigma^2) from the member mean and
// standard deviation).
//
// The paper notes that the Gaussian has no closed form (Sec. 4.3) and samples
// it by Monte Carlo.  Here the 1-D integrals of Eq. 3 / Eq. 4,
//   P_min = int phi_v S_e S_n S_w S_s,  P_max = int phi_v F_e F_n F_w F_s,
//   t1 = int phi_v S_e F_n S_w F_s,     t2 = int phi_v F_e S_n F_w S_s,
// are evaluated deterministically in one sweep.  Coordinates are in units of
// the vertex: t = (x - mu_v) / sigma_v, so phi_v dt is the standard normal
// and neighbour n enters through z_n = (t - d_n) r_n with
// d_n = (mu_n - mu_v) / sigma_v and r_n = sigma_v / sigma_n.
// The sweep covers t in [-C, C] (the rest of phi weighs 2e-9 for C = 6 and
// 1.3e-17 for C = 8.5) and cuts it at the points d_n + c_k / r_n of every
// neighbour and c_k of the vertex, c_k running over K fixed multiples of the
// standard deviation in [-C, C].  Every panel therefore spans at most
// ~2 (FP32) or ~1.5 (FP64) standard deviations of every distribution that
// varies on it, and a fixed Gauss-Legendre rule of N nodes integrates it to
// ~1e-8 (FP32: C = 6, c = 0, +-2, +-4, +-6, N = 6) or ~1e-14 (FP64:
// C = 8.5, c = 0, +-1.5, +-3, +-4.5, +-6, +-8.5, N = 10) absolute over the
// whole integral.  S and F come from one erfc of |z|, so both tails keep full
// relative precision.  The cuts are merged on the fly by one cursor per
// distribution (each sequence is already sorted), as in the histogram sweep.
#pragma once

#include <cmath>

#include "cp_device.hpp"
#include "cp_mc_math.hpp"

namespace cp {

template <typename T>
struct GaussRule;
template <>
struct GaussRule<float> {
  static constexpr int K = 7, N = 6;
  static constexpr float c[7] = {-6.f, -4.f, -2.f, 0.f, 2.f, 4.f, 6.f};
};
template <>
struct GaussRule<double> {
  static constexpr int K = 11, N = 10;
  static constexpr double c[11] = {-8.5, -6.0, -4.5, -3.0, -1.5, 0.0, 1.5, 3.0, 4.5, 6.0, 8.5};
};

// erfc(x) for x >= 0 and e^x for x <= 0 (the only arguments here).  FP32 on
// the device: the hardware-instruction forms of cp_mc_math.hpp (fractional
// error below ~2e-7, against ~1e-7 for the library functions); FP64 and
// host code: the C library.
CP_HD float gerfc(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return erfc_pos(x);
#else
  return erfcf(x);
#endif
}
CP_HD double gerfc(double x) { return erfc(x); }
CP_HD float gexp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return exp_neg(x);
#else
  return expf(x);
#endif
}
CP_HD double gexp(double x) { return exp(x); }

// out = (P_min, P_max, t1, t2) of a vertex with valid parameters; neighbour
// order e, n, w, s; absent neighbours contribute 1; the saddle terms are
// computed only when `interior` (all four present) and are 0 otherwise.
template <typename T>
CP_HD void gauss_vertex(T mv, T sv, const T (&mn)[4], const T (&sn)[4], const bool (&pres)[4], T (&out)[4]) {
  using R = GaussRule<T>;
  constexpr int K = R::K, N = R::N;
  constexpr T C = R::c[K - 1];
  const T big = T(4) * C;  // beyond every panel end
  const T isv = crcp(sv);
  T d[4], s[4], r[4], nx[4];
  int k[4];
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    d[n] = (mn[n] - mv) * isv;
    s[n] = sn[n] * isv;
    r[n] = sv * crcp(sn[n]);
    k[n] = 0;
    nx[n] = pres[n] ? cfma(T(R::c[0]), s[n], d[n]) : big;
    // skip the cuts at or below the window start
    for (int q = 0; q < K && pres[n] && !(nx[n] > -C); ++q) {
      k[n] += 1;
      nx[n] = k[n] < K ? cfma(T(R::c[k[n]]), s[n], d[n]) : big;
    }
  }
  int kv = 1;
  T nv = T(R::c[1]);
  T x0 = -C;
  T acc[4] = {T(0), T(0), T(0), T(0)};
  constexpr T rs2 = T(0.70710678118654752440);
  for (int it = 0; it < 5 * K; ++it) {
    if (!(x0 < C)) break;
    T x1 = nv;
#pragma unroll
    for (int n = 0; n < 4; ++n) x1 = tmin(x1, nx[n]);
    const T mid = (x0 + x1) * T(0.5), hl = (x1 - x0) * T(0.5);
    T p[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const T t = cfma(hl, T(GL<N>::x[j]), mid);
      const T phi = T(GL<N>::w[j]) * gexp(T(-0.5) * t * t);
      T q0 = phi, q1 = phi, q2 = phi, q3 = phi;
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        if (!pres[n]) continue;
        const T z = (t - d[n]) * r[n];
        const T e = T(0.5) * gerfc(fabs(z) * rs2);
        const T S = z > T(0) ? e : T(1) - e;
        const T F = z > T(0) ? T(1) - e : e;
        q0 *= S;
        q1 *= F;
        // e, w (n = 0, 2) take S in t1 and F in t2; n, s the reverse
        q2 *= (n & 1) ? F : S;
        q3 *= (n & 1) ? S : F;
      }
      p[0] += q0;
      p[1] += q1;
      p[2] += q2;
      p[3] += q3;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = cfma(p[q], hl, acc[q]);
    // advance every cursor that sits at x1
    if (nv == x1) {
      kv += 1;
      nv = kv < K ? T(R::c[kv]) : big;
    }
#pragma unroll
    for (int n = 0; n < 4; ++n)
      if (nx[n] == x1) {
        k[n] += 1;
        nx[n] = k[n] < K ? cfma(T(R::c[k[n]]), s[n], d[n]) : big;
      }
    x0 = x1;
  }
  constexpr T inv_sqrt_2pi = T(0.39894228040143267794);
  const bool interior = pres[0] && pres[1] && pres[2] && pres[3];
  out[0] = acc[0] * inv_sqrt_2pi;
  out[1] = acc[1] * inv_sqrt_2pi;
  out[2] = interior ? acc[2] * inv_sqrt_2pi : T(0);
  out[3] = interior ? acc[3] * inv_sqrt_2pi : T(0);
}

// Weighted Jacobian of one stencil: jac[2 slot + q] = g_min dP_min/dtheta_q
// + g_max dP_max/dtheta_q, theta = (mu, sigma), slots v, e, n, w, s (absent
// neighbours: 0); also P_min and P_max.  In vertex units, with
// p_n(x) = phi(z_n) / sigma_n the density of neighbour n:
//   dP_min/dmu_n    = int phi(t) p_n prod_{k!=n} S_k dt,
//   dP_min/dsigma_n = int phi(t) p_n z_n prod_{k!=n} S_k dt,
// and for P_max the same with F and the opposite sign (dF = -dS).  The
// vertex slot follows from translation invariance (dP/dmu_v = -sum_n
// dP/dmu_n) and scale invariance about mu_v (sigma_v dP/dsigma_v = -sum_n
// ((mu_n - mu_v) dP/dmu_n + sigma_n dP/dsigma_n)).  Same panels and rule as
// gauss_vertex; the leave-one-out products come from prefix / suffix
// products.
template <typename T>
CP_HD void gauss_vertex_jac(T mv, T sv, const T (&mn)[4], const T (&sn)[4], const bool (&pres)[4], T gmin,
                            T gmax, T (&jac)[10], T& pmin, T& pmax) {
  using R = GaussRule<T>;
  // Positions (panel ends, nodes, z_n) in FP64 for both dtypes: in FP32 a
  // node's t carries half an ulp of |t| <= 6 (2.4e-7), which z_n multiplies
  // by sigma_v / sigma_n; the derivative integrands p_n z_n would inherit a
  // relative error of that size for narrow neighbours.  The factors
  // themselves (erfc, exp) and the sums stay in T.
  using P = double;
  constexpr int K = R::K, N = R::N;
  constexpr P C = R::c[K - 1];
  const P big = P(4) * C;
  const P isv = P(1) / P(sv);
  P d[4], s[4], r[4], nx[4];
  int k[4];
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    d[n] = (P(mn[n]) - P(mv)) * isv;
    s[n] = P(sn[n]) * isv;
    r[n] = P(sv) / P(sn[n]);
    k[n] = 0;
    nx[n] = pres[n] ? cfma(P(R::c[0]), s[n], d[n]) : big;
    for (int q = 0; q < K && pres[n] && !(nx[n] > -C); ++q) {
      k[n] += 1;
      nx[n] = k[n] < K ? cfma(P(R::c[k[n]]), s[n], d[n]) : big;
    }
  }
  int kv = 1;
  P nv = P(R::c[1]);
  P x0 = -C;
  // panel sums in T (z_n keeps its sign on a panel: its mean is a cut), the
  // sums over panels in FP64: dP/dsigma_n cancels between the panels below
  // and above the neighbour's mean.  The upstream weights enter at every
  // node (g_min times the S integrand, -g_max times the F one, one sum per
  // derivative): half the accumulators of separate P_min and P_max sums.
  P fS = P(0), fF = P(0);
  P a[4] = {P(0), P(0), P(0), P(0)}, b[4] = {P(0), P(0), P(0), P(0)};
  const T ngmax = -gmax;
  constexpr T rs2 = T(0.70710678118654752440);
  for (int it = 0; it < 5 * K; ++it) {
    if (!(x0 < C)) break;
    P x1 = nv;
#pragma unroll
    for (int n = 0; n < 4; ++n) x1 = tmin(x1, nx[n]);
    const P mid = (x0 + x1) * P(0.5), hlp = (x1 - x0) * P(0.5);
    const T hl = T(hlp);
    T pS = T(0), pF = T(0), qa[4], qb[4];
#pragma unroll
    for (int n = 0; n < 4; ++n) qa[n] = qb[n] = T(0);
    // the node loop stays a loop (the rule's nodes and weights are read from
    // constant memory): unrolled, its live values do not fit the registers
#pragma unroll 1
    for (int j = 0; j < N; ++j) {
      const P tp = cfma(hlp, P(GL<N>::x[j]), mid);
      const T t = T(tp);
      const T phi = T(GL<N>::w[j]) * gexp(T(-0.5) * t * t);
      T S[4], F[4], z[4], pz[4];
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        S[n] = F[n] = T(1);
        z[n] = pz[n] = T(0);
        if (!pres[n]) continue;
        z[n] = T((tp - d[n]) * r[n]);
        const T e = T(0.5) * gerfc(fabs(z[n]) * rs2);
        S[n] = z[n] > T(0) ? e : T(1) - e;
        F[n] = z[n] > T(0) ? T(1) - e : e;
        pz[n] = gexp(T(-0.5) * z[n] * z[n]);
      }
      // prefix products carry the node weight and the vertex density
      T preS[5], preF[5], sufS[5], sufF[5];
      preS[0] = preF[0] = phi;
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        preS[n + 1] = preS[n] * S[n];
        preF[n + 1] = preF[n] * F[n];
      }
      sufS[4] = sufF[4] = T(1);
#pragma unroll
      for (int n = 3; n >= 0; --n) {
        sufS[n] = sufS[n + 1] * S[n];
        sufF[n] = sufF[n + 1] * F[n];
      }
      pS += preS[4];
      pF += preF[4];
#pragma unroll
      for (int n = 0; n < 4; ++n) {
        const T l = pz[n] * cfma(gmin, preS[n] * sufS[n + 1], ngmax * (preF[n] * sufF[n + 1]));
        qa[n] += l;
        qb[n] = cfma(l, z[n], qb[n]);
      }
    }
    fS = cfma(P(pS), hlp, fS);
    fF = cfma(P(pF), hlp, fF);
#pragma unroll
    for (int n = 0; n < 4; ++n) {
      a[n] = cfma(P(qa[n]), hlp, a[n]);
      b[n] = cfma(P(qb[n]), hlp, b[n]);
    }
    if (nv == x1) {
      kv += 1;
      nv = kv < K ? P(R::c[kv]) : big;
    }
#pragma unroll
    for (int n = 0; n < 4; ++n)
      if (nx[n] == x1) {
        k[n] += 1;
        nx[n] = k[n] < K ? cfma(P(R::c[k[n]]), s[n], d[n]) : big;
      }
    x0 = x1;
  }
  constexpr T inv_sqrt_2pi = T(0.39894228040143267794), inv_2pi = T(0.15915494309189533577);
  pmin = T(fS * P(inv_sqrt_2pi));
  pmax = T(fF * P(inv_sqrt_2pi));
  // the vertex slot sums terms that cancel (the invariances): in FP64
  P smu = P(0), ssg = P(0);
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    jac[2 + 2 * n] = jac[3 + 2 * n] = T(0);
    if (!pres[n]) continue;
    const P c = P(inv_2pi) / P(sn[n]);
    const P dmu = c * a[n];  // g-weighted dP/dmu_n
    const P dsg = c * b[n];  // g-weighted dP/dsigma_n
    jac[2 + 2 * n] = T(dmu);
    jac[3 + 2 * n] = T(dsg);
    smu += dmu;
    ssg = cfma(d[n], dmu, cfma(s[n], dsg, ssg));
  }
  jac[0] = T(-smu);
  jac[1] = T(-ssg);
}

}  // namespace cp
