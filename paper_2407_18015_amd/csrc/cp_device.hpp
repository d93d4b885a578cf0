// cp_device.hpp -- device-side building blocks of the closed-form kernels.
//
// Every routine works in a vertex-local coordinate frame: all breakpoints
// are differences of parameters of nearby vertices, so their magnitude is
// the distribution width rather than the data value.  The paper warns that
// its high-order templates become unstable for large or fractional data
// values (Sec. 4.3); in FP32 a node placed in global coordinates near 0.5
// already carries 3e-8 of rounding, which is 5e-6 of a 0.006-wide
// Epanechnikov kernel.  In the local frame the error is relative to the
// widths, and nothing is ever expanded into monomials.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

// Pure arithmetic is host+device so it can also be exercised on the CPU.
#define CP_HD __host__ __device__ __forceinline__

namespace cp {

// Fused multiply-add in the operand precision (FP32 stays FP32).
template <typename T>
CP_HD T cfma(T a, T b, T c);
template <>
CP_HD float cfma<float>(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}
template <>
CP_HD double cfma<double>(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}

// Reciprocal: the hardware v_rcp_f32 (1 ulp) in FP32 device code, exact
// division otherwise.  Parameters are reciprocated once per vertex.
template <typename T>
CP_HD T crcp(T x) {
  return T(1) / x;
}
template <>
CP_HD float crcp<float>(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}

// ---------------------------------------------------------------------------
// Gauss-Legendre rules on [-1, 1]; an N-point rule integrates polynomials of
// degree <= 2N-1 exactly.
// ---------------------------------------------------------------------------
template <int N>
struct GL;
template <>
struct GL<1> {
  static constexpr double x[1] = {0.0};
  static constexpr double w[1] = {2.0};
};
template <>
struct GL<2> {
  static constexpr double x[2] = {-0.57735026918962576451, 0.57735026918962576451};
  static constexpr double w[2] = {1.0, 1.0};
};
template <>
struct GL<3> {
  static constexpr double x[3] = {-0.77459666924148337704, 0.0, 0.77459666924148337704};
  static constexpr double w[3] = {0.55555555555555555556, 0.88888888888888888889,
                                  0.55555555555555555556};
};
template <>
struct GL<4> {
  static constexpr double x[4] = {-0.86113631159405257522, -0.33998104358485626480, 0.33998104358485626480,
                                  0.86113631159405257522};
  static constexpr double w[4] = {0.34785484513745385737, 0.65214515486254614263, 0.65214515486254614263,
                                  0.34785484513745385737};
};
template <>
struct GL<5> {
  static constexpr double x[5] = {-0.90617984593866399280, -0.53846931010568309104, 0.0,
                                  0.53846931010568309104, 0.90617984593866399280};
  static constexpr double w[5] = {0.23692688505618908751, 0.47862867049936646804,
                                  0.56888888888888888889, 0.47862867049936646804,
                                  0.23692688505618908751};
};
template <>
struct GL<6> {
  static constexpr double x[6] = {-0.93246951420315202781, -0.66120938646626451366,
                                  -0.23861918608319690863, 0.23861918608319690863,
                                  0.66120938646626451366,  0.93246951420315202781};
  static constexpr double w[6] = {0.17132449237917034504, 0.36076157304813860757,
                                  0.46791393457269104739, 0.46791393457269104739,
                                  0.36076157304813860757, 0.17132449237917034504};
};
template <>
struct GL<7> {
  static constexpr double x[7] = {-0.94910791234275852453, -0.74153118559939443986, -0.40584515137739716691, 0.0,
                                  0.40584515137739716691,  0.74153118559939443986,  0.94910791234275852453};
  static constexpr double w[7] = {0.12948496616886969327, 0.27970539148927666790, 0.38183005050511894495,
                                  0.41795918367346938776, 0.38183005050511894495, 0.27970539148927666790,
                                  0.12948496616886969327};
};
template <>
struct GL<8> {
  static constexpr double x[8] = {-0.96028985649753623168, -0.79666647741362673959,
                                  -0.52553240991632898582, -0.18343464249564980494,
                                  0.18343464249564980494,  0.52553240991632898582,
                                  0.79666647741362673959,  0.96028985649753623168};
  static constexpr double w[8] = {0.10122853629037625915, 0.22238103445337447054,
                                  0.31370664587788728734, 0.36268378337836198297,
                                  0.36268378337836198297, 0.31370664587788728734,
                                  0.22238103445337447054, 0.10122853629037625915};
};
template <>
struct GL<10> {
  static constexpr double x[10] = {-0.97390652851717172008, -0.86506336668898451073, -0.67940956829902440623,
                                   -0.43339539412924719080, -0.14887433898163121088, 0.14887433898163121088,
                                   0.43339539412924719080,  0.67940956829902440623,  0.86506336668898451073,
                                   0.97390652851717172008};
  static constexpr double w[10] = {0.066671344308688137594, 0.14945134915058059315, 0.21908636251598204400,
                                   0.26926671930999635509,  0.29552422471475287017, 0.29552422471475287017,
                                   0.26926671930999635509,  0.21908636251598204400, 0.14945134915058059315,
                                   0.066671344308688137594};
};

// What the N-point rule misses on y^(2N) over [-1, 1],
// 2^(2N+1) (N!)^4 / ((2N+1) ((2N)!)^2): for a polynomial of degree <= 2N+1
// whose y^(2N) coefficient is c, the integral is the rule's sum plus e c (an
// odd top term integrates to zero under both).
template <int N>
struct GLRem;
template <>
struct GLRem<1> {
  static constexpr double e = 2.0 / 3.0;
};
template <>
struct GLRem<2> {
  static constexpr double e = 8.0 / 45.0;
};
template <>
struct GLRem<4> {
  static constexpr double e = 128.0 / 11025.0;
};
template <>
struct GLRem<7> {
  static constexpr double e = 512.0 / 2760615.0;
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
template <typename T>
CP_HD T tmin(T a, T b) {
  return b < a ? b : a;
}
template <typename T>
CP_HD T tmax(T a, T b) {
  return a < b ? b : a;
}
// minimum of two values known not to be NaN (one v_min instruction instead
// of a compare and a select)
CP_HD inline float fmin_nn(float a, float b) { return __builtin_fminf(a, b); }
CP_HD inline double fmin_nn(double a, double b) { return __builtin_fmin(a, b); }
template <typename T>
CP_HD T tclamp(T v, T lo, T hi) {
  return tmin(tmax(v, lo), hi);
}
template <typename T>
CP_HD T qnan() {
  return __builtin_nan("");
}

// Compare-exchange of key k with a payload of P values (and an int tag).
template <typename T, int P>
CP_HD void cswap(T& ka, T& kb, T (&pa)[P], T (&pb)[P], int& ta, int& tb) {
  const bool s = kb < ka;
  T t = s ? kb : ka;
  kb = s ? ka : kb;
  ka = t;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    T u = s ? pb[p] : pa[p];
    pb[p] = s ? pa[p] : pb[p];
    pa[p] = u;
  }
  int v = s ? tb : ta;
  tb = s ? ta : tb;
  ta = v;
}

// Sorting network for four keys (5 comparators), payload follows its key.
template <typename T, int P>
CP_HD void sort4(T (&k)[4], T (&p)[4][P], int (&tag)[4]) {
  cswap<T, P>(k[0], k[1], p[0], p[1], tag[0], tag[1]);
  cswap<T, P>(k[2], k[3], p[2], p[3], tag[2], tag[3]);
  cswap<T, P>(k[0], k[2], p[0], p[2], tag[0], tag[2]);
  cswap<T, P>(k[1], k[3], p[1], p[3], tag[1], tag[3]);
  cswap<T, P>(k[1], k[2], p[1], p[2], tag[1], tag[2]);
}

// The same network, recording whether each comparator swapped, so that
// values computed in sorted order can be taken back to neighbour order by
// unsort4 (the comparators in reverse order, each its own inverse): ten
// selects per array instead of a select per (slot, neighbour) pair.
template <typename T, int P>
CP_HD void cswap_rec(T& ka, T& kb, T (&pa)[P], T (&pb)[P], bool& s) {
  s = kb < ka;
  T t = s ? kb : ka;
  kb = s ? ka : kb;
  ka = t;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    T u = s ? pb[p] : pa[p];
    pb[p] = s ? pa[p] : pb[p];
    pa[p] = u;
  }
}

template <typename T, int P>
CP_HD void sort4_rec(T (&k)[4], T (&p)[4][P], bool (&sw)[5]) {
  cswap_rec<T, P>(k[0], k[1], p[0], p[1], sw[0]);
  cswap_rec<T, P>(k[2], k[3], p[2], p[3], sw[1]);
  cswap_rec<T, P>(k[0], k[2], p[0], p[2], sw[2]);
  cswap_rec<T, P>(k[1], k[3], p[1], p[3], sw[3]);
  cswap_rec<T, P>(k[1], k[2], p[1], p[2], sw[4]);
}

template <typename T>
CP_HD void uswap(T& a, T& b, bool s) {
  const T t = s ? b : a;
  b = s ? a : b;
  a = t;
}

template <typename T>
CP_HD void unsort4(T (&v)[4], const bool (&sw)[5]) {
  uswap(v[1], v[2], sw[4]);
  uswap(v[1], v[3], sw[3]);
  uswap(v[0], v[2], sw[2]);
  uswap(v[2], v[3], sw[1]);
  uswap(v[0], v[1], sw[0]);
}

// ===========================================================================
// Uniform model (Sec. 4.3).  Local frame with origin at the vertex lower
// end: vertex support [0, Lv]; neighbour i support [a_i, b_i].
//
// Task 1 (Sec. 4.1.1): b_min = min(Lv, b_i); nothing if b_min <= 0.  Start
// points clamped to [0, b_min] and sorted give the pieces
// [0,c0], [c0,c1], [c1,c2], [c2,c3], [c3,b_min]; on piece k exactly the k
// neighbours sorted first have started (Tasks 2-3, Template k+1), so every
// lane runs the same five pieces (empty ones contribute zero).
// On piece k the integrand (1/Lv) prod_{i<k} (b_i - x)/L_i has degree k:
// Gauss-Legendre with 1 and 2 nodes is exact for k = 1 and 3; k = 2 and 4
// take 1 and 2 nodes plus the rule's remainder on the top-degree term (its
// coefficient the product of the factors' slopes).
// ===========================================================================
template <typename T>
struct UniSide {
  T Lv, iLv;
  T c[4];      // sorted clamped start points
  T b[4];      // matching upper ends
  T iL[4];     // matching 1/(b - a)
  bool sw[5];  // comparator swaps of the sort (unsort4 restores neighbour order)
  T bmin;
  bool empty;
};

template <typename T>
CP_HD void uni_setup(UniSide<T>& s, T Lv, T iLv, const T (&a)[4], const T (&b)[4], const T (&iL)[4],
                     const bool (&pres)[4]) {
  s.Lv = Lv;
  s.iLv = iLv;
  T bmin = Lv;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (pres[i]) bmin = tmin(bmin, b[i]);
  s.bmin = bmin;
  s.empty = !(bmin > T(0));
  T key[4];
  T pay[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    // an absent neighbour is a factor that would start at b_min (never
    // active on a non-empty piece); finite stand-ins keep empty pieces finite
    key[i] = pres[i] ? tclamp(a[i], T(0), bmin) : bmin;
    pay[i][0] = pres[i] ? b[i] : T(3) * Lv;
    pay[i][1] = pres[i] ? iL[i] : iLv;
  }
  sort4_rec<T, 2>(key, pay, s.sw);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    s.c[i] = key[i];
    s.b[i] = pay[i][0];
    s.iL[i] = pay[i][1];
  }
}

// integral over [l, r] of prod_{i<K} (b_i - x) iL_i  (times nothing else);
// REM: K = 2N, and the y^K coefficient prod be_i gets the rule's remainder
template <typename T, int K, int N, bool REM = false>
CP_HD T uni_piece(const UniSide<T>& s, T l, T r) {
  static_assert(REM ? K == 2 * N : K <= 2 * N - 1, "rule too small for the piece");
  const T mid = (l + r) * T(0.5), hl = (r - l) * T(0.5);
  T al[K], be[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    al[i] = (s.b[i] - mid) * s.iL[i];
    be[i] = hl * s.iL[i];
  }
  T sum = T(0);
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const T x = T(GL<N>::x[j]);
    T prod = T(1);
#pragma unroll
    for (int i = 0; i < K; ++i) prod *= cfma(-be[i], x, al[i]);
    sum = cfma(T(GL<N>::w[j]), prod, sum);
  }
  if constexpr (REM) {
    T c = be[0];
#pragma unroll
    for (int i = 1; i < K; ++i) c *= be[i];
    sum = cfma(T(GLRem<N>::e), c, sum);  // (-be_i) for each of an even number of factors
  }
  return sum * hl;
}

template <typename T>
CP_HD T uni_side_value(const UniSide<T>& s) {
  if (s.empty) return T(0);
  T acc = s.c[0];  // piece 0: no factor
  acc += uni_piece<T, 1, 1>(s, s.c[0], s.c[1]);
  acc += uni_piece<T, 2, 1, true>(s, s.c[1], s.c[2]);
  acc += uni_piece<T, 3, 2>(s, s.c[2], s.c[3]);
  acc += uni_piece<T, 4, 2, true>(s, s.c[3], s.bmin);
  return acc * s.iLv;
}

// Local derivatives of one side:  f(Lv, a_i, b_i) = (1/Lv) int_0^{b_min} prod S_i
//   df/da_i = (1/L_i) int_{i active} p_v prod_k S_k
//   df/db_i = (1/L_i) int_{i active} p_v (prod_{k!=i} S_k - prod_k S_k)
//   df/dLv  = (-f + prod_i S_i(Lv)) / Lv
template <typename T>
struct UniGrad {
  T f, dLv;
  T da[4], db[4];  // by neighbour index 0..3
};

// REM: K = 2N; the leave-one-out sums (degree K - 1) are exact, the full
// product (degree K) gets the rule's remainder on prod be_i
template <typename T, int K, int N, bool REM = false>
CP_HD void uni_piece_grad(const UniSide<T>& s, T l, T r, T& full, T (&loo)[4]) {
  static_assert(REM ? K == 2 * N : K <= 2 * N - 1, "rule too small for the piece");
  const T mid = (l + r) * T(0.5), hl = (r - l) * T(0.5);
  T al[K], be[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    al[i] = (s.b[i] - mid) * s.iL[i];
    be[i] = hl * s.iL[i];
  }
  T sf = T(0), sl[K];
#pragma unroll
  for (int i = 0; i < K; ++i) sl[i] = T(0);
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const T x = T(GL<N>::x[j]);
    const T wj = T(GL<N>::w[j]);
    T f[K], pre[K + 1], suf[K + 1];
#pragma unroll
    for (int i = 0; i < K; ++i) f[i] = cfma(-be[i], x, al[i]);
    pre[0] = T(1);
#pragma unroll
    for (int i = 0; i < K; ++i) pre[i + 1] = pre[i] * f[i];
    suf[K] = T(1);
#pragma unroll
    for (int i = K - 1; i >= 0; --i) suf[i] = suf[i + 1] * f[i];
    sf = cfma(wj, pre[K], sf);
#pragma unroll
    for (int i = 0; i < K; ++i) sl[i] = cfma(wj, pre[i] * suf[i + 1], sl[i]);
  }
  if constexpr (REM) {
    T c = be[0];
#pragma unroll
    for (int i = 1; i < K; ++i) c *= be[i];
    sf = cfma(T(GLRem<N>::e), c, sf);
  }
  full = sf * hl;
#pragma unroll
  for (int i = 0; i < K; ++i) loo[i] += sl[i] * hl;
}

template <typename T>
CP_HD void uni_side_grad(const UniSide<T>& s, UniGrad<T>& g) {
  g.f = T(0);
  g.dLv = T(0);
#pragma unroll
  for (int i = 0; i < 4; ++i) g.da[i] = g.db[i] = T(0);
  if (s.empty) return;
  T I[5];
  T loo[4] = {T(0), T(0), T(0), T(0)};  // sorted slots; accumulated over pieces where active
  T act[4] = {T(0), T(0), T(0), T(0)};  // full integral over pieces where slot is active
  I[0] = s.c[0];
  uni_piece_grad<T, 1, 1>(s, s.c[0], s.c[1], I[1], loo);
  uni_piece_grad<T, 2, 1, true>(s, s.c[1], s.c[2], I[2], loo);
  uni_piece_grad<T, 3, 2>(s, s.c[2], s.c[3], I[3], loo);
  uni_piece_grad<T, 4, 2, true>(s, s.c[3], s.bmin, I[4], loo);
  // slot i is active on pieces i+1..4
  act[3] = I[4];
  act[2] = act[3] + I[3];
  act[1] = act[2] + I[2];
  act[0] = act[1] + I[1];
  const T iLv = s.iLv;
  const T f = (act[0] + I[0]) * iLv;
  g.f = f;
  // product of the survival factors at x = Lv (zero unless b_min = Lv)
  T gend = T(0);
  if (!(s.bmin < s.Lv)) {
    gend = T(1);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      // a factor that has not started at Lv is 1 (also an absent neighbour)
      T v = tmin(T(1), (s.b[i] - s.Lv) * s.iL[i]);
      gend *= (s.c[i] < s.Lv) ? tmax(v, T(0)) : T(1);
    }
  }
  g.dLv = (gend - f) * iLv;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    g.da[i] = act[i] * iLv * s.iL[i];
    g.db[i] = (loo[i] - act[i]) * iLv * s.iL[i];
  }
  // sorted slots -> neighbour index
  unsort4(g.da, s.sw);
  unsort4(g.db, s.sw);
}

// ===========================================================================
// Epanechnikov model (Sec. 4.3).  Local frame with origin at the vertex
// centre: vertex support [-wv, wv], neighbour i centre d_i, half-width w_i.
// pdf_v = 3/(4 wv) (1 - t^2), S_i = (1 - u)^2 (2 + u) / 4 with t = x/wv,
// u = (x - d_i)/w_i.  Piece k (k neighbours started) has degree 2 + 3k
// (the paper's order-15 remark, Sec. 4.3): Gauss-Legendre with 3 and 6
// nodes is exact for k = 1 and 3; k = 2 and 4 (degree 8 and 14) take 4 and 7
// nodes plus the rule's remainder on the top-degree term, whose coefficient
// is a product of the factors' leading coefficients; piece 0 is the vertex
// CDF in closed form.
// ===========================================================================
template <typename T>
struct EpaSide {
  T wv, iwv;
  T c[4], d[4], iw[4];
  bool sw[5];  // comparator swaps of the sort (unsort4 restores neighbour order)
  T bmin;
  bool empty;
};

template <typename T>
CP_HD void epa_setup(EpaSide<T>& s, T wv, T iwv, const T (&d)[4], const T (&w)[4], const T (&iw)[4],
                     const bool (&pres)[4]) {
  s.wv = wv;
  s.iwv = iwv;
  T bmin = wv;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (pres[i]) bmin = tmin(bmin, d[i] + w[i]);
  s.bmin = bmin;
  s.empty = !(bmin > -wv);
  constexpr int P = 2;
  T key[4];
  T pay[4][P];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    key[i] = pres[i] ? tclamp(d[i] - w[i], -wv, bmin) : bmin;
    pay[i][0] = pres[i] ? d[i] : T(3) * wv;
    pay[i][1] = pres[i] ? iw[i] : s.iwv;
  }
  sort4_rec<T, P>(key, pay, s.sw);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    s.c[i] = key[i];
    s.d[i] = pay[i][0];
    s.iw[i] = pay[i][1];
  }
}

// 4 * vertex CDF at x: (1 + t)^2 (2 - t), t = x / wv
template <typename T>
CP_HD T epa_cdf4(const EpaSide<T>& s, T x) {
  const T t = x * s.iwv;
  const T o = T(1) + t;
  return o * o * (T(2) - t);
}

// 4 S(u) = u^3 - 3u + 2 in Horner form: three fused multiply-adds.  On a
// piece where the factor has started, u is in [-1, 1] and the rounding error
// is at most a few ulp of 3 in absolute terms.
template <typename T>
CP_HD T epa_s4(T u) {
  return cfma(cfma(u, u, T(-3)), u, T(2));
}

// integral over [l, r] of (1 - t^2) prod_{i<K} 4 S_i   (unscaled): the
// N-point rule, plus (REM) its remainder when the integrand's degree 2 + 3K
// is 2N: the y^(2N) coefficient is -bv^2 prod bu_i^3
template <typename T, int K, int N, bool REM = false>
CP_HD T epa_piece(const EpaSide<T>& s, T l, T r) {
  static_assert(REM ? 2 + 3 * K == 2 * N : 2 + 3 * K <= 2 * N - 1, "rule too small for the piece");
  const T mid = (l + r) * T(0.5), hl = (r - l) * T(0.5);
  const T av = mid * s.iwv, bv = hl * s.iwv;
  T au[K], bu[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    au[i] = (mid - s.d[i]) * s.iw[i];  // u = au + bu x
    bu[i] = hl * s.iw[i];
  }
  T sum = T(0);
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const T x = T(GL<N>::x[j]);
    const T t = cfma(bv, x, av);
    T prod = cfma(-t, t, T(1));
#pragma unroll
    for (int i = 0; i < K; ++i) prod *= epa_s4(cfma(bu[i], x, au[i]));
    sum = cfma(T(GL<N>::w[j]), prod, sum);
  }
  if constexpr (REM) {
    T c = bv * bv;
#pragma unroll
    for (int i = 0; i < K; ++i) c *= bu[i] * bu[i] * bu[i];
    sum = cfma(T(-GLRem<N>::e), c, sum);
  }
  return sum * hl;
}

template <typename T>
CP_HD T epa_side_value(const EpaSide<T>& s) {
  if (s.empty) return T(0);
  const T kv = T(0.75) * s.iwv;  // pdf scale 3/(4 wv)
  T acc = epa_cdf4(s, s.c[0]) * T(0.25);
  T p = epa_piece<T, 1, 3>(s, s.c[0], s.c[1]) * T(0.25);
  p += epa_piece<T, 2, 4, true>(s, s.c[1], s.c[2]) * T(0.0625);
  p += epa_piece<T, 3, 6>(s, s.c[2], s.c[3]) * T(0.015625);
  p += epa_piece<T, 4, 7, true>(s, s.c[3], s.bmin) * T(0.00390625);
  return acc + kv * p;
}

// Local derivatives of one side, f(wv, d_i, w_i):
//   df/dd_i = int p_v p_i prod_{k!=i} S_k          (dS/dm = pdf)
//   df/dw_i = int p_v u_i p_i prod_{k!=i} S_k      (dS/dw = u pdf)
// and df/dwv = -(1/wv) sum_i (d_i df/dd_i + w_i df/dw_i), the scale
// invariance of P about the vertex centre (wv df/dwv + sum_i (d_i df/dd_i +
// w_i df/dw_i) = 0), which the caller forms in neighbour order (absent
// neighbours have zero derivatives): it equals -(1/wv) sum_i int x p_v p_i
// prod_{k!=i} S_k, since x = d_i + w_i u_i, and avoids integrating
// dpdf_v/dwv, whose integral over the support is 0 and cancels.  WF: also
// return f itself (the fused forward).
template <typename T>
struct EpaGrad {
  T f;
  T dd[4], dw[4];  // by neighbour index
};

// One piece with K started neighbours (sorted slots 0..K-1), N nodes.  The
// slot sums, times the piece's factor sc = 4^-(K-1) and its half-length, are
// added straight into the side's accumulators ad / aw (by sorted slot); WF:
// the piece's value, times fsc = 4^-K and the half-length, into `full`.
// The position sums have degree 3K + 1, the width sums and the value 3K + 2;
// REM: N = (3K + 2) / 2 nodes and the rule's remainder, from the y^(2N)
// coefficient, which is bv^2 prod_k bu_k^3 for every width sum (the leading
// coefficients -bv^2, -bu_i^2 and bu_i of its own factors, bu_k^3 of the
// others) and its negative for the value.
template <typename T, int K, int N, bool REM, bool WF>
CP_HD void epa_piece_grad(const EpaSide<T>& s, T l, T r, T sc, T fsc, T& full, T (&ad)[4], T (&aw)[4]) {
  static_assert(REM ? 3 * K + 2 == 2 * N : 3 * K + 2 <= 2 * N - 1, "rule too small for the piece");
  const T mid = (l + r) * T(0.5), hl = (r - l) * T(0.5);
  const T av = mid * s.iwv, bv = hl * s.iwv;
  T au[K], bu[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    au[i] = (mid - s.d[i]) * s.iw[i];  // u = au + bu x
    bu[i] = hl * s.iw[i];
  }
  T sf = T(0), sd[K], sww[K];
#pragma unroll
  for (int i = 0; i < K; ++i) sd[i] = sww[i] = T(0);
#pragma unroll
  for (int j = 0; j < N; ++j) {
    const T x = T(GL<N>::x[j]);
    const T t = cfma(bv, x, av);
    T u[K], S[K], pre[K + 1], suf[K + 1];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      u[i] = cfma(bu[i], x, au[i]);
      S[i] = epa_s4(u[i]);  // 4 S_i
    }
    // prefix products carry the node weight and the vertex pdf
    // (weight * 4 wv/3 * pdf_v = w_j (1 - t^2))
    pre[0] = T(GL<N>::w[j]) * cfma(-t, t, T(1));
#pragma unroll
    for (int i = 0; i < K; ++i) pre[i + 1] = pre[i] * S[i];
    suf[K] = T(1);
#pragma unroll
    for (int i = K - 1; i >= 0; --i) suf[i] = suf[i + 1] * S[i];
    if (WF) sf += pre[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
      // (4 w_i / 3) p_i = 1 - u^2
      const T lw = cfma(-u[i], u[i], T(1)) * (pre[i] * suf[i + 1]);
      sd[i] += lw;
      sww[i] = cfma(lw, u[i], sww[i]);
    }
  }
  if constexpr (REM) {
    T c = bv * bv;
#pragma unroll
    for (int i = 0; i < K; ++i) c *= bu[i] * bu[i] * bu[i];
    const T ec = T(GLRem<N>::e) * c;
    if (WF) sf -= ec;
#pragma unroll
    for (int i = 0; i < K; ++i) sww[i] += ec;
  }
  const T ps = sc * hl;
  if (WF) full = cfma(sf, fsc * hl, full);
#pragma unroll
  for (int i = 0; i < K; ++i) {
    ad[i] = cfma(sd[i], ps, ad[i]);
    aw[i] = cfma(sww[i], ps, aw[i]);
  }
}

template <typename T, bool WF = true>
CP_HD void epa_side_grad(const EpaSide<T>& s, EpaGrad<T>& g) {
  g.f = T(0);
#pragma unroll
  for (int i = 0; i < 4; ++i) g.dd[i] = g.dw[i] = T(0);
  if (s.empty) return;
  // neighbour slot i collects the pieces k > i, its factor p_i carrying
  // 3/(4 w_i) and the other started factors 4^-(k-1); the value of piece k
  // carries 4^-k
  T ad[4] = {T(0), T(0), T(0), T(0)}, aw[4] = {T(0), T(0), T(0), T(0)};
  T full = T(0);
  epa_piece_grad<T, 1, 3, false, WF>(s, s.c[0], s.c[1], T(1), T(0.25), full, ad, aw);
  epa_piece_grad<T, 2, 4, true, WF>(s, s.c[1], s.c[2], T(0.25), T(0.0625), full, ad, aw);
  epa_piece_grad<T, 3, 6, false, WF>(s, s.c[2], s.c[3], T(0.0625), T(0.015625), full, ad, aw);
  epa_piece_grad<T, 4, 7, true, WF>(s, s.c[3], s.bmin, T(0.015625), T(0.00390625), full, ad, aw);
  const T kv = T(0.75) * s.iwv;
  if (WF) g.f = cfma(kv, full, epa_cdf4(s, s.c[0]) * T(0.25));
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const T ki = T(0.75) * s.iw[i] * kv;
    g.dd[i] = ki * ad[i];
    g.dw[i] = ki * aw[i];
  }
  // sorted slots -> neighbour index
  unsort4(g.dd, s.sw);
  unsort4(g.dw, s.sw);
}

}  // namespace cp
