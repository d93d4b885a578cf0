// host_checks.cpp -- host-only build of the library's per-vertex routines and
// adjoint-buffer bookkeeping, for a CPU run under AddressSanitizer and
// UndefinedBehaviorSanitizer (test infrastructure; built by
// tests/test_host_sanitized.py with the HIP compiler's host pass only).
//
//   host_checks field <in> <out>
//     in:  int32 model, dtype (0 FP32, 1 FP64), H, W, nbins; then FP64
//          params [n_param][H][W], g_min [H][W], g_max [H][W]
//     out: FP64 p_min [H][W], p_max [H][W], grad [n_param][H][W]
//   The field is evaluated vertex by vertex with the same per-vertex
//   routines the kernels call (vertex_fwd_ue, vertex_jac_vals,
//   hist_vertex_minmax, hist_stencil_jac), from a zero-padded copy laid out
//   like a staged tile, and the adjoint is gathered as the kernels gather it.
//   host_checks pool
//     exercises the workspace bookkeeping with a counting allocator.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "cp_hist_bwd.hpp"
#include "cp_internal.hpp"
#include "cp_tiles.hpp"
#include "cp_workspace.hpp"

namespace {

template <typename T>
struct Grid {
  int H, W, nb, np;
  int PX, PY, E;  // padded grid: (H + 2) x (W + 2), plane size E
  std::vector<T> par;  // [np][E], zero halo
  int at(int y, int x) const { return (y + 1) * PX + (x + 1); }
};

template <typename T>
Grid<T> padded(const std::vector<double>& p, int np, int H, int W, int nb) {
  Grid<T> g{H, W, nb, np, W + 2, H + 2, (H + 2) * (W + 2), {}};
  g.par.assign((size_t)np * g.E, T(0));
  for (int k = 0; k < np; ++k)
    for (int y = 0; y < H; ++y)
      for (int x = 0; x < W; ++x) g.par[(size_t)k * g.E + g.at(y, x)] = (T)p[((size_t)k * H + y) * W + x];
  return g;
}

template <typename T, int MODEL>
void run_ue(const std::vector<double>& p, const std::vector<double>& gmin, const std::vector<double>& gmax, int H,
            int W, std::vector<double>& out) {
  Grid<T> g = padded<T>(p, 2, H, W, 0);
  const size_t nv = (size_t)H * W;
  std::vector<T> jac((size_t)10 * nv);
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      const int e = g.at(y, x);
      const int en[4] = {e + 1, e - g.PX, e - 1, e + g.PX};
      const bool pres[4] = {x + 1 < W, y > 0, x > 0, y + 1 < H};
      T pmin, pmax;
      cp::vertex_fwd_ue<T, MODEL>(g.par.data(), g.E, e, en, pres, pmin, pmax);
      const size_t v = (size_t)y * W + x;
      out[v] = (double)pmin;
      out[nv + v] = (double)pmax;
      T q0[4], q1[4];
      for (int i = 0; i < 4; ++i) {
        q0[i] = pres[i] ? g.par[en[i]] : T(0);
        q1[i] = pres[i] ? g.par[g.E + en[i]] : T(1);
      }
      T j[10], a, b;
      cp::vertex_jac_vals<T, MODEL, true>(g.par[e], g.par[g.E + e], q0, q1, pres, (T)gmin[v], (T)gmax[v], j, a, b);
      for (int k = 0; k < 10; ++k) jac[(size_t)k * nv + v] = j[k];
    }
  // gather: own slot + e slot of the west neighbour, w of the east, s of the
  // north, n of the south (slots v, e, n, w, s at jac planes 0, 2, 4, 6, 8)
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x)
      for (int q = 0; q < 2; ++q) {
        const size_t v = (size_t)y * W + x;
        T s = jac[(size_t)q * nv + v];
        if (x + 1 < W) s += jac[(size_t)(6 + q) * nv + v + 1];
        if (x > 0) s += jac[(size_t)(2 + q) * nv + v - 1];
        if (y > 0) s += jac[(size_t)(8 + q) * nv + v - W];
        if (y + 1 < H) s += jac[(size_t)(4 + q) * nv + v + W];
        out[(2 + q) * nv + v] = (double)s;
      }
}

template <typename T>
void run_hist(const std::vector<double>& p, const std::vector<double>& gmin, const std::vector<double>& gmax, int H,
              int W, int h, std::vector<double>& out) {
  Grid<T> g = padded<T>(p, 2 + h, H, W, h);
  g.par.resize((size_t)(3 + h) * g.E, T(0));  // zero plane after the suffix sums (U_h)
  cp::hist_stage_validity<T, 1>(g.par.data(), g.E, h, 0);
  std::vector<T> raw = g.par;  // validity-marked masses (for the Jacobian routine)
  cp::hist_stage_suffix<T, 1>(g.par.data(), g.E, h, 0);
  const size_t nv = (size_t)H * W;
  std::vector<T> J((size_t)cp::hist_ws_planes(h) * nv, T(0));
  const cp::HistLds<T> L{g.par.data(), g.E, h, T(1) / T(h)};
  const cp::HistSuf<T> U{g.par.data(), g.E, h};
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      const int e = g.at(y, x);
      const int en[4] = {e + 1, e - g.PX, e - 1, e + g.PX};
      const bool pres[4] = {x + 1 < W, y > 0, x > 0, y + 1 < H};
      const size_t v = (size_t)y * W + x;
      bool ok = L.valid(e);
      for (int i = 0; i < 4; ++i) ok = ok && (!pres[i] || L.valid(en[i]));
      T pmin = cp::qnan<T>(), pmax = cp::qnan<T>();
      if (ok) {
        const T lov = g.par[e], hiv = g.par[g.E + e];
        T lo[4], hi[4];
        for (int i = 0; i < 4; ++i) {
          lo[i] = g.par[en[i]] - lov;
          hi[i] = g.par[g.E + en[i]] - lov;
        }
        cp::hist_vertex_minmax(U, e, en, pres, hiv - lov, lo, hi, pmin, pmax);
      }
      out[v] = (double)pmin;
      out[nv + v] = (double)pmax;
      T a, b;
      cp::JPlanes<T> jp{J.data(), (uint32_t)nv, (int64_t)v, h};
      cp::hist_stencil_jac(L, U, g.par.data(), g.E, g.PX, e, y, x, H, W, (T)gmin[v], (T)gmax[v], jp, a, b);
    }
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      const size_t v = (size_t)y * W + x;
      out[2 * nv + v] = 0.0;
      out[3 * nv + v] = 0.0;
      // the tails of the four neighbours' stencils (u is the west neighbour
      // of its east neighbour, and so on) apply to every bin
      const auto tl = [&](int i, size_t w) { return J[(size_t)(5 * h + i) * nv + w]; };
      for (int k = 0; k < h; ++k) {
        T s = J[(size_t)(0 * h + k) * nv + v];
        if (x + 1 < W) s += J[(size_t)(3 * h + k) * nv + v + 1] + tl(2, v + 1);
        if (x > 0) s += J[(size_t)(1 * h + k) * nv + v - 1] + tl(0, v - 1);
        if (y > 0) s += J[(size_t)(4 * h + k) * nv + v - W] + tl(3, v - W);
        if (y + 1 < H) s += J[(size_t)(2 * h + k) * nv + v + W] + tl(1, v + W);
        out[(size_t)(4 + k) * nv + v] = (double)s;
      }
    }
}

int field(const char* in, const char* outp) {
  FILE* f = std::fopen(in, "rb");
  if (!f) return 2;
  int32_t hdr[5];
  if (std::fread(hdr, sizeof(hdr), 1, f) != 1) return 2;
  const int model = hdr[0], dt = hdr[1], H = hdr[2], W = hdr[3], nb = hdr[4];
  const int np = model == CP_HISTOGRAM ? 2 + nb : 2;
  const size_t nv = (size_t)H * W;
  std::vector<double> p((size_t)np * nv), gmin(nv), gmax(nv);
  if (std::fread(p.data(), sizeof(double), p.size(), f) != p.size()) return 2;
  if (std::fread(gmin.data(), sizeof(double), nv, f) != nv) return 2;
  if (std::fread(gmax.data(), sizeof(double), nv, f) != nv) return 2;
  std::fclose(f);
  std::vector<double> out((size_t)(2 + np) * nv);
  if (model == CP_UNIFORM)
    dt ? run_ue<double, CP_UNIFORM>(p, gmin, gmax, H, W, out) : run_ue<float, CP_UNIFORM>(p, gmin, gmax, H, W, out);
  else if (model == CP_EPANECHNIKOV)
    dt ? run_ue<double, CP_EPANECHNIKOV>(p, gmin, gmax, H, W, out)
       : run_ue<float, CP_EPANECHNIKOV>(p, gmin, gmax, H, W, out);
  else if (model == CP_HISTOGRAM)
    dt ? run_hist<double>(p, gmin, gmax, H, W, nb, out) : run_hist<float>(p, gmin, gmax, H, W, nb, out);
  else
    return 3;
  FILE* o = std::fopen(outp, "wb");
  if (!o) return 2;
  std::fwrite(out.data(), sizeof(double), out.size(), o);
  std::fclose(o);
  return 0;
}

// ---------------------------------------------------------------------------
// workspace bookkeeping with a counting allocator
// ---------------------------------------------------------------------------
int g_allocs = 0, g_frees = 0;
int count_alloc(void** out, size_t bytes) {
  *out = std::malloc(bytes);
  ++g_allocs;
  return *out ? 0 : 1;
}
void count_free(int, void* p) {
  std::free(p);
  ++g_frees;
}

#define EXPECT(c)                                                   \
  do {                                                              \
    if (!(c)) {                                                     \
      std::fprintf(stderr, "pool check failed: %s (line %d)\n", #c, __LINE__); \
      return 1;                                                     \
    }                                                               \
  } while (0)

int pool() {
  const cp::PoolOps ops{count_alloc, count_free};
  cp::WorkspacePool w;
  int s1 = 0, s2 = 0;  // two stream handles
  void *a = nullptr, *b = nullptr, *c = nullptr, *d = nullptr;
  EXPECT(w.get(0, &s1, 1000, ops, &a) == 0 && a);
  std::memset(a, 1, 1000);
  EXPECT(w.get(0, &s1, 500, ops, &b) == 0 && b == a);  // smaller: reused
  EXPECT(w.get(0, &s2, 500, ops, &c) == 0 && c != a);  // other stream: its own
  EXPECT(w.get(1, &s1, 500, ops, &d) == 0 && d != a && d != c);  // other device
  EXPECT(g_allocs == 3 && g_frees == 0);
  void* e = nullptr;
  EXPECT(w.get(0, &s1, 4000, ops, &e) == 0 && e != a);  // grown: a is retired, not freed
  std::memset(a, 2, 1000);  // still valid memory (a captured graph may write it)
  std::memset(e, 3, 4000);
  EXPECT(g_allocs == 4 && g_frees == 0 && w.held() == 4);
  void* f = nullptr;
  EXPECT(w.get(0, &s1, 4000, ops, &f) == 0 && f == e);
  w.release(ops);
  EXPECT(g_frees == 4 && w.held() == 0);
  EXPECT(w.get(0, &s1, 10, ops, &a) == 0 && g_allocs == 5);  // usable after release
  w.release(ops);
  EXPECT(g_frees == 5);
  std::printf("pool ok\n");
  return 0;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc == 4 && !std::strcmp(argv[1], "field")) return field(argv[2], argv[3]);
  if (argc == 2 && !std::strcmp(argv[1], "pool")) return pool();
  std::fprintf(stderr, "usage: host_checks field <in> <out> | pool\n");
  return 2;
}
