// cp_batched.hip -- many fields of uneven size and mixed closed-form models
// in one persistent launch per pass.
//
// Small fields under-fill 256 CUs when launched one by one (a 128^2 field is
// 64 forward tiles); the batched form flattens every field into tiles, deals
// the tiles to a grid of resident blocks by a longest-processing-time rule
// over a per-vertex cost model, and lets each block walk its own list.  The
// tile lists depend only on the shapes, so they are built and uploaded once
// per shape signature; the field table (data pointers) is refreshed only when
// a pointer changes.  With CP_BATCH_GRAPH the launches are captured once per
// signature into a HIP graph and replayed.
//
// Forward-only and adjoint plans use separate kernel instantiations (each
// carries only the register budget of its own tile routines).  Histogram
// adjoint tiles write their per-stencil Jacobians to a workspace owned by the
// plan, and a second persistent launch gathers them; forward values are
// written by the adjoint tiles when both are requested.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <queue>
#include <vector>

#include "cp_hist_bwd.hpp"
#include "cp_internal.hpp"
#include "cp_tiles.hpp"

namespace cp {

namespace {

constexpr int kNT = 256;
constexpr int kBwdF32 = 30, kBwdF64 = 14;  // uniform / Epanechnikov adjoint tile edges
constexpr int kGatherChunk = 256;          // histogram gather: vertices per tile
constexpr size_t kMaxLds = 160 * 1024;

enum { KIND_FWD = 0, KIND_BWD = 1, KIND_GATHER = 2 };
enum { PASS_FWD = 0, PASS_BWD = 1, PASS_GATHER = 2 };

struct BatchTile {
  int field, ty0, tx0, kind;  // gather tiles: ty0 = first flat vertex index
};

template <typename T>
struct BatchField {
  FieldPtrs<T> p;
  T* J;  // histogram adjoint workspace ([5][h][H][W]) or null
  int model;
};

// histogram gather over vertices [i0, i0 + n) of one field (flat y*W + x)
template <typename T>
__device__ __forceinline__ void hist_gather_chunk(const FieldPtrs<T>& f, const T* __restrict__ J, int64_t i0,
                                                  int tid) {
  const int64_t plane = (int64_t)f.H * f.W;
  const int64_t id = i0 + tid;
  if (id >= plane) return;
  const int y = (int)(id / f.W), x = (int)(id - (int64_t)y * f.W);
  const int h = f.nb;
  const int64_t at = (int64_t)y * f.rs + x;
  f.grad[at] = T(0);
  f.grad[f.ps + at] = T(0);
  for (int k = 0; k < h; ++k) {
    T g = J[(int64_t)(0 * h + k) * plane + id];
    if (x + 1 < f.W) g += J[(int64_t)(3 * h + k) * plane + id + 1];
    if (x > 0) g += J[(int64_t)(1 * h + k) * plane + id - 1];
    if (y > 0) g += J[(int64_t)(4 * h + k) * plane + id - f.W];
    if (y + 1 < f.H) g += J[(int64_t)(2 * h + k) * plane + id + f.W];
    f.grad[(int64_t)(2 + k) * f.ps + at] = g;
  }
}

template <typename T, int PASS>
__global__ __launch_bounds__(kNT) void k_batched(const BatchField<T>* __restrict__ fields,
                                                 const BatchTile* __restrict__ tiles, const int* __restrict__ start) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* lds = reinterpret_cast<T*>(smem);
  const int tid = threadIdx.x;
  const int b = blockIdx.x;
  const int t1 = start[b + 1];
  for (int t = start[b]; t < t1; ++t) {
    const BatchTile tl = tiles[t];
    const BatchField<T> F = fields[tl.field];
    if (PASS == PASS_FWD) {
      if (F.model == CP_UNIFORM)
        tile_fwd_ue<T, CP_UNIFORM, 4>(F.p, tl.ty0, tl.tx0, lds, tid);
      else if (F.model == CP_EPANECHNIKOV)
        tile_fwd_ue<T, CP_EPANECHNIKOV, 4>(F.p, tl.ty0, tl.tx0, lds, tid);
      else
        tile_fwd_hist<T, 4>(F.p, tl.ty0, tl.tx0, lds, tid);
    } else if (PASS == PASS_BWD) {
      constexpr int OB = sizeof(T) == 4 ? kBwdF32 : kBwdF64;
      if (F.model == CP_UNIFORM)
        tile_bwd_ue<T, CP_UNIFORM, OB, OB, kNT>(F.p, tl.ty0, tl.tx0, lds, tid);
      else if (F.model == CP_EPANECHNIKOV)
        tile_bwd_ue<T, CP_EPANECHNIKOV, OB, OB, kNT>(F.p, tl.ty0, tl.tx0, lds, tid);
      else
        tile_hist_sweep<T, 4>(F.p, tl.ty0, tl.tx0, lds, tid, F.J);
    } else {
      hist_gather_chunk<T>(F.p, F.J, tl.ty0, tid);
    }
  }
}

// Relative cost per vertex (forward, adjoint), measured on MI355X with the
// per-field kernels at 2048^2 (uniform forward = 1); histograms scale with
// the number of bin edges.
double vertex_cost(int model, int nb, bool bwd) {
  if (model == CP_UNIFORM) return bwd ? 2.0 : 1.0;
  if (model == CP_EPANECHNIKOV) return bwd ? 4.3 : 1.9;
  return (bwd ? 5.6 : 2.3) * (nb + 1);
}

size_t tile_lds_bytes(int model, int nb, bool bwd, size_t el) {
  if (model == CP_HISTOGRAM) return el * (size_t)hist_planes(nb) * (kFwdTX + 2) * 6;
  if (!bwd) return el * 2 * (kFwdTX + 2) * 6;
  if (el == 4) return el * bwd_ue_lds_elems<kBwdF32, kBwdF32>();
  return el * bwd_ue_lds_elems<kBwdF64, kBwdF64>();
}

struct Pass {
  int grid = 0;
  size_t lds = 0;
  int* d_start = nullptr;
  BatchTile* d_tiles = nullptr;
};

struct Plan {
  int dtype = 0;
  bool bwd = false;
  Pass main, gather;  // gather.grid == 0: no histogram adjoint
  void* d_fields = nullptr;
  void* d_ws = nullptr;             // histogram Jacobians of all fields
  std::vector<size_t> ws_offset;    // bytes, per field (SIZE_MAX: none)
  std::vector<unsigned char> host_fields;  // last uploaded field table
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  ~Plan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (Pass* p : {&main, &gather}) {
      if (p->d_start) (void)hipFree(p->d_start);
      if (p->d_tiles) (void)hipFree(p->d_tiles);
    }
    if (d_fields) (void)hipFree(d_fields);
    if (d_ws) (void)hipFree(d_ws);
  }
};

std::mutex g_mu;
std::map<std::vector<int64_t>, std::unique_ptr<Plan>> g_plans;
int g_num_cu = 0;

template <typename T, int PASS>
hipError_t prepare_kernel(size_t lds, int* per_cu) {
  const void* k = reinterpret_cast<const void*>(k_batched<T, PASS>);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k, kNT, lds);
}

hipError_t prepare(int dtype, int pass, size_t lds, int* per_cu) {
  if (dtype == CP_F64) {
    if (pass == PASS_FWD) return prepare_kernel<double, PASS_FWD>(lds, per_cu);
    if (pass == PASS_BWD) return prepare_kernel<double, PASS_BWD>(lds, per_cu);
    return prepare_kernel<double, PASS_GATHER>(lds, per_cu);
  }
  if (pass == PASS_FWD) return prepare_kernel<float, PASS_FWD>(lds, per_cu);
  if (pass == PASS_BWD) return prepare_kernel<float, PASS_BWD>(lds, per_cu);
  return prepare_kernel<float, PASS_GATHER>(lds, per_cu);
}

// Deal tiles to resident blocks (longest processing time first) and upload.
cp_status_t build_pass(const std::vector<BatchTile>& tiles, const std::vector<double>& cost, int dtype, int pass,
                       size_t lds, Pass& P) {
  int per_cu = 0;
  if (prepare(dtype, pass, lds, &per_cu) != hipSuccess) return CP_EDEVICE;
  per_cu = std::max(per_cu, 1);
  const int grid = std::max(1, std::min<int>((int)tiles.size(), g_num_cu * per_cu));
  std::vector<int> order(tiles.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  using Item = std::pair<double, int>;
  std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
  for (int b = 0; b < grid; ++b) heap.push({0.0, b});
  std::vector<std::vector<int>> lists(grid);
  for (int t : order) {
    Item it = heap.top();
    heap.pop();
    lists[it.second].push_back(t);
    heap.push({it.first + cost[t], it.second});
  }
  std::vector<int> start(grid + 1, 0);
  std::vector<BatchTile> flat;
  flat.reserve(tiles.size());
  for (int b = 0; b < grid; ++b) {
    start[b] = (int)flat.size();
    std::sort(lists[b].begin(), lists[b].end());  // field / row order within a block
    for (int t : lists[b]) flat.push_back(tiles[t]);
  }
  start[grid] = (int)flat.size();
  P.grid = grid;
  P.lds = lds;
  if (hipMalloc(&P.d_start, sizeof(int) * start.size()) != hipSuccess) return CP_ENOMEM;
  if (hipMalloc(&P.d_tiles, sizeof(BatchTile) * std::max<size_t>(flat.size(), 1)) != hipSuccess) return CP_ENOMEM;
  if (hipMemcpy(P.d_start, start.data(), sizeof(int) * start.size(), hipMemcpyHostToDevice) != hipSuccess)
    return CP_EDEVICE;
  if (!flat.empty() &&
      hipMemcpy(P.d_tiles, flat.data(), sizeof(BatchTile) * flat.size(), hipMemcpyHostToDevice) != hipSuccess)
    return CP_EDEVICE;
  return CP_OK;
}

cp_status_t build_plan(int n, const Field* fs, bool bwd, Plan& P, const char** why) {
  const size_t el = fs[0].dtype == CP_F64 ? 8 : 4;
  P.dtype = fs[0].dtype;
  P.bwd = bwd;
  if (g_num_cu == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return CP_EDEVICE;
    if (hipDeviceGetAttribute(&g_num_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return CP_EDEVICE;
  }
  std::vector<BatchTile> tiles, gtiles;
  std::vector<double> cost, gcost;
  size_t lds = 0, ws = 0;
  P.ws_offset.assign(n, SIZE_MAX);
  for (int i = 0; i < n; ++i) {
    const Field& f = fs[i];
    int ox = kFwdTX, oy = 4;
    if (bwd && f.model != CP_HISTOGRAM) ox = oy = el == 4 ? kBwdF32 : kBwdF64;
    lds = std::max(lds, tile_lds_bytes(f.model, f.nb, bwd, el));
    const double c = vertex_cost(f.model, f.nb, bwd) * ox * oy;
    for (int ty = 0; ty < f.H; ty += oy)
      for (int tx = 0; tx < f.W; tx += ox) {
        tiles.push_back(BatchTile{i, ty, tx, bwd ? KIND_BWD : KIND_FWD});
        cost.push_back(c);
      }
    if (bwd && f.model == CP_HISTOGRAM) {
      const int64_t plane = (int64_t)f.H * f.W;
      P.ws_offset[i] = ws;
      ws += el * (size_t)5 * f.nb * plane;
      ws = (ws + 255) / 256 * 256;
      for (int64_t v = 0; v < plane; v += kGatherChunk) {
        gtiles.push_back(BatchTile{i, (int)v, 0, KIND_GATHER});
        gcost.push_back(1.0);
      }
    }
  }
  if (lds > kMaxLds) {
    *why = "batched: staged planes exceed the LDS of a workgroup (too many bins for this dtype)";
    return CP_EUNSUPPORTED;
  }
  cp_status_t s = build_pass(tiles, cost, P.dtype, bwd ? PASS_BWD : PASS_FWD, lds, P.main);
  if (s != CP_OK) return s;
  if (!gtiles.empty()) {
    s = build_pass(gtiles, gcost, P.dtype, PASS_GATHER, 0, P.gather);
    if (s != CP_OK) return s;
    if (hipMalloc(&P.d_ws, ws) != hipSuccess) return CP_ENOMEM;
  }
  P.host_fields.clear();
  const size_t fb = (el == 4 ? sizeof(BatchField<float>) : sizeof(BatchField<double>)) * (size_t)n;
  if (hipMalloc(&P.d_fields, fb) != hipSuccess) return CP_ENOMEM;
  return CP_OK;
}

template <typename T>
void fill_fields(int n, const Field* fs, const Plan& P, const void* const* params, void* const* pmin,
                 void* const* pmax, const void* const* gmin, const void* const* gmax, void* const* grad, bool fwd,
                 bool bwd, std::vector<unsigned char>& out) {
  out.assign(sizeof(BatchField<T>) * (size_t)n, 0);
  BatchField<T>* bf = reinterpret_cast<BatchField<T>*>(out.data());
  for (int i = 0; i < n; ++i) {
    const Field& f = fs[i];
    FieldPtrs<T> p{};
    p.params = static_cast<const T*>(params[i]);
    p.pmin = fwd ? static_cast<T*>(pmin[i]) : nullptr;
    p.pmax = fwd ? static_cast<T*>(pmax[i]) : nullptr;
    p.gmin = bwd ? static_cast<const T*>(gmin[i]) : nullptr;
    p.gmax = bwd ? static_cast<const T*>(gmax[i]) : nullptr;
    p.grad = bwd ? static_cast<T*>(grad[i]) : nullptr;
    p.H = f.H;
    p.W = f.W;
    p.nb = f.nb;
    p.rs = f.rs;
    p.ps = f.plane();
    bf[i].p = p;
    bf[i].model = f.model;
    bf[i].J = P.ws_offset[i] == SIZE_MAX ? nullptr
                                         : reinterpret_cast<T*>(static_cast<unsigned char*>(P.d_ws) + P.ws_offset[i]);
  }
}

template <typename T>
hipError_t launch_typed(const Plan& P, hipStream_t st) {
  const auto* F = static_cast<const BatchField<T>*>(P.d_fields);
  if (P.bwd)
    hipLaunchKernelGGL((k_batched<T, PASS_BWD>), dim3(P.main.grid), dim3(kNT), P.main.lds, st, F, P.main.d_tiles,
                       P.main.d_start);
  else
    hipLaunchKernelGGL((k_batched<T, PASS_FWD>), dim3(P.main.grid), dim3(kNT), P.main.lds, st, F, P.main.d_tiles,
                       P.main.d_start);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || P.gather.grid == 0) return e;
  hipLaunchKernelGGL((k_batched<T, PASS_GATHER>), dim3(P.gather.grid), dim3(kNT), 0, st, F, P.gather.d_tiles,
                     P.gather.d_start);
  return hipGetLastError();
}

hipError_t launch(const Plan& P, hipStream_t st) {
  return P.dtype == CP_F64 ? launch_typed<double>(P, st) : launch_typed<float>(P, st);
}

}  // namespace

cp_status_t batched(int n, const Field* fs, const void* const* params, void* const* pmin, void* const* pmax,
                    const void* const* gmin, const void* const* gmax, void* const* grad, uint32_t flags,
                    hipStream_t st, const char** why) {
  const bool fwd = flags & CP_BATCH_FWD, bwd = flags & CP_BATCH_BWD;
  if (flags & CP_BATCH_PER_FIELD) {
    for (int i = 0; i < n; ++i) {
      hipError_t e = hipSuccess;
      if (fwd) e = cf_forward(fs[i], params[i], pmin[i], pmax[i], st);
      if (bwd && e == hipSuccess) e = cf_backward(fs[i], params[i], gmin[i], gmax[i], grad[i], st);
      if (e != hipSuccess) {
        *why = "batched: per-field launch failed";
        return CP_EDEVICE;
      }
    }
    return CP_OK;
  }
  std::vector<int64_t> key;
  key.reserve(4 + 4 * (size_t)n);
  key.push_back(n);
  key.push_back(fs[0].dtype);
  key.push_back(flags & (CP_BATCH_FWD | CP_BATCH_BWD));
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CP_EDEVICE;
  key.push_back(dev);
  for (int i = 0; i < n; ++i) {
    key.push_back(fs[i].H);
    key.push_back(fs[i].W);
    key.push_back(fs[i].rs);
    key.push_back(fs[i].model * 1000 + fs[i].nb);
  }
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_plans.find(key);
  if (it == g_plans.end()) {
    auto P = std::make_unique<Plan>();
    cp_status_t s = build_plan(n, fs, bwd, *P, why);
    if (s != CP_OK) return s;
    it = g_plans.emplace(key, std::move(P)).first;
  }
  Plan& P = *it->second;
  std::vector<unsigned char> table;
  if (P.dtype == CP_F64)
    fill_fields<double>(n, fs, P, params, pmin, pmax, gmin, gmax, grad, fwd, bwd, table);
  else
    fill_fields<float>(n, fs, P, params, pmin, pmax, gmin, gmax, grad, fwd, bwd, table);
  if (table != P.host_fields) {
    // pageable source: the copy is staged before the call returns, so the
    // host vector may be reused at once
    if (hipMemcpyAsync(P.d_fields, table.data(), table.size(), hipMemcpyHostToDevice, st) != hipSuccess) {
      *why = "batched: field-table upload failed";
      return CP_EDEVICE;
    }
    P.host_fields.swap(table);
  }
  if (!(flags & CP_BATCH_GRAPH)) {
    if (launch(P, st) != hipSuccess) {
      *why = "batched: launch failed";
      return CP_EDEVICE;
    }
    return CP_OK;
  }
  if (!P.exec) {
    hipStream_t cs;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return CP_EDEVICE;
    bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
    ok = ok && launch(P, cs) == hipSuccess;
    hipGraph_t g = nullptr;
    ok = (hipStreamEndCapture(cs, &g) == hipSuccess) && ok;
    (void)hipStreamDestroy(cs);
    if (!ok || !g) {
      if (g) (void)hipGraphDestroy(g);
      *why = "batched: graph capture failed";
      return CP_EDEVICE;
    }
    if (hipGraphInstantiate(&P.exec, g, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(g);
      P.exec = nullptr;
      *why = "batched: graph instantiation failed";
      return CP_EDEVICE;
    }
    P.graph = g;
  }
  if (hipGraphLaunch(P.exec, st) != hipSuccess) {
    *why = "batched: graph launch failed";
    return CP_EDEVICE;
  }
  return CP_OK;
}

void batched_release() {
  std::lock_guard<std::mutex> lk(g_mu);
  g_plans.clear();
}

}  // namespace cp
