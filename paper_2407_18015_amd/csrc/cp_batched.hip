// cp_batched.hip -- many fields of uneven size and mixed closed-form models
// in one persistent launch.
//
// Small fields under-fill 256 CUs when launched one by one (a 128^2 field is
// 64 forward tiles); the batched form flattens every field into tiles, deals
// the tiles to a grid of resident blocks by a longest-processing-time rule
// over a per-vertex cost model, and lets each block walk its own list.  The
// tile lists depend only on the shapes, so they are built and uploaded once
// per shape signature; the field table (data pointers) is refreshed only when
// a pointer changes.  With CP_BATCH_GRAPH the launch is captured once per
// signature into a HIP graph and replayed.
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
constexpr int kBwdF32 = 30, kBwdF64 = 14, kBwdHist = 14;  // adjoint tile edges
constexpr size_t kMaxLds = 160 * 1024;

struct BatchTile {
  int field, ty0, tx0, kind;  // kind 0 = forward tile, 1 = adjoint (fused) tile
};

template <typename T>
struct BatchField {
  FieldPtrs<T> p;
  int model;
};

template <typename T>
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
    if (tl.kind == 0) {
      if (F.model == CP_UNIFORM)
        tile_fwd_ue<T, CP_UNIFORM, 4>(F.p, tl.ty0, tl.tx0, lds, tid);
      else if (F.model == CP_EPANECHNIKOV)
        tile_fwd_ue<T, CP_EPANECHNIKOV, 4>(F.p, tl.ty0, tl.tx0, lds, tid);
      else
        tile_fwd_hist<T, 4>(F.p, tl.ty0, tl.tx0, lds, tid);
    } else {
      constexpr int OB = sizeof(T) == 4 ? kBwdF32 : kBwdF64;
      if (F.model == CP_UNIFORM)
        tile_bwd_ue<T, CP_UNIFORM, OB, OB, kNT>(F.p, tl.ty0, tl.tx0, lds, tid);
      else if (F.model == CP_EPANECHNIKOV)
        tile_bwd_ue<T, CP_EPANECHNIKOV, OB, OB, kNT>(F.p, tl.ty0, tl.tx0, lds, tid);
      else
        tile_bwd_hist<T, kBwdHist, kBwdHist, kNT>(F.p, tl.ty0, tl.tx0, lds, tid);
    }
  }
}

// relative cost per vertex (forward, adjoint) by model, used for balancing
double vertex_cost(int model, int nb, bool bwd) {
  if (model == CP_UNIFORM) return bwd ? 3.0 : 1.0;
  if (model == CP_EPANECHNIKOV) return bwd ? 10.0 : 3.5;
  return (bwd ? 12.0 : 4.0) * (nb + 1);
}

size_t tile_lds_bytes(int model, int nb, bool bwd, size_t el) {
  if (!bwd) {
    if (model == CP_HISTOGRAM) return el * (size_t)hist_planes(nb) * (kFwdTX + 2) * 6;
    return el * 2 * (kFwdTX + 2) * 6;
  }
  if (model == CP_HISTOGRAM) return el * hist_bwd_lds_elems<kBwdHist, kBwdHist>(nb);
  if (el == 4) return el * bwd_ue_lds_elems<kBwdF32, kBwdF32>();
  return el * bwd_ue_lds_elems<kBwdF64, kBwdF64>();
}

struct Plan {
  int dtype = 0, grid = 0;
  size_t lds = 0;
  int* d_start = nullptr;
  BatchTile* d_tiles = nullptr;
  void* d_fields = nullptr;
  size_t field_bytes = 0;
  std::vector<unsigned char> host_fields;  // last uploaded field table
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  ~Plan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (d_start) (void)hipFree(d_start);
    if (d_tiles) (void)hipFree(d_tiles);
    if (d_fields) (void)hipFree(d_fields);
  }
};

std::mutex g_mu;
std::map<std::vector<int64_t>, std::unique_ptr<Plan>> g_plans;
int g_num_cu = 0;

template <typename T>
hipError_t occupancy(size_t lds, int* blocks) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, reinterpret_cast<const void*>(k_batched<T>), kNT,
                                                      lds);
}

template <typename T>
hipError_t set_lds(size_t lds) {
  if (lds <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k_batched<T>), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds);
}

cp_status_t build_plan(int n, const Field* fs, bool fwd, bool bwd, Plan& P, const char** why) {
  const size_t el = fs[0].dtype == CP_F64 ? 8 : 4;
  P.dtype = fs[0].dtype;
  std::vector<BatchTile> tiles;
  std::vector<double> cost;
  size_t lds = 0;
  for (int i = 0; i < n; ++i) {
    const Field& f = fs[i];
    const bool adj = bwd;  // adjoint tiles also write P when requested
    int ox, oy;
    if (adj) {
      ox = oy = f.model == CP_HISTOGRAM ? kBwdHist : (el == 4 ? kBwdF32 : kBwdF64);
    } else {
      ox = kFwdTX;
      oy = 4;
    }
    lds = std::max(lds, tile_lds_bytes(f.model, f.nb, adj, el));
    const double c = vertex_cost(f.model, f.nb, adj) * ox * oy;
    for (int ty = 0; ty < f.H; ty += oy)
      for (int tx = 0; tx < f.W; tx += ox) {
        tiles.push_back(BatchTile{i, ty, tx, adj ? 1 : 0});
        cost.push_back(c);
      }
  }
  (void)fwd;
  if (lds > kMaxLds) {
    *why = "batched: staged planes exceed the LDS of a workgroup (too many bins for this dtype)";
    return CP_EUNSUPPORTED;
  }
  hipError_t e = el == 4 ? set_lds<float>(lds) : set_lds<double>(lds);
  if (e != hipSuccess) return CP_EDEVICE;
  int per_cu = 0;
  e = el == 4 ? occupancy<float>(lds, &per_cu) : occupancy<double>(lds, &per_cu);
  if (e != hipSuccess) return CP_EDEVICE;
  if (g_num_cu == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return CP_EDEVICE;
    if (hipDeviceGetAttribute(&g_num_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return CP_EDEVICE;
  }
  per_cu = std::max(per_cu, 1);
  const int grid = std::max(1, std::min<int>((int)tiles.size(), g_num_cu * per_cu));
  // longest-processing-time: biggest tiles first, each to the least-loaded block
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
    // walk a block's tiles in field/row order for locality
    std::sort(lists[b].begin(), lists[b].end());
    for (int t : lists[b]) flat.push_back(tiles[t]);
  }
  start[grid] = (int)flat.size();
  P.grid = grid;
  P.lds = lds;
  P.field_bytes = (el == 4 ? sizeof(BatchField<float>) : sizeof(BatchField<double>)) * (size_t)n;
  if (hipMalloc(&P.d_start, sizeof(int) * start.size()) != hipSuccess) return CP_ENOMEM;
  if (hipMalloc(&P.d_tiles, sizeof(BatchTile) * std::max<size_t>(flat.size(), 1)) != hipSuccess) return CP_ENOMEM;
  if (hipMalloc(&P.d_fields, P.field_bytes) != hipSuccess) return CP_ENOMEM;
  if (hipMemcpy(P.d_start, start.data(), sizeof(int) * start.size(), hipMemcpyHostToDevice) != hipSuccess)
    return CP_EDEVICE;
  if (!flat.empty() &&
      hipMemcpy(P.d_tiles, flat.data(), sizeof(BatchTile) * flat.size(), hipMemcpyHostToDevice) != hipSuccess)
    return CP_EDEVICE;
  return CP_OK;
}

template <typename T>
void fill_fields(int n, const Field* fs, const void* const* params, void* const* pmin, void* const* pmax,
                 const void* const* gmin, const void* const* gmax, void* const* grad, bool fwd, bool bwd,
                 std::vector<unsigned char>& out) {
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
  }
}

hipError_t launch(const Plan& P, hipStream_t st) {
  if (P.dtype == CP_F64)
    hipLaunchKernelGGL(k_batched<double>, dim3(P.grid), dim3(kNT), P.lds, st,
                       static_cast<const BatchField<double>*>(P.d_fields), P.d_tiles, P.d_start);
  else
    hipLaunchKernelGGL(k_batched<float>, dim3(P.grid), dim3(kNT), P.lds, st,
                       static_cast<const BatchField<float>*>(P.d_fields), P.d_tiles, P.d_start);
  return hipGetLastError();
}

}  // namespace

cp_status_t batched(int n, const Field* fs, const void* const* params, void* const* pmin, void* const* pmax,
                    const void* const* gmin, const void* const* gmax, void* const* grad, uint32_t flags,
                    hipStream_t st, const char** why) {
  const bool fwd = flags & CP_BATCH_FWD, bwd = flags & CP_BATCH_BWD;
  if (flags & CP_BATCH_PER_FIELD) {
    for (int i = 0; i < n; ++i) {
      hipError_t e = hipSuccess;
      if (fwd && !bwd) e = cf_forward(fs[i], params[i], pmin[i], pmax[i], st);
      if (bwd) {
        if (fwd) e = cf_forward(fs[i], params[i], pmin[i], pmax[i], st);
        if (e == hipSuccess) e = cf_backward(fs[i], params[i], gmin[i], gmax[i], grad[i], st);
      }
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
    cp_status_t s = build_plan(n, fs, fwd, bwd, *P, why);
    if (s != CP_OK) return s;
    it = g_plans.emplace(key, std::move(P)).first;
  }
  Plan& P = *it->second;
  std::vector<unsigned char> table;
  if (P.dtype == CP_F64)
    fill_fields<double>(n, fs, params, pmin, pmax, gmin, gmax, grad, fwd, bwd, table);
  else
    fill_fields<float>(n, fs, params, pmin, pmax, gmin, gmax, grad, fwd, bwd, table);
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
