// cp_batched.hip -- many fields of uneven size and mixed closed-form models
// in one persistent launch per pass.
//
// Small fields under-fill 256 CUs when launched one by one (a 128^2 field is
// 64 forward tiles); the batched form flattens every field into tiles, orders
// them by a per-vertex cost model (most expensive first, then field and row
// order) and lets a grid of resident blocks take them from a device-side
// queue: block after block claims the next tile with one atomic, so blocks
// that draw cheap tiles simply take more of them.  The last block to leave
// resets the queue, so every launch (and every graph replay) starts from a
// zeroed counter without a memset.  The tile lists depend only on the
// shapes, so they are built and uploaded once per shape signature; the field
// table (data pointers) is refreshed only when a pointer changes.  With CP_BATCH_GRAPH the launches are captured once per
// signature into a HIP graph and replayed.
//
// Every pass is its own kernel instantiation and persistent launch: histogram
// tiles and uniform / Epanechnikov tiles run in separate passes, so each
// carries only the registers and LDS of its own tile routine (the latency-
// bound histogram sweep keeps the occupancy of its per-field kernel).
// Histogram adjoint tiles write their per-stencil Jacobians to a workspace
// owned by the plan, and a last pass gathers them; forward values are written
// by the adjoint tiles when both are requested.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
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

enum { PASS_FWD_UE = 0, PASS_FWD_HIST = 1, PASS_BWD_UE = 2, PASS_BWD_HIST = 3, PASS_GATHER = 4, NPASS = 5 };

struct BatchTile {
  int field, ty0, tx0, pad;  // gather tiles: ty0 = first flat vertex index
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

// The FP32 histogram forward pass keeps the 5 waves per SIMD of its per-field
// kernel (the tile loop would otherwise push it one register over).
template <typename T, int PASS>
constexpr int batched_min_waves() {
  return sizeof(T) == 4 && PASS == PASS_FWD_HIST ? 5 : 1;
}

// Tiles are claimed in chunks of `chunk` consecutive entries (neighbouring
// tiles of one field, so halo lines are reused in the claiming CU's L2).
// queue[0]: next unclaimed chunk; queue[1]: blocks that have left.  The claim
// of the next chunk is issued before the current one is processed, so its
// latency overlaps the tile's own loads.  Every block leaves once the counter
// has passed the last chunk (the loop ends for all).
template <typename T, int PASS>
__global__ __launch_bounds__(kNT, (batched_min_waves<T, PASS>())) void k_batched(
    const BatchField<T>* __restrict__ fields, const BatchTile* __restrict__ tiles, int ntiles, int chunk,
    int* queue) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int claimed;
  T* lds = reinterpret_cast<T*>(smem);
  const int tid = threadIdx.x;
  constexpr int OB = sizeof(T) == 4 ? kBwdF32 : kBwdF64;
  const int nchunks = (ntiles + chunk - 1) / chunk;
  if (tid == 0) claimed = atomicAdd(&queue[0], 1);
  __syncthreads();
  int c = claimed;
  __syncthreads();  // every thread has read `claimed` before it is rewritten
  while (c < nchunks) {
    int ahead = 0;
    if (tid == 0) ahead = atomicAdd(&queue[0], 1);
    const int t1 = min(ntiles, (c + 1) * chunk);
    for (int t = c * chunk; t < t1; ++t) {
      const BatchTile tl = tiles[t];
      const BatchField<T> F = fields[tl.field];
      if (PASS == PASS_FWD_UE) {
        if (F.model == CP_UNIFORM)
          tile_fwd_ue<T, CP_UNIFORM, 4>(F.p, tl.ty0, tl.tx0, lds, tid);
        else
          tile_fwd_ue<T, CP_EPANECHNIKOV, 4>(F.p, tl.ty0, tl.tx0, lds, tid);
      } else if (PASS == PASS_FWD_HIST) {
        tile_fwd_hist<T, 4>(F.p, tl.ty0, tl.tx0, lds, tid);
      } else if (PASS == PASS_BWD_UE) {
        if (F.model == CP_UNIFORM)
          tile_bwd_ue<T, CP_UNIFORM, OB, OB, kNT>(F.p, tl.ty0, tl.tx0, lds, tid);
        else
          tile_bwd_ue<T, CP_EPANECHNIKOV, OB, OB, kNT>(F.p, tl.ty0, tl.tx0, lds, tid);
      } else if (PASS == PASS_BWD_HIST) {
        tile_hist_sweep<T, 4>(F.p, tl.ty0, tl.tx0, lds, tid, F.J);
      } else {
        hist_gather_chunk<T>(F.p, F.J, tl.ty0, tid);
      }
    }
    if (tid == 0) claimed = ahead;
    __syncthreads();
    c = claimed;
    __syncthreads();
  }
  if (tid == 0) {
    __threadfence();
    // the last block out has seen every claim: reset the queue for the next launch
    if (atomicAdd(&queue[1], 1) == (int)gridDim.x - 1) {
      atomicExch(&queue[0], 0);
      atomicExch(&queue[1], 0);
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
  int kind = 0;
  int grid = 0;
  size_t lds = 0;
  int ntiles = 0;
  int chunk = 1;
  int* d_queue = nullptr;  // 2 counters, zero between launches
  BatchTile* d_tiles = nullptr;
};

struct Plan {
  int dtype = 0;
  bool bwd = false;
  std::vector<Pass> passes;  // launched in this order
  void* d_fields = nullptr;
  void* d_ws = nullptr;             // histogram Jacobians of all fields
  std::vector<size_t> ws_offset;    // bytes, per field (SIZE_MAX: none)
  std::vector<unsigned char> host_fields;  // last uploaded field table
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  ~Plan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (Pass& p : passes) {
      if (p.d_queue) (void)hipFree(p.d_queue);
      if (p.d_tiles) (void)hipFree(p.d_tiles);
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

template <typename T>
hipError_t prepare_typed(int pass, size_t lds, int* per_cu) {
  switch (pass) {
    case PASS_FWD_UE:
      return prepare_kernel<T, PASS_FWD_UE>(lds, per_cu);
    case PASS_FWD_HIST:
      return prepare_kernel<T, PASS_FWD_HIST>(lds, per_cu);
    case PASS_BWD_UE:
      return prepare_kernel<T, PASS_BWD_UE>(lds, per_cu);
    case PASS_BWD_HIST:
      return prepare_kernel<T, PASS_BWD_HIST>(lds, per_cu);
    default:
      return prepare_kernel<T, PASS_GATHER>(lds, per_cu);
  }
}

hipError_t prepare(int dtype, int pass, size_t lds, int* per_cu) {
  return dtype == CP_F64 ? prepare_typed<double>(pass, lds, per_cu) : prepare_typed<float>(pass, lds, per_cu);
}

// Order the tiles (most expensive first; field / row order among equals),
// size the resident grid and upload.
cp_status_t build_pass(const std::vector<BatchTile>& tiles, const std::vector<double>& cost, int dtype, int pass,
                       size_t lds, Pass& P) {
  int per_cu = 0;
  if (prepare(dtype, pass, lds, &per_cu) != hipSuccess) return CP_EDEVICE;
  per_cu = std::max(per_cu, 1);
  const int grid = std::max(1, std::min<int>((int)tiles.size(), g_num_cu * per_cu));
  std::vector<int> order(tiles.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<BatchTile> flat;
  flat.reserve(tiles.size());
  for (int t : order) flat.push_back(tiles[t]);
  P.kind = pass;
  P.grid = grid;
  P.lds = lds;
  P.ntiles = (int)flat.size();
  // cheap tiles are claimed several at a time
  P.chunk = pass == PASS_FWD_UE || pass == PASS_GATHER ? 4 : 1;
  if (hipMalloc(&P.d_queue, 2 * sizeof(int)) != hipSuccess) return CP_ENOMEM;
  if (hipMemset(P.d_queue, 0, 2 * sizeof(int)) != hipSuccess) return CP_EDEVICE;
  if (hipMalloc(&P.d_tiles, sizeof(BatchTile) * std::max<size_t>(flat.size(), 1)) != hipSuccess) return CP_ENOMEM;
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
  std::vector<BatchTile> tiles[NPASS];
  std::vector<double> cost[NPASS];
  size_t lds[NPASS] = {0, 0, 0, 0, 0}, ws = 0;
  P.ws_offset.assign(n, SIZE_MAX);
  for (int i = 0; i < n; ++i) {
    const Field& f = fs[i];
    const bool hist = f.model == CP_HISTOGRAM;
    const int pass = bwd ? (hist ? PASS_BWD_HIST : PASS_BWD_UE) : (hist ? PASS_FWD_HIST : PASS_FWD_UE);
    int ox = kFwdTX, oy = 4;
    if (pass == PASS_BWD_UE) ox = oy = el == 4 ? kBwdF32 : kBwdF64;
    lds[pass] = std::max(lds[pass], tile_lds_bytes(f.model, f.nb, bwd, el));
    const double c = vertex_cost(f.model, f.nb, bwd) * ox * oy;
    // columns of tiles (a claimed chunk stacks vertically and shares halo rows)
    for (int tx = 0; tx < f.W; tx += ox)
      for (int ty = 0; ty < f.H; ty += oy) {
        tiles[pass].push_back(BatchTile{i, ty, tx, 0});
        cost[pass].push_back(c);
      }
    if (pass == PASS_BWD_HIST) {
      const int64_t plane = (int64_t)f.H * f.W;
      P.ws_offset[i] = ws;
      ws += el * (size_t)5 * f.nb * plane;
      ws = (ws + 255) / 256 * 256;
      for (int64_t v = 0; v < plane; v += kGatherChunk) {
        tiles[PASS_GATHER].push_back(BatchTile{i, (int)v, 0, 0});
        cost[PASS_GATHER].push_back(1.0);
      }
    }
  }
  for (int q = 0; q < NPASS; ++q)
    if (lds[q] > kMaxLds) {
      *why = "batched: staged planes exceed the LDS of a workgroup (too many bins for this dtype)";
      return CP_EUNSUPPORTED;
    }
  // histogram passes first (the longest), the gather last (it reads their Jacobians)
  for (int q : {PASS_FWD_HIST, PASS_BWD_HIST, PASS_FWD_UE, PASS_BWD_UE, PASS_GATHER}) {
    if (tiles[q].empty()) continue;
    P.passes.emplace_back();
    cp_status_t s = build_pass(tiles[q], cost[q], P.dtype, q, lds[q], P.passes.back());
    if (s != CP_OK) return s;
  }
  if (ws > 0 && hipMalloc(&P.d_ws, ws) != hipSuccess) return CP_ENOMEM;
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
  for (const Pass& q : P.passes) {
    const dim3 g(q.grid), b(kNT);
    switch (q.kind) {
      case PASS_FWD_UE:
        hipLaunchKernelGGL((k_batched<T, PASS_FWD_UE>), g, b, q.lds, st, F, q.d_tiles, q.ntiles, q.chunk, q.d_queue);
        break;
      case PASS_FWD_HIST:
        hipLaunchKernelGGL((k_batched<T, PASS_FWD_HIST>), g, b, q.lds, st, F, q.d_tiles, q.ntiles, q.chunk, q.d_queue);
        break;
      case PASS_BWD_UE:
        hipLaunchKernelGGL((k_batched<T, PASS_BWD_UE>), g, b, q.lds, st, F, q.d_tiles, q.ntiles, q.chunk, q.d_queue);
        break;
      case PASS_BWD_HIST:
        hipLaunchKernelGGL((k_batched<T, PASS_BWD_HIST>), g, b, q.lds, st, F, q.d_tiles, q.ntiles, q.chunk, q.d_queue);
        break;
      default:
        hipLaunchKernelGGL((k_batched<T, PASS_GATHER>), g, b, q.lds, st, F, q.d_tiles, q.ntiles, q.chunk, q.d_queue);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
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
