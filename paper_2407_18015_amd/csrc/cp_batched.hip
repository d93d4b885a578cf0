// cp_batched.hip -- many fields of uneven size and mixed closed-form models
// in one launch per pass.
//
// Small fields under-fill 256 CUs when launched one by one (a 128^2 field is
// 64 forward tiles); the batched form flattens every field into tiles, orders
// them by a per-vertex cost model (most expensive first, then field and row
// order) and launches them as one grid per pass, one tile per block, which the
// dispatcher hands out in that order as slots free up.  A persistent form is
// the alternative the autotuner also times: a grid of resident blocks takes
// the tiles from a device-side queue, block after block claiming the next
// chunk with one atomic, so blocks that draw cheap tiles take more of them.  The last block to leave
// resets the queue, so every launch (and every graph replay) starts from a
// zeroed counter without a memset.  The tile lists depend only on the
// shapes, so they are built and uploaded once per shape signature; the field
// table (data pointers) is refreshed only when a pointer changes.  With CP_BATCH_GRAPH the launches are captured once per
// signature into a HIP graph and replayed.
//
// The one-tile-per-block form (`chunk` 0 in a plan) keeps the registers of
// the per-field kernels (the histogram sweeps: 96 and 80 VGPRs against 109
// and 94 inside the claim loop) and saves the claims.
//
// Every pass is its own kernel instantiation and launch: histogram
// tiles and uniform / Epanechnikov tiles run in separate passes, so each
// carries only the registers and LDS of its own tile routine (the latency-
// bound histogram sweep keeps the occupancy of its per-field kernel).
// Histogram adjoint tiles write their per-stencil Jacobians to a workspace
// owned by the plan, and a last pass gathers them; forward values are written
// by the adjoint tiles when both are requested.  A plan used from a second
// stream waits (on the device) for the first stream's last use of it, so
// calls on different streams never share a tile queue while it is in flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <sstream>
#include <string>
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
constexpr int kGatherChunk = 256;          // histogram gather: vertices per tile
constexpr size_t kMaxLds = 160 * 1024;

enum { PASS_FWD_UE = 0, PASS_FWD_HIST = 1, PASS_BWD_UE = 2, PASS_BWD_HIST = 3, PASS_GATHER = 4, NPASS = 5 };

// Tile variants of each pass (the tuner picks one per pass; variant 0 is the
// default).  Forward and histogram passes: 64 x (4 << v) vertices, one, two
// or (uniform / Epanechnikov forward) four rows per thread.  Uniform /
// Epanechnikov adjoint: output tiles of
// bwd_ox x bwd_oy (FP32 30x30, 14x14, 62x30; FP64 14x14, 30x14, 30x30), i.e.
// 1 to 8 stencils per thread.  The tile shape changes no per-vertex
// arithmetic: every variant gives the same results bit for bit.
constexpr int n_variants(int pass) {
  return pass == PASS_BWD_UE || pass == PASS_FWD_UE ? 3 : (pass == PASS_GATHER ? 1 : 2);
}
__host__ __device__ constexpr int bwd_ox(bool f32, int v) { return f32 ? (v == 2 ? 62 : (v == 1 ? 14 : 30)) : (v == 0 ? 14 : 30); }
__host__ __device__ constexpr int bwd_oy(bool f32, int v) { return f32 ? (v == 1 ? 14 : 30) : (v == 2 ? 30 : 14); }

struct BatchTile {
  int field, ty0, tx0, pad;  // gather tiles: ty0 = first flat vertex index
};

template <typename T>
struct BatchField {
  FieldPtrs<T> p;
  T* J;  // histogram adjoint workspace ([5 h + 4][H][W]) or null
  int model;
};

// The FP32 histogram forward pass keeps the 5 waves per SIMD of its per-field
// kernel (the tile loop would otherwise push it one register over), and the
// FP32 histogram adjoint sweep 4 (at 132 registers it would drop to 3: the
// tuned 64 x 8 variant then ran 7% longer).
template <typename T, int PASS>
constexpr int batched_min_waves() {
  return sizeof(T) == 4 && PASS == PASS_FWD_HIST ? 5 : (sizeof(T) == 4 && PASS == PASS_BWD_HIST ? 4 : 1);
}

// Tiles are claimed in chunks of `chunk` consecutive entries (neighbouring
// tiles of one field, so halo lines are reused in the claiming CU's L2).
// queue[0]: next unclaimed chunk; queue[1]: blocks that have left.  The claim
// of the next chunk is issued before the current one is processed, so its
// latency overlaps the tile's own loads.  Every block leaves once the counter
// has passed the last chunk (the loop ends for all).
template <typename T, int PASS, int V>
__device__ __forceinline__ void batched_tile(const BatchField<T>* __restrict__ fields, const BatchTile tl, T* lds,
                                             int tid) {
  constexpr int TY = 4 << V;
  constexpr int OX = bwd_ox(sizeof(T) == 4, V), OY = bwd_oy(sizeof(T) == 4, V);
  const BatchField<T> F = fields[tl.field];
  if constexpr (PASS == PASS_FWD_UE) {
    if (F.model == CP_UNIFORM)
      tile_fwd_ue<T, CP_UNIFORM, TY, kNT>(F.p, tl.ty0, tl.tx0, lds, tid);
    else
      tile_fwd_ue<T, CP_EPANECHNIKOV, TY, kNT>(F.p, tl.ty0, tl.tx0, lds, tid);
  } else if constexpr (PASS == PASS_FWD_HIST) {
    tile_fwd_hist<T, TY, kNT>(F.p, tl.ty0, tl.tx0, lds, tid);
  } else if constexpr (PASS == PASS_BWD_UE) {
    if (F.model == CP_UNIFORM)
      tile_bwd_ue<T, CP_UNIFORM, OX, OY, kNT>(F.p, tl.ty0, tl.tx0, lds, tid);
    else
      tile_bwd_ue<T, CP_EPANECHNIKOV, OX, OY, kNT>(F.p, tl.ty0, tl.tx0, lds, tid);
  } else if constexpr (PASS == PASS_BWD_HIST) {
    tile_hist_sweep<T, TY, kNT>(F.p, tl.ty0, tl.tx0, lds, tid, F.J);
  } else {
    hist_gather_vertex<T>(F.p, F.J, (int64_t)tl.ty0 + tid);
  }
}

// One tile per block, blocks in the table's order (the dispatcher hands them
// out as slots free up, most expensive first): no claim loop around the tile,
// so a pass keeps the registers of its per-field kernel.
template <typename T, int PASS, int V>
__global__ __launch_bounds__(kNT) void k_batched_flat(const BatchField<T>* __restrict__ fields,
                                                      const BatchTile* __restrict__ tiles) {
  extern __shared__ __align__(16) unsigned char smem[];
  batched_tile<T, PASS, V>(fields, tiles[blockIdx.x], reinterpret_cast<T*>(smem), threadIdx.x);
}

template <typename T, int PASS, int V>
__global__ __launch_bounds__(kNT, (batched_min_waves<T, PASS>())) void k_batched(
    const BatchField<T>* __restrict__ fields, const BatchTile* __restrict__ tiles, int ntiles, int chunk,
    int* queue) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int claimed;
  T* lds = reinterpret_cast<T*>(smem);
  const int tid = threadIdx.x;
  constexpr int TY = 4 << V;
  constexpr int OX = bwd_ox(sizeof(T) == 4, V), OY = bwd_oy(sizeof(T) == 4, V);
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
      batched_tile<T, PASS, V>(fields, tiles[t], lds, tid);
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

template <typename T>
const void* kernel_flat_of(int pass, int v) {
  switch (pass * 4 + v) {
    case PASS_FWD_UE * 4 + 0: return reinterpret_cast<const void*>(k_batched_flat<T, PASS_FWD_UE, 0>);
    case PASS_FWD_UE * 4 + 1: return reinterpret_cast<const void*>(k_batched_flat<T, PASS_FWD_UE, 1>);
    case PASS_FWD_UE * 4 + 2: return reinterpret_cast<const void*>(k_batched_flat<T, PASS_FWD_UE, 2>);
    case PASS_FWD_HIST * 4 + 0: return reinterpret_cast<const void*>(k_batched_flat<T, PASS_FWD_HIST, 0>);
    case PASS_FWD_HIST * 4 + 1: return reinterpret_cast<const void*>(k_batched_flat<T, PASS_FWD_HIST, 1>);
    case PASS_BWD_UE * 4 + 0: return reinterpret_cast<const void*>(k_batched_flat<T, PASS_BWD_UE, 0>);
    case PASS_BWD_UE * 4 + 1: return reinterpret_cast<const void*>(k_batched_flat<T, PASS_BWD_UE, 1>);
    case PASS_BWD_UE * 4 + 2: return reinterpret_cast<const void*>(k_batched_flat<T, PASS_BWD_UE, 2>);
    case PASS_BWD_HIST * 4 + 0: return reinterpret_cast<const void*>(k_batched_flat<T, PASS_BWD_HIST, 0>);
    case PASS_BWD_HIST * 4 + 1: return reinterpret_cast<const void*>(k_batched_flat<T, PASS_BWD_HIST, 1>);
    default: return reinterpret_cast<const void*>(k_batched_flat<T, PASS_GATHER, 0>);
  }
}

template <typename T>
const void* kernel_of(int pass, int v) {
  switch (pass * 4 + v) {
    case PASS_FWD_UE * 4 + 0: return reinterpret_cast<const void*>(k_batched<T, PASS_FWD_UE, 0>);
    case PASS_FWD_UE * 4 + 1: return reinterpret_cast<const void*>(k_batched<T, PASS_FWD_UE, 1>);
    case PASS_FWD_UE * 4 + 2: return reinterpret_cast<const void*>(k_batched<T, PASS_FWD_UE, 2>);
    case PASS_FWD_HIST * 4 + 0: return reinterpret_cast<const void*>(k_batched<T, PASS_FWD_HIST, 0>);
    case PASS_FWD_HIST * 4 + 1: return reinterpret_cast<const void*>(k_batched<T, PASS_FWD_HIST, 1>);
    case PASS_BWD_UE * 4 + 0: return reinterpret_cast<const void*>(k_batched<T, PASS_BWD_UE, 0>);
    case PASS_BWD_UE * 4 + 1: return reinterpret_cast<const void*>(k_batched<T, PASS_BWD_UE, 1>);
    case PASS_BWD_UE * 4 + 2: return reinterpret_cast<const void*>(k_batched<T, PASS_BWD_UE, 2>);
    case PASS_BWD_HIST * 4 + 0: return reinterpret_cast<const void*>(k_batched<T, PASS_BWD_HIST, 0>);
    case PASS_BWD_HIST * 4 + 1: return reinterpret_cast<const void*>(k_batched<T, PASS_BWD_HIST, 1>);
    default: return reinterpret_cast<const void*>(k_batched<T, PASS_GATHER, 0>);
  }
}

// Relative cost per vertex (forward, adjoint), measured on MI355X with the
// per-field kernels at 2048^2 (uniform forward = 1: 40.6 us; uniform adjoint
// 64.7 us, Epanechnikov forward 85 us and adjoint 147.5 us, 10-bin histogram
// forward 0.545 ms and adjoint 1.41 ms); histograms scale with the number of
// bin edges.  The costs only order the tiles of one pass (longest first), so
// within a pass only the ratios between models matter.
double vertex_cost(int model, int nb, bool bwd) {
  if (model == CP_UNIFORM) return bwd ? 1.6 : 1.0;
  if (model == CP_EPANECHNIKOV) return bwd ? 3.6 : 2.1;
  return (bwd ? 3.2 : 1.2) * (nb + 1);
}

const char* pass_name(int pass) {
  static const char* names[NPASS] = {"forward", "histogram forward", "adjoint", "histogram adjoint sweep",
                                     "histogram gather"};
  return names[pass];
}

// output tile extents of a pass variant
void pass_geom(int pass, int v, size_t el, int& ox, int& oy) {
  if (pass == PASS_BWD_UE) {
    ox = bwd_ox(el == 4, v);
    oy = bwd_oy(el == 4, v);
  } else if (pass == PASS_GATHER) {
    ox = kGatherChunk;
    oy = 1;
  } else {
    ox = kFwdTX;
    oy = 4 << v;
  }
}

size_t tile_lds_bytes(int pass, int v, int nb, size_t el) {
  int ox, oy;
  pass_geom(pass, v, el, ox, oy);
  if (pass == PASS_FWD_HIST || pass == PASS_BWD_HIST) return el * (size_t)hist_planes(nb) * (ox + 2) * (oy + 2);
  if (pass == PASS_FWD_UE) return el * 2 * (ox + 2) * (oy + 2);
  if (pass == PASS_BWD_UE) return el * 8 * (size_t)(ox + 2) * (oy + 2);
  return 0;
}

struct Pass {
  int kind = 0;
  int variant = 0;
  int grid = 0;
  size_t lds = 0;
  int ntiles = 0;
  int chunk = 1;
  double ms = -1.0;        // tuned launch time (ms), < 0 when not tuned
  int* d_queue = nullptr;  // 2 counters, zero between launches
  BatchTile* d_tiles = nullptr;
  void release() {
    if (d_queue) (void)hipFree(d_queue);
    if (d_tiles) (void)hipFree(d_tiles);
    d_queue = nullptr;
    d_tiles = nullptr;
  }
};

struct Plan {
  int dtype = 0;
  bool bwd = false;
  bool tuned = false;
  std::vector<Field> fields;
  std::vector<Pass> passes;  // launched in this order
  void* d_fields = nullptr;
  void* d_ws = nullptr;             // histogram Jacobians of all fields
  std::vector<size_t> ws_offset;    // bytes, per field (SIZE_MAX: none)
  std::vector<unsigned char> host_fields;  // last uploaded field table
  bool from_table = false;          // tuning choices read from the tuning table
  hipStream_t last = nullptr;       // stream of the last call that used the plan
  hipEvent_t done = nullptr;        // recorded on `last` after that call's launches
  bool used = false;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
  ~Plan() {
    drop_graph();
    for (Pass& p : passes) p.release();
    if (d_fields) (void)hipFree(d_fields);
    if (d_ws) (void)hipFree(d_ws);
    if (done) (void)hipEventDestroy(done);
  }
};

std::mutex g_mu;
std::map<std::vector<int64_t>, std::unique_ptr<Plan>> g_plans;
int g_num_cu = 0;

const void* kernel_for(int dtype, int pass, int v) {
  return dtype == CP_F64 ? kernel_of<double>(pass, v) : kernel_of<float>(pass, v);
}

// the one-tile-per-block form of a pass
const void* kernel_flat_for(int dtype, int pass, int v) {
  return dtype == CP_F64 ? kernel_flat_of<double>(pass, v) : kernel_flat_of<float>(pass, v);
}

// resident blocks per CU of a pass variant (0: it cannot run)
hipError_t blocks_per_cu(int dtype, int pass, int v, size_t lds, int* per_cu) {
  const void* k = kernel_for(dtype, pass, v);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k, kNT, lds);
}

// The tiles of one pass variant over every field of that pass, most
// expensive first (field and column order among equals: a claimed chunk
// stacks tiles vertically and shares their halo rows).
void pass_tiles(const std::vector<Field>& fs, int pass, int v, size_t el, std::vector<BatchTile>& out,
                int& max_nb) {
  int ox, oy;
  pass_geom(pass, v, el, ox, oy);
  std::vector<BatchTile> tiles;
  std::vector<double> cost;
  max_nb = 0;
  for (int i = 0; i < (int)fs.size(); ++i) {
    const Field& f = fs[i];
    const bool hist = f.model == CP_HISTOGRAM;
    const bool mine = pass == PASS_FWD_UE || pass == PASS_BWD_UE ? !hist : hist;
    if (!mine) continue;
    max_nb = std::max(max_nb, f.nb);
    if (pass == PASS_GATHER) {
      const int64_t plane = (int64_t)f.H * f.W;
      for (int64_t t = 0; t < plane; t += kGatherChunk) {
        tiles.push_back(BatchTile{i, (int)t, 0, 0});
        cost.push_back(1.0);
      }
      continue;
    }
    const double c = vertex_cost(f.model, f.nb, pass == PASS_BWD_UE || pass == PASS_BWD_HIST) * ox * oy;
    for (int tx = 0; tx < f.W; tx += ox)
      for (int ty = 0; ty < f.H; ty += oy) {
        tiles.push_back(BatchTile{i, ty, tx, 0});
        cost.push_back(c);
      }
  }
  std::vector<int> order(tiles.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  out.clear();
  out.reserve(tiles.size());
  for (int t : order) out.push_back(tiles[t]);
}

// Build (allocate, upload) the pass `pass` in variant v.  CP_EUNSUPPORTED:
// the variant does not fit a workgroup.
cp_status_t build_pass(const Plan& P, int pass, int v, int chunk, Pass& out) {
  const size_t el = P.dtype == CP_F64 ? 8 : 4;
  std::vector<BatchTile> flat;
  int max_nb = 0;
  pass_tiles(P.fields, pass, v, el, flat, max_nb);
  const size_t lds = tile_lds_bytes(pass, v, max_nb, el);
  if (lds > kMaxLds) return CP_EUNSUPPORTED;
  int per_cu = 0;
  if (blocks_per_cu(P.dtype, pass, v, lds, &per_cu) != hipSuccess) return CP_EDEVICE;
  if (per_cu < 1) return CP_EUNSUPPORTED;
  const void* fk = kernel_flat_for(P.dtype, pass, v);
  if (fk && lds > 65536 &&
      hipFuncSetAttribute(fk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return CP_EDEVICE;
  Pass Q;
  Q.kind = pass;
  Q.variant = v;
  Q.lds = lds;
  Q.ntiles = (int)flat.size();
  Q.grid = std::max(1, std::min<int>(Q.ntiles, g_num_cu * per_cu));
  Q.chunk = chunk;
  if (hipMalloc(&Q.d_queue, 2 * sizeof(int)) != hipSuccess) return CP_ENOMEM;
  if (hipMemset(Q.d_queue, 0, 2 * sizeof(int)) != hipSuccess) {
    Q.release();
    return CP_EDEVICE;
  }
  if (hipMalloc(&Q.d_tiles, sizeof(BatchTile) * std::max<size_t>(flat.size(), 1)) != hipSuccess) {
    Q.release();
    return CP_ENOMEM;
  }
  if (!flat.empty() &&
      hipMemcpy(Q.d_tiles, flat.data(), sizeof(BatchTile) * flat.size(), hipMemcpyHostToDevice) != hipSuccess) {
    Q.release();
    return CP_EDEVICE;
  }
  out = Q;
  return CP_OK;
}

// default: one tile per block (0); on the 64-field benchmark the tuner chose
// it for every pass in most runs (histogram passes always)
int default_chunk(int) { return 0; }

cp_status_t build_plan(int n, const Field* fs, bool bwd, Plan& P, const char** why) {
  const size_t el = fs[0].dtype == CP_F64 ? 8 : 4;
  P.dtype = fs[0].dtype;
  P.bwd = bwd;
  P.fields.assign(fs, fs + n);
  if (g_num_cu == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return CP_EDEVICE;
    if (hipDeviceGetAttribute(&g_num_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return CP_EDEVICE;
  }
  bool present[NPASS] = {false, false, false, false, false};
  size_t ws = 0;
  P.ws_offset.assign(n, SIZE_MAX);
  for (int i = 0; i < n; ++i) {
    const Field& f = fs[i];
    const bool hist = f.model == CP_HISTOGRAM;
    present[bwd ? (hist ? PASS_BWD_HIST : PASS_BWD_UE) : (hist ? PASS_FWD_HIST : PASS_FWD_UE)] = true;
    if (hist && bwd) {
      present[PASS_GATHER] = true;
      P.ws_offset[i] = ws;
      ws += el * (size_t)hist_ws_planes(f.nb) * f.H * (size_t)f.W;
      ws = (ws + 255) / 256 * 256;
    }
  }
  // histogram passes first (the longest), the gather last (it reads their Jacobians)
  for (int q : {PASS_FWD_HIST, PASS_BWD_HIST, PASS_FWD_UE, PASS_BWD_UE, PASS_GATHER}) {
    if (!present[q]) continue;
    Pass Q;
    cp_status_t s = build_pass(P, q, 0, default_chunk(q), Q);
    if (s == CP_EUNSUPPORTED) {
      *why = "batched: staged planes exceed the LDS of a workgroup (too many bins for this dtype)";
      return s;
    }
    if (s != CP_OK) return s;
    P.passes.push_back(Q);
  }
  if (ws > 0 && hipMalloc(&P.d_ws, ws) != hipSuccess) return CP_ENOMEM;
  if (hipEventCreateWithFlags(&P.done, hipEventDisableTiming) != hipSuccess) return CP_EDEVICE;
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

hipError_t launch_pass(const Plan& P, const Pass& q, hipStream_t st) {
  const void* fields = P.d_fields;
  const BatchTile* tiles = q.d_tiles;
  int ntiles = q.ntiles, chunk = q.chunk;
  int* queue = q.d_queue;
  hipError_t e;
  if (q.chunk == 0) {  // one tile per block, in the table's order
    if (ntiles == 0) return hipSuccess;
    void* fargs[] = {&fields, &tiles};
    e = hipLaunchKernel(kernel_flat_for(P.dtype, q.kind, q.variant), dim3(ntiles), dim3(kNT), fargs, q.lds, st);
  } else {
    void* args[] = {&fields, &tiles, &ntiles, &chunk, &queue};
    e = hipLaunchKernel(kernel_for(P.dtype, q.kind, q.variant), dim3(q.grid), dim3(kNT), args, q.lds, st);
  }
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t launch(const Plan& P, hipStream_t st) {
  for (const Pass& q : P.passes) {
    hipError_t e = launch_pass(P, q, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// mean time (ms) of `reps` back-to-back launches of one pass on st
cp_status_t time_pass(const Plan& P, const Pass& q, hipStream_t st, int reps, double& ms) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return CP_EDEVICE;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return CP_EDEVICE;
  }
  bool ok = launch_pass(P, q, st) == hipSuccess;  // warm-up
  ok = ok && hipEventRecord(a, st) == hipSuccess;
  for (int r = 0; r < reps && ok; ++r) ok = launch_pass(P, q, st) == hipSuccess;
  ok = ok && hipEventRecord(b, st) == hipSuccess && hipEventSynchronize(b) == hipSuccess;
  float t = 0.f;
  ok = ok && hipEventElapsedTime(&t, a, b) == hipSuccess;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  ms = t / reps;
  return ok ? CP_OK : CP_EDEVICE;
}

// Autotuner: for every pass, time each tile variant with each claim chunk
// and with one tile per block, on the plan's own
// fields (the field table must be current) and keep the fastest.  Every
// trial writes the pass's outputs, with the same values.
cp_status_t tune(Plan& P, hipStream_t st) {
  constexpr int kReps = 3;
  const int chunks[] = {0, 1, 2, 4, 8};
  for (Pass& cur : P.passes) {
    Pass best = cur;
    double best_ms = 0.0;
    cp_status_t s = time_pass(P, cur, st, kReps, best_ms);
    if (s != CP_OK) return s;
    // `best` shares its device tables with `cur` or with one built candidate;
    // a built candidate's tables are freed as soon as it is not the best
    for (int v = 0; v < n_variants(cur.kind); ++v) {
      Pass cand;
      const bool built = v != cur.variant;
      if (!built) {
        cand = cur;
      } else {
        s = build_pass(P, cur.kind, v, 1, cand);
        if (s == CP_EUNSUPPORTED) continue;
        if (s != CP_OK) return s;
      }
      for (int c : chunks) {
        if (!built && c == cur.chunk) continue;
        if (c == 0 && !kernel_flat_for(P.dtype, cur.kind, v)) continue;
        cand.chunk = c;
        double ms = 0.0;
        s = time_pass(P, cand, st, kReps, ms);
        if (s != CP_OK) {
          if (built && best.d_tiles != cand.d_tiles) cand.release();
          return s;
        }
        if (ms < best_ms) {
          if (best.d_tiles != cur.d_tiles && best.d_tiles != cand.d_tiles) best.release();
          best = cand;
          best_ms = ms;
        }
      }
      if (built && best.d_tiles != cand.d_tiles) cand.release();
    }
    if (best.d_tiles != cur.d_tiles) cur.release();
    best.ms = best_ms;
    cur = best;
  }
  P.tuned = true;
  return CP_OK;
}

// ---------------------------------------------------------------------------
// Tuning table: with CPCRIT_TUNE_CACHE naming a text file, every plan the
// autotuner times appends one line, and a later CP_BATCH_TUNE call (another
// process, or after cp_release) with the same shapes on the same kind of GPU
// takes the recorded choices instead of timing again.  Line format:
//   cpcrit-tune-1 <arch> <CUs> <n> <dtype> <flags> {<H> <W> <rs> <model*1000+nbins>}*n
//   | {<pass kind> <tile variant> <chunk> <ms>}*
// The last line with a matching key wins; unreadable lines are skipped.
// ---------------------------------------------------------------------------
std::string tune_key(int n, const Field* fs, uint32_t flags) {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "";
  std::ostringstream k;
  k << "cpcrit-tune-1 " << prop.gcnArchName << ' ' << prop.multiProcessorCount << ' ' << n << ' ' << fs[0].dtype
    << ' ' << (flags & (CP_BATCH_FWD | CP_BATCH_BWD));
  for (int i = 0; i < n; ++i) k << ' ' << fs[i].H << ' ' << fs[i].W << ' ' << fs[i].rs << ' ' << fs[i].model * 1000 + fs[i].nb;
  return k.str();
}

struct TunedPass {
  int kind, variant, chunk;
  double ms;
};

bool tune_table_lookup(const char* path, const std::string& key, std::vector<TunedPass>& out) {
  FILE* fh = std::fopen(path, "r");
  if (!fh) return false;
  std::string line;
  bool found = false;
  int c;
  while (true) {
    line.clear();
    while ((c = std::fgetc(fh)) != EOF && c != '\n') line.push_back((char)c);
    const size_t bar = line.find(" | ");
    if (bar != std::string::npos && line.compare(0, bar, key) == 0 && bar == key.size()) {
      std::istringstream rest(line.substr(bar + 3));
      std::vector<TunedPass> v;
      TunedPass t;
      while (rest >> t.kind >> t.variant >> t.chunk >> t.ms) v.push_back(t);
      if (!v.empty()) {
        out = v;
        found = true;
      }
    }
    if (c == EOF) break;
  }
  std::fclose(fh);
  return found;
}

void tune_table_store(const char* path, const std::string& key, const Plan& P) {
  FILE* fh = std::fopen(path, "a");
  if (!fh) return;
  std::string line = key + " |";
  char buf[96];
  for (const Pass& q : P.passes) {
    std::snprintf(buf, sizeof buf, " %d %d %d %.6f", q.kind, q.variant, q.chunk, q.ms);
    line += buf;
  }
  line += '\n';
  std::fputs(line.c_str(), fh);
  std::fclose(fh);
}

// Apply recorded choices to the plan; false (plan unchanged in its
// choices) when a recorded variant does not fit these fields any more.
cp_status_t tune_table_apply(Plan& P, const std::vector<TunedPass>& rec, bool& applied) {
  applied = false;
  for (const TunedPass& t : rec)
    if (t.kind < 0 || t.kind >= NPASS || t.variant < 0 || t.variant >= n_variants(t.kind) || t.chunk < 0 ||
        (t.chunk == 0 && !kernel_flat_for(P.dtype, t.kind, t.variant)))
      return CP_OK;
  for (Pass& cur : P.passes) {
    for (const TunedPass& t : rec) {
      if (t.kind != cur.kind) continue;
      if (t.variant != cur.variant) {
        Pass Q;
        cp_status_t s = build_pass(P, cur.kind, t.variant, t.chunk, Q);
        if (s == CP_EUNSUPPORTED) return CP_OK;
        if (s != CP_OK) return s;
        cur.release();
        cur = Q;
      }
      cur.chunk = t.chunk;
      cur.ms = t.ms;
    }
  }
  P.tuned = true;
  P.from_table = true;
  applied = true;
  return CP_OK;
}

std::string describe(const Plan& P) {
  const size_t el = P.dtype == CP_F64 ? 8 : 4;
  std::string out = P.tuned ? (P.passes.empty() || P.passes[0].ms >= 0.0 ? (P.from_table ? "tuned (table)" : "tuned")
                                                                           : "pinned")
                            : "default";
  char buf[256];
  for (const Pass& q : P.passes) {
    int ox, oy;
    pass_geom(q.kind, q.variant, el, ox, oy);
    if (q.chunk == 0)
      std::snprintf(buf, sizeof buf, "; %s: shape %d (tile %dx%d), one tile per block, %d tiles", pass_name(q.kind),
                    q.variant, ox, oy, q.ntiles);
    else
      std::snprintf(buf, sizeof buf, "; %s: shape %d (tile %dx%d), chunk %d, %d tiles, grid %d", pass_name(q.kind),
                    q.variant, ox, oy, q.chunk, q.ntiles, q.grid);
    out += buf;
    if (q.ms >= 0.0) {
      std::snprintf(buf, sizeof buf, ", %.4f ms", q.ms);
      out += buf;
    }
  }
  return out;
}

std::vector<int64_t> plan_key(int n, const Field* fs, uint32_t flags, int dev) {
  std::vector<int64_t> key;
  key.reserve(4 + 4 * (size_t)n);
  key.push_back(n);
  key.push_back(fs[0].dtype);
  key.push_back(flags & (CP_BATCH_FWD | CP_BATCH_BWD));
  key.push_back(dev);
  for (int i = 0; i < n; ++i) {
    key.push_back(fs[i].H);
    key.push_back(fs[i].W);
    key.push_back(fs[i].rs);
    key.push_back(fs[i].model * 1000 + fs[i].nb);
  }
  return key;
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
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CP_EDEVICE;
  const std::vector<int64_t> key = plan_key(n, fs, flags, dev);
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_plans.find(key);
  if (it == g_plans.end()) {
    auto P = std::make_unique<Plan>();
    cp_status_t s = build_plan(n, fs, bwd, *P, why);
    if (s != CP_OK) return s;
    it = g_plans.emplace(key, std::move(P)).first;
  }
  Plan& P = *it->second;
  hipStreamCaptureStatus capst = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &capst) != hipSuccess) return CP_EDEVICE;
  const bool capturing = capst != hipStreamCaptureStatusNone;
  // the plan's tile queues, field table and workspace may still be in use by
  // the last call on another stream: order this stream after it
  if (P.used && P.last != st) {
    if (capturing) {
      *why = "batched: the plan was last used on another stream; make an uncaptured call on this stream first";
      return CP_EINVAL;
    }
    if (hipStreamWaitEvent(st, P.done, 0) != hipSuccess) return CP_EDEVICE;
  }
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
  if ((flags & CP_BATCH_TUNE) && !P.tuned) {
    if (capturing) {
      *why = "batched: tuning times launches and cannot run while the stream is being captured";
      return CP_EINVAL;
    }
    const char* table = std::getenv("CPCRIT_TUNE_CACHE");
    const std::string tkey = table && *table ? tune_key(n, fs, flags) : std::string();
    std::vector<TunedPass> rec;
    bool applied = false;
    if (!tkey.empty() && tune_table_lookup(table, tkey, rec)) {
      cp_status_t s = tune_table_apply(P, rec, applied);
      if (s != CP_OK) {
        *why = "batched: rebuilding a recorded plan failed";
        return s;
      }
    }
    if (!applied) {
      cp_status_t s = tune(P, st);
      if (s != CP_OK) {
        *why = "batched: tuning launch failed";
        return s;
      }
      if (!tkey.empty()) tune_table_store(table, tkey, P);
    }
    P.drop_graph();  // captured with the default configuration
  }
  // every path below ends by marking the plan as used on st
  const auto used_on = [&]() -> cp_status_t {
    if (capturing) return CP_OK;
    if (hipEventRecord(P.done, st) != hipSuccess) return CP_EDEVICE;
    P.last = st;
    P.used = true;
    return CP_OK;
  };
  if (!(flags & CP_BATCH_GRAPH)) {
    if (launch(P, st) != hipSuccess) {
      *why = "batched: launch failed";
      return CP_EDEVICE;
    }
    return used_on();
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
  return used_on();
}

cp_status_t batched_pin(int n, const Field* fs, uint32_t flags, const int* shape, const int* chunk,
                        const char** why) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CP_EDEVICE;
  const std::vector<int64_t> key = plan_key(n, fs, flags, dev);
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_plans.find(key);
  if (it == g_plans.end()) {
    auto P = std::make_unique<Plan>();
    cp_status_t s = build_plan(n, fs, (flags & CP_BATCH_BWD) != 0, *P, why);
    if (s != CP_OK) return s;
    it = g_plans.emplace(key, std::move(P)).first;
  }
  Plan& P = *it->second;
  for (int q = 0; q < NPASS; ++q)
    if (shape[q] >= n_variants(q)) {
      *why = "batched pin: no such tile shape for this pass";
      return CP_EINVAL;
    }
  for (Pass& cur : P.passes) {
    const int v = shape[cur.kind] < 0 ? cur.variant : shape[cur.kind];
    // >= 1: tiles per claim; -1: one tile per block (chunk 0); else keep
    const int c = chunk[cur.kind] >= 1 ? chunk[cur.kind] : (chunk[cur.kind] == -1 ? 0 : cur.chunk);
    if (v == cur.variant) {
      cur.chunk = c;
    } else {
      Pass Q;
      cp_status_t s = build_pass(P, cur.kind, v, c, Q);
      if (s == CP_EUNSUPPORTED) *why = "batched pin: the tile shape does not fit a workgroup";
      if (s != CP_OK) return s;
      cur.release();
      cur = Q;
    }
    cur.ms = -1.0;
  }
  P.tuned = true;  // a pinned plan is not tuned over
  P.drop_graph();
  return CP_OK;
}

bool batched_describe(int n, const Field* fs, uint32_t flags, std::string& out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  const std::vector<int64_t> key = plan_key(n, fs, flags, dev);
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_plans.find(key);
  if (it == g_plans.end()) return false;
  out = describe(*it->second);
  return true;
}

void batched_release() {
  std::lock_guard<std::mutex> lk(g_mu);
  g_plans.clear();
}

}  // namespace cp
