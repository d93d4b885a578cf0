// cp_api.cpp -- the extern "C" entry points of include/cpcrit.h: argument
// validation, option defaults and dispatch to the kernels.  Nothing here
// computes probabilities; every step runs on the device.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "cp_internal.hpp"
#include "cp_workspace.hpp"
#include "cpcrit.h"

namespace {

thread_local std::string g_last;

cp_status_t fail(cp_status_t s, const char* msg) {
  g_last = msg ? msg : "";
  return s;
}

cp_status_t device_fail(hipError_t e, const char* what) {
  g_last = std::string(what) + ": " + hipGetErrorString(e);
  return CP_EDEVICE;
}

// `sampling`: the call draws Monte Carlo samples (forward / backward of the
// Gaussian model); the fit does not use nsamples / estimator.
cp_status_t check_desc(const cp_field_desc_t* d, cp::Field& f, bool sampling = true) {
  if (!d) return fail(CP_EINVAL, "descriptor is NULL");
  if (d->height < 1 || d->width < 1) return fail(CP_EINVAL, "height and width must be >= 1");
  if (d->model < CP_UNIFORM || d->model > CP_GAUSSIAN) return fail(CP_EINVAL, "unknown model");
  if (d->dtype != CP_F32 && d->dtype != CP_F64) return fail(CP_EINVAL, "unknown dtype");
  const int64_t rs = d->row_stride == 0 ? d->width : d->row_stride;
  if (rs < d->width) return fail(CP_EINVAL, "row_stride is smaller than width");
  if ((int64_t)d->height * d->width > (int64_t)INT_MAX / 2) return fail(CP_EINVAL, "grid too large");
  if (d->model == CP_HISTOGRAM && (d->nbins < 1 || d->nbins > cp::kMaxBins))
    return fail(CP_EINVAL, "nbins must be in 1..32");
  if (d->model == CP_MVGAUSS) {
    if (d->dtype != CP_F32) return fail(CP_EUNSUPPORTED, "the Gaussian model samples in FP32 only");
    if (sampling && d->nsamples < 1) return fail(CP_EINVAL, "nsamples must be >= 1");
    if (sampling && d->estimator != CP_MC_CONDITIONAL && d->estimator != CP_MC_HIT)
      return fail(CP_EINVAL, "unknown estimator");
  }
  f.H = d->height;
  f.W = d->width;
  f.rs = rs;
  f.model = d->model;
  f.dtype = d->dtype;
  f.nb = d->model == CP_HISTOGRAM ? d->nbins : 0;
  f.ns = d->nsamples;
  f.est = d->estimator;
  f.seed = d->seed;
  f.fid = d->field_id;
  const int64_t np = cp::n_params(f.model, f.nb);
  if (f.plane() > INT64_MAX / (np > 0 ? np : 1)) return fail(CP_EINVAL, "grid too large");
  return CP_OK;
}

// Fit options with their defaults filled in; eps = the degenerate half-width
// scale in effect.
cp_status_t check_fit_opts(const cp::Field& f, int32_t n_members, const cp_fit_opts_t* opts, cp_fit_opts_t& o,
                           double& eps) {
  if (n_members < 1) return fail(CP_EINVAL, "n_members must be >= 1");
  o = cp_fit_opts_t{1, 1.06, 1e-6, 0.0};
  if (opts) o = *opts;
  if (o.ddof < 0) return fail(CP_EDOMAIN, "ddof must be >= 0");
  if (!(o.bw_factor > 0.0)) return fail(CP_EDOMAIN, "bw_factor must be > 0");
  if (!(o.cov_jitter >= 0.0)) return fail(CP_EDOMAIN, "cov_jitter must be >= 0");
  eps = o.degenerate_eps > 0.0 ? o.degenerate_eps : (f.dtype == CP_F64 ? 0x1p-30 : 0x1p-20);
  if ((f.model == CP_EPANECHNIKOV || f.model == CP_GAUSSIAN) && n_members > 1 && n_members - o.ddof < 1)
    return fail(CP_EDOMAIN, "n_members - ddof must be >= 1");
  if (f.model == CP_MVGAUSS && (n_members < 2 || n_members - o.ddof < 1))
    return fail(CP_EDOMAIN, "the Gaussian fit needs n_members >= 2 and n_members - ddof >= 1");
  return CP_OK;
}

}  // namespace

namespace cp {
int n_params(int model, int nb) {
  if (model == CP_HISTOGRAM) return 2 + nb;
  if (model == CP_MVGAUSS) return 16;
  return 2;
}

namespace {
int ws_alloc(void** out, size_t bytes) { return (int)hipMalloc(out, bytes); }
void ws_free(int dev, void* p) {
  (void)hipSetDevice(dev);
  (void)hipFree(p);
}
const PoolOps kWsOps{ws_alloc, ws_free};
WorkspacePool g_ws;
}  // namespace

hipError_t workspace(size_t bytes, hipStream_t st, void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  return (hipError_t)g_ws.get(dev, st, bytes, kWsOps, out);
}

void workspace_release() {
  int cur = 0;
  const bool have = hipGetDevice(&cur) == hipSuccess;
  g_ws.release(kWsOps);
  if (have) (void)hipSetDevice(cur);
}

size_t backward_scratch_bytes(const Field& f) {
  const size_t nv = (size_t)f.H * (size_t)f.W;
  if (f.model == CP_HISTOGRAM) return (f.dtype == CP_F64 ? 8 : 4) * (size_t)hist_ws_planes(f.nb) * nv;
  if (f.model == CP_MVGAUSS) return sizeof(double) * 5 * nv;
  return 0;
}

hipError_t adjoint_scratch(size_t bytes, hipStream_t st, const Scratch& scr, void** out) {
  if (!scr.ptr) return workspace(bytes, st, out);
  if (bytes > scr.bytes) return hipErrorInvalidValue;
  *out = scr.ptr;
  return hipSuccess;
}
}  // namespace cp

// ---------------------------------------------------------------------------
// Fixed adjoint scratch for cp_prob_backward_noalloc: a device array that
// exists on every GPU the library's code is loaded on, for the life of the
// process.  Host code must not pass `scratch` itself to a kernel (on the host
// it names a stand-in, not device memory): its device address is looked up
// once per device with hipGetSymbolAddress and kept in g_noalloc_ptr.
// ---------------------------------------------------------------------------
namespace {
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kNoAllocMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kNoAllocMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call there).
hipError_t noalloc_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_noalloc_ptr[dev] = p;
  }
  *out = g_noalloc_ptr[dev];
  return hipSuccess;
}
}  // namespace

extern "C" {

int32_t cp_n_params(int32_t model, int32_t nbins) {
  if (model < CP_UNIFORM || model > CP_GAUSSIAN) return -1;
  if (model == CP_HISTOGRAM && (nbins < 1 || nbins > cp::kMaxBins)) return -1;
  return cp::n_params(model, nbins);
}

const char* cp_status_string(cp_status_t s) {
  switch (s) {
    case CP_OK:
      return "ok";
    case CP_EINVAL:
      return "invalid argument";
    case CP_EDOMAIN:
      return "invalid option value";
    case CP_ENOMEM:
      return "out of device memory";
    case CP_EDEVICE:
      return "HIP call failed";
    case CP_EUNSUPPORTED:
      return "unsupported combination";
  }
  return "unknown status";
}

const char* cp_last_error(void) { return g_last.c_str(); }

cp_status_t cpu_fit_params(const cp_field_desc_t* desc, const void* members, int32_t n_members,
                           const cp_fit_opts_t* opts, void* params, void* stream) {
  cp::Field f;
  cp_status_t s = check_desc(desc, f, false);
  if (s != CP_OK) return s;
  if (!members || !params) return fail(CP_EINVAL, "members / params is NULL");
  cp_fit_opts_t o;
  double eps;
  s = check_fit_opts(f, n_members, opts, o, eps);
  if (s != CP_OK) return s;
  hipError_t e = cp::fit_params(f, members, n_members, o.ddof, o.bw_factor, o.cov_jitter, eps, params,
                                static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "fit launch");
  return CP_OK;
}

cp_status_t cp_fit_forward(const cp_field_desc_t* desc, const void* members, int32_t n_members,
                           const cp_fit_opts_t* opts, void* params, void* p_min, void* p_max, void* stream) {
  cp::Field f;
  cp_status_t s = check_desc(desc, f);
  if (s != CP_OK) return s;
  if (!members || !params || !p_min || !p_max) return fail(CP_EINVAL, "members / params / p_min / p_max is NULL");
  cp_fit_opts_t o;
  double eps;
  s = check_fit_opts(f, n_members, opts, o, eps);
  if (s != CP_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (cp::fit_forward_fusable(f, members, params)) {
    e = cp::fit_forward_ue(f, members, n_members, cp::fit_wscale(f.model, n_members, o.ddof, o.bw_factor), eps,
                           params, p_min, p_max, st);
    if (e != hipSuccess) return device_fail(e, "fit + forward launch");
    return CP_OK;
  }
  e = cp::fit_params(f, members, n_members, o.ddof, o.bw_factor, o.cov_jitter, eps, params, st);
  if (e != hipSuccess) return device_fail(e, "fit launch");
  if (f.model == CP_MVGAUSS)
    e = cp::mvg_forward(f, static_cast<const double*>(params), static_cast<float*>(p_min),
                        static_cast<float*>(p_max), st);
  else
    e = cp::cf_forward(f, params, p_min, p_max, st);
  if (e != hipSuccess) return device_fail(e, "forward launch");
  return CP_OK;
}

cp_status_t cp_fit_error_bound(const cp_field_desc_t* desc, const void* decompressed, double eb, void* params,
                               void* stream) {
  cp::Field f;
  cp_status_t s = check_desc(desc, f, false);
  if (s != CP_OK) return s;
  if (f.model != CP_UNIFORM) return fail(CP_EUNSUPPORTED, "error-bound fit: the model is uniform");
  if (!decompressed || !params) return fail(CP_EINVAL, "decompressed / params is NULL");
  if (!(eb > 0.0) || !(eb < 1e300)) return fail(CP_EDOMAIN, "eb must be positive and finite");
  if (f.dtype == CP_F32 && !((float)(eb * 0.5) > 0.0f && (float)(eb * 0.5) < 3.0e38f))
    return fail(CP_EDOMAIN, "eb / 2 is not a positive finite FP32 value");
  hipError_t e = cp::fit_error_bound(f, decompressed, eb, params, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "error-bound fit launch");
  return CP_OK;
}

cp_status_t cp_prob_forward(const cp_field_desc_t* desc, const void* params, void* p_min, void* p_max,
                            void* stream) {
  cp::Field f;
  cp_status_t s = check_desc(desc, f);
  if (s != CP_OK) return s;
  if (!params || !p_min || !p_max) return fail(CP_EINVAL, "params / p_min / p_max is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (f.model == CP_MVGAUSS)
    e = cp::mvg_forward(f, static_cast<const double*>(params), static_cast<float*>(p_min),
                        static_cast<float*>(p_max), st);
  else
    e = cp::cf_forward(f, params, p_min, p_max, st);
  if (e != hipSuccess) return device_fail(e, "forward launch");
  return CP_OK;
}

cp_status_t cp_prob_backward(const cp_field_desc_t* desc, const void* params, const void* g_min,
                             const void* g_max, void* grad_params, void* stream) {
  cp::Field f;
  cp_status_t s = check_desc(desc, f);
  if (s != CP_OK) return s;
  if (!params || !g_min || !g_max || !grad_params) return fail(CP_EINVAL, "a backward argument is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (f.model == CP_MVGAUSS)
    e = cp::mvg_backward(f, static_cast<const double*>(params), static_cast<const float*>(g_min),
                         static_cast<const float*>(g_max), static_cast<double*>(grad_params), st);
  else
    e = cp::cf_backward(f, params, g_min, g_max, grad_params, st);
  if (e == hipErrorInvalidValue && f.model == CP_HISTOGRAM)
    return fail(CP_EUNSUPPORTED, "histogram adjoint: too many bins for this dtype's LDS budget");
  if (e != hipSuccess) return device_fail(e, "backward launch");
  return CP_OK;
}

cp_status_t cp_prob_backward_noalloc(const cp_field_desc_t* desc, const void* params, const void* g_min,
                                     const void* g_max, void* grad_params, void* stream) {
  cp::Field f;
  cp_status_t s = check_desc(desc, f);
  if (s != CP_OK) return s;
  if (!params || !g_min || !g_max || !grad_params) return fail(CP_EINVAL, "a backward argument is NULL");
  const size_t need = cp::backward_scratch_bytes(f);
  if (need > kNoAllocScratchBytes) {
    char msg[160];
    std::snprintf(msg, sizeof msg, "allocation-free adjoint: this field needs %zu bytes of scratch, the fixed "
                  "array holds %zu", need, kNoAllocScratchBytes);
    return fail(CP_EINVAL, msg);
  }
  void* ptr = nullptr;
  hipError_t e = noalloc_scratch(&ptr);
  if (e != hipSuccess) return device_fail(e, "scratch symbol lookup");
  const cp::Scratch scr{ptr, kNoAllocScratchBytes};
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (f.model == CP_MVGAUSS)
    e = cp::mvg_backward(f, static_cast<const double*>(params), static_cast<const float*>(g_min),
                         static_cast<const float*>(g_max), static_cast<double*>(grad_params), st, scr);
  else
    e = cp::cf_backward(f, params, g_min, g_max, grad_params, st, scr);
  if (e == hipErrorInvalidValue && f.model == CP_HISTOGRAM)
    return fail(CP_EUNSUPPORTED, "histogram adjoint: too many bins for this dtype's LDS budget");
  if (e != hipSuccess) return device_fail(e, "backward launch");
  return CP_OK;
}

cp_status_t cp_prob_classify(const cp_field_desc_t* desc, const void* params, void* p_min, void* p_max,
                             void* p_saddle, void* p_regular, void* terms, void* stream) {
  cp::Field f;
  cp_status_t s = check_desc(desc, f, false);
  if (s != CP_OK) return s;
  if (f.model == CP_MVGAUSS) return fail(CP_EUNSUPPORTED, "classify: closed-form models only");
  if (!params) return fail(CP_EINVAL, "params is NULL");
  if (!p_min && !p_max && !p_saddle && !p_regular && !terms) return fail(CP_EINVAL, "no output requested");
  hipError_t e = cp::cf_classify(f, params, p_min, p_max, p_saddle, p_regular, terms,
                                 static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "classify launch");
  return CP_OK;
}

cp_status_t cp_prob_semianalytical(const cp_field_desc_t* desc, const void* params, void* p_min, void* p_max,
                                   void* terms, void* stream) {
  cp::Field f;
  cp_status_t s = check_desc(desc, f, false);
  if (s != CP_OK) return s;
  if (f.model != CP_HISTOGRAM) return fail(CP_EUNSUPPORTED, "semianalytical: histogram model only");
  if (desc->nsamples < 1) return fail(CP_EINVAL, "nsamples must be >= 1");
  if (!params) return fail(CP_EINVAL, "params is NULL");
  if (!p_min && !p_max && !terms) return fail(CP_EINVAL, "no output requested");
  hipError_t e = cp::semi_forward(f, params, p_min, p_max, terms, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "semianalytical launch");
  return CP_OK;
}

cp_status_t cp_prob_batched(int32_t n, const cp_field_desc_t* descs, const void* const* params, void* const* p_min,
                            void* const* p_max, const void* const* g_min, const void* const* g_max,
                            void* const* grad_params, uint32_t flags, void* stream) {
  if (n < 1 || !descs || !params) return fail(CP_EINVAL, "n < 1 or descs / params is NULL");
  const bool fwd = flags & CP_BATCH_FWD, bwd = flags & CP_BATCH_BWD;
  if (!fwd && !bwd) return fail(CP_EINVAL, "flags select neither forward nor backward");
  if (flags & ~(CP_BATCH_FWD | CP_BATCH_BWD | CP_BATCH_GRAPH | CP_BATCH_PER_FIELD | CP_BATCH_TUNE))
    return fail(CP_EINVAL, "unknown flag bits");
  if (fwd && (!p_min || !p_max)) return fail(CP_EINVAL, "p_min / p_max arrays are NULL");
  if (bwd && (!g_min || !g_max || !grad_params)) return fail(CP_EINVAL, "backward arrays are NULL");
  std::vector<cp::Field> fs(n);
  for (int i = 0; i < n; ++i) {
    cp_status_t s = check_desc(&descs[i], fs[i]);
    if (s != CP_OK) return s;
    if (fs[i].model == CP_MVGAUSS || fs[i].model == CP_GAUSSIAN)
      return fail(CP_EUNSUPPORTED, "batched: Gaussian fields are not accepted");
    if (fs[i].dtype != fs[0].dtype) return fail(CP_EINVAL, "batched: all fields must share one dtype");
    if (!params[i] || (fwd && (!p_min[i] || !p_max[i])) ||
        (bwd && (!g_min[i] || !g_max[i] || !grad_params[i])))
      return fail(CP_EINVAL, "batched: a field pointer is NULL");
  }
  const char* why = "batched call failed";
  cp_status_t s = cp::batched(n, fs.data(), params, p_min, p_max, g_min, g_max, grad_params, flags,
                              static_cast<hipStream_t>(stream), &why);
  if (s != CP_OK) return fail(s, why);
  return CP_OK;
}

cp_status_t cp_batched_pin(int32_t n, const cp_field_desc_t* descs, uint32_t flags, const int32_t* shape,
                           const int32_t* chunk) {
  if (n < 1 || !descs || !shape || !chunk) return fail(CP_EINVAL, "n < 1 or a NULL array");
  if (!(flags & (CP_BATCH_FWD | CP_BATCH_BWD))) return fail(CP_EINVAL, "flags select neither forward nor backward");
  std::vector<cp::Field> fs(n);
  for (int i = 0; i < n; ++i) {
    cp_status_t s = check_desc(&descs[i], fs[i]);
    if (s != CP_OK) return s;
    if (fs[i].model == CP_MVGAUSS || fs[i].model == CP_GAUSSIAN)
      return fail(CP_EUNSUPPORTED, "batched: Gaussian fields are not accepted");
    if (fs[i].dtype != fs[0].dtype) return fail(CP_EINVAL, "batched: all fields must share one dtype");
  }
  int sh[CP_NUM_PASSES], ch[CP_NUM_PASSES];
  for (int q = 0; q < CP_NUM_PASSES; ++q) {
    sh[q] = shape[q];
    ch[q] = chunk[q];
  }
  const char* why = "batched pin failed";
  cp_status_t s = cp::batched_pin(n, fs.data(), flags, sh, ch, &why);
  if (s != CP_OK) return fail(s, why);
  return CP_OK;
}

const char* cp_batched_describe(int32_t n, const cp_field_desc_t* descs, uint32_t flags) {
  static thread_local std::string text;
  if (n < 1 || !descs) return nullptr;
  std::vector<cp::Field> fs(n);
  for (int i = 0; i < n; ++i)
    if (check_desc(&descs[i], fs[i]) != CP_OK) return nullptr;
  if (!cp::batched_describe(n, fs.data(), flags, text)) return nullptr;
  return text.c_str();
}

cp_status_t cp_release(void) {
  cp::batched_release();
  cp::workspace_release();
  return CP_OK;
}

cp_status_t cp_philox4x32_10(int64_t n, const uint32_t* counters, uint64_t seed, uint32_t* out, void* stream) {
  if (n < 0 || (n > 0 && (!counters || !out))) return fail(CP_EINVAL, "bad philox arguments");
  hipError_t e = cp::philox_raw(n, counters, seed, out, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return device_fail(e, "philox launch");
  return CP_OK;
}

cp_status_t cp_gauss_legendre(int32_t n, double* nodes, double* weights) {
  if (!nodes || !weights) return fail(CP_EINVAL, "NULL output");
  if (!cp::gl_table(n, nodes, weights)) return fail(CP_EINVAL, "no rule with that many nodes");
  return CP_OK;
}

}  // extern "C"
