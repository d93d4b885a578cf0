// cp_internal.hpp -- host-side declarations shared by the library's sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <string>

#include "cpcrit.h"

namespace cp {

constexpr int kMaxBins = 32;

// planes of the histogram adjoint's workspace ([5 h + 4][H][W]): the
// entries of the five stencil slots per bin, then one tail per neighbour
__host__ __device__ constexpr int64_t hist_ws_planes(int h) { return 5 * (int64_t)h + 4; }

// A validated field description (row_stride resolved).
struct Field {
  int H = 0, W = 0;
  int64_t rs = 0;  // row stride (elements)
  int model = 0, dtype = 0, nb = 0, ns = 0, est = 0;
  uint64_t seed = 0;
  uint32_t fid = 0;
  int64_t plane() const { return (int64_t)H * rs; }
};

int n_params(int model, int nb);

// closed-form models (uniform, Epanechnikov, histogram)
hipError_t cf_forward(const Field& f, const void* params, void* pmin, void* pmax, hipStream_t st);
// Device memory for the per-stencil partials of an adjoint: a caller-given
// region (ptr, bytes), or the library-owned workspace when ptr is null.
struct Scratch {
  void* ptr = nullptr;
  size_t bytes = 0;
};
// bytes of per-stencil partials the adjoint of field f passes through memory
// (0: the model's adjoint needs none)
size_t backward_scratch_bytes(const Field& f);
// the region an adjoint uses: the caller's (hipErrorInvalidValue if too
// small), else the library workspace of (device, st)
hipError_t adjoint_scratch(size_t bytes, hipStream_t st, const Scratch& scr, void** out);

hipError_t cf_backward(const Field& f, const void* params, const void* gmin, const void* gmax, void* grad,
                       hipStream_t st, const Scratch& scr = Scratch());

// classification (min, max, saddle, regular); any output may be null
hipError_t cf_classify(const Field& f, const void* params, void* pmin, void* pmax, void* psad, void* preg,
                       void* terms, hipStream_t st);

// semianalytical histogram estimator; any output may be null
hipError_t semi_forward(const Field& f, const void* params, void* pmin, void* pmax, void* terms, hipStream_t st);

// fitting from members
hipError_t fit_params(const Field& f, const void* members, int M, int ddof, double bw, double jitter,
                      double eps, void* params, hipStream_t st);
hipError_t fit_error_bound(const Field& f, const void* decompressed, double eb, void* params, hipStream_t st);
// fit + forward of a uniform / Epanechnikov field in one launch; applicable
// when width, row stride and both base addresses are multiples of 16 bytes
bool fit_forward_fusable(const Field& f, const void* members, const void* params);
hipError_t fit_forward_ue(const Field& f, const void* members, int M, double wscale, double eps, void* params,
                          void* pmin, void* pmax, hipStream_t st);

// Epanechnikov half-width bw * sd * M^(-1/5), Gaussian sigma = sd; both as
// wscale * sqrt(sum of squared deviations about the mean)
inline double fit_wscale(int model, int M, int ddof, double bw) {
  if (M - ddof <= 0) return 0.0;
  if (model == CP_GAUSSIAN) return 1.0 / std::sqrt((double)(M - ddof));
  return bw * std::pow((double)M, -0.2) / std::sqrt((double)(M - ddof));
}

// multivariate Gaussian
hipError_t mvg_forward(const Field& f, const double* params, float* pmin, float* pmax, hipStream_t st);
hipError_t mvg_backward(const Field& f, const double* params, const float* gmin, const float* gmax,
                        double* grad, hipStream_t st, const Scratch& scr = Scratch());
hipError_t philox_raw(int64_t n, const uint32_t* ctr, uint64_t seed, uint32_t* out, hipStream_t st);

// Library-owned device workspace (per-stencil adjoint partials) of the
// current device for work on stream st, grown on demand (a replaced buffer
// stays allocated until workspace_release, since a captured graph may still
// write it); the adjoints that gather through memory share it along one
// stream.
hipError_t workspace(size_t bytes, hipStream_t st, void** out);
void workspace_release();

// batched persistent launch
cp_status_t batched(int n, const Field* fields, const void* const* params, void* const* pmin,
                    void* const* pmax, const void* const* gmin, const void* const* gmax,
                    void* const* grad, uint32_t flags, hipStream_t st, const char** why);
// text description of the plan a batched call with these shapes and flags
// uses (false: no such plan yet)
bool batched_describe(int n, const Field* fields, uint32_t flags, std::string& out);
// fix tile shapes / chunks of a plan (index by pass kind; < 0: keep)
cp_status_t batched_pin(int n, const Field* fields, uint32_t flags, const int* shape, const int* chunk,
                        const char** why);
void batched_release();

// Gauss-Legendre tables (host copies)
bool gl_table(int n, double* x, double* w);

}  // namespace cp
