/*
 * cpcrit.h -- C ABI of the MI355X critical-point probability library.
 *
 * The library computes, for every vertex of a 2-D regular grid whose values
 * are random variables, the probability that the vertex is a local minimum
 * or a local maximum against its (up to) four axis neighbours (Athawale et
 * al., arXiv 2407.18015, Sec. 3 problem setting; Eq. 1 and Eq. 3 for the
 * minimum, Sec. 4.1.2 / 4.2 for the maximum by negation).  Vertex values are
 * independent (Sec. 3), so
 *
 *     P_min(v) = integral pdf_v(x) prod_n Pr(X_n > x) dx,
 *     P_max(v) = integral pdf_v(x) prod_n Pr(X_n < x) dx,
 *
 * evaluated exactly, piece by piece between the merged support breakpoints
 * (Sec. 4.1.1 Tasks 1-3), for the uniform and Epanechnikov models (Sec. 4.3)
 * and the histogram model (Sec. 4.4.1, Eq. 5).  A correlated multivariate
 * Gaussian over the 5-point stencil (the prior-work model of Sec. 5.2/5.3) is
 * estimated by Monte Carlo.  Gradients of the probabilities with respect to
 * the model parameters, fitting from ensemble members (Sec. 5.1-5.3) and a
 * batched entry point for many fields complete the interface.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array arguments are DEVICE pointers owned by the caller, on the
 *    current HIP device (the one `stream` belongs to); the library never
 *    frees or retains them.  Calls are asynchronous on
 *    `stream` (a hipStream_t; NULL = the null stream): results are ready
 *    once the caller synchronises that stream.
 *  - A field is H x W vertices.  Every plane (parameters, probabilities,
 *    upstream gradients, parameter gradients, members) is row-major with
 *    `row_stride` elements between rows (0 means W) and H * row_stride
 *    elements between consecutive planes of one array.
 *  - Vertex (y, x) has neighbours e = (y, x+1), n = (y-1, x), w = (y, x-1),
 *    s = (y+1, x).  Neighbours outside the grid are not part of the stencil
 *    (edge vertices have 3, corners 2, a 1x1 grid none, giving P = 1).
 *  - Element type of parameters, probabilities and gradients = desc->dtype,
 *    except the multivariate Gaussian, whose parameters and parameter
 *    gradients are always FP64 (see below) and whose probabilities are FP32.
 *  - Argument errors are reported synchronously through the return value
 *    and nothing is launched.  Per-vertex domain errors (lo >= hi, width <= 0,
 *    non-finite parameters, negative masses) produce NaN in that vertex's
 *    outputs; they are not reported through the status.
 *  - cp_last_error() returns a thread-local text for the last non-OK status.
 *
 * Parameter layouts ([n_param][H][row_stride])
 * --------------------------------------------
 *  CP_UNIFORM       2 planes: lo, hi                    pdf 1/(hi-lo) on [lo,hi]
 *  CP_EPANECHNIKOV  2 planes: m, w                      pdf 3/(4w)(1-((x-m)/w)^2)
 *                                                       on [m-w, m+w]
 *  CP_HISTOGRAM     2 + nbins planes: lo, hi, mass_0..  nbins equal-width bins on
 *                                                       [lo,hi]; pdf mass_j/Delta
 *  CP_GAUSSIAN      2 planes: mu, sigma                  independent N(mu, sigma^2)
 *                   (the parametric comparison model of Sec. 5.2).  No closed
 *                   form exists; the 1-D integrals are evaluated by a fixed
 *                   composite Gauss-Legendre rule on panels cut at multiples of
 *                   every sigma of the stencil, accurate to ~1e-8 (FP32) and
 *                   ~1e-14 (FP64) absolute.  Forward, classification and
 *                   adjoint; cp_prob_batched returns CP_EUNSUPPORTED.
 *  CP_MVGAUSS       16 FP64 planes: mean, then the packed lower-triangular
 *                   Cholesky factor L (row-major: L00, L10, L11, L20, ...,
 *                   L44) of the covariance of (e, n, w, s, v) at that vertex.
 *                   Rows/columns of absent neighbours are identity.
 */
#ifndef CPCRIT_H
#define CPCRIT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CP_OK = 0,
  CP_EINVAL = 1,       /* null pointer, bad size, bad enum, bad option */
  CP_EDOMAIN = 2,      /* invalid option value (e.g. n_members - ddof < 1) */
  CP_ENOMEM = 3,       /* the library could not allocate its own tables */
  CP_EDEVICE = 4,      /* a HIP call failed (launch, copy, graph) */
  CP_EUNSUPPORTED = 5  /* model x dtype x operation not provided */
} cp_status_t;

typedef enum {
  CP_UNIFORM = 0,
  CP_EPANECHNIKOV = 1,
  CP_HISTOGRAM = 2,
  CP_MVGAUSS = 3,  /* correlated Gaussian over the stencil, Monte Carlo */
  CP_GAUSSIAN = 4  /* independent Gaussian per vertex, deterministic quadrature */
} cp_model_t;
typedef enum { CP_F32 = 0, CP_F64 = 1 } cp_dtype_t;

/* Monte Carlo estimator of the multivariate Gaussian model */
typedef enum {
  CP_MC_CONDITIONAL = 0, /* mean over samples of Pr(vertex extreme | neighbours),
                            the vertex integrated in closed form (differentiable) */
  CP_MC_HIT = 1          /* fraction of samples in which the vertex is extreme */
} cp_mc_estimator_t;

typedef struct {
  int32_t height, width;
  int64_t row_stride; /* elements between rows; 0 = width */
  int32_t model;      /* cp_model_t */
  int32_t dtype;      /* cp_dtype_t */
  int32_t nbins;      /* CP_HISTOGRAM: bins per vertex, 1..32 */
  int32_t nsamples;   /* CP_MVGAUSS: samples per vertex, >= 1 */
  uint64_t seed;      /* CP_MVGAUSS: Philox key */
  uint32_t field_id;  /* CP_MVGAUSS: third Philox counter word */
  int32_t estimator;  /* CP_MVGAUSS: cp_mc_estimator_t */
} cp_field_desc_t;

typedef struct {
  int32_t ddof;          /* degrees of freedom removed from the std / covariance (1) */
  double bw_factor;      /* Epanechnikov half-width = bw_factor * std * M^(-1/5) (1.06) */
  double cov_jitter;     /* added to the covariance diagonal (1e-6) */
  double degenerate_eps; /* all members equal: lo/hi = x -/+ eps*max(1,|x|), Epanechnikov
                            w = eps*max(1,|m|); <= 0 selects 2^-20 (FP32) / 2^-30 (FP64) */
} cp_fit_opts_t;

/*
 * Fit the per-vertex model of desc->model from ensemble members
 * (Sec. 5.1 and 5.2: uniform range = member min/max; Epanechnikov from the
 * member mean and standard deviation; independent Gaussian: mu = mean,
 * sigma = std(ddof); Sec. 4.4: histogram with nbins bins
 * over the member range, mass = count / M, a member at relative position t
 * falls in bin floor(t * nbins) computed in desc->dtype, the maximum in the
 * last bin; Sec. 5.2/5.3: multivariate Gaussian from the member covariance of
 * the 5-point stencil, FP64 Cholesky).
 *   members  [n_members][H][row_stride], desc->dtype (FP32 for CP_MVGAUSS)
 *   params   output, layout of desc->model (above)
 *   opts     NULL selects the defaults in parentheses above
 */
cp_status_t cpu_fit_params(const cp_field_desc_t* desc, const void* members, int32_t n_members,
                           const cp_fit_opts_t* opts, void* params, void* stream);

/*
 * Fit followed by forward, as cpu_fit_params then cp_prob_forward with the
 * same arguments (results equal bit for bit): params, p_min and p_max are
 * all written.  For CP_UNIFORM and CP_EPANECHNIKOV fields whose width and
 * row stride are multiples of 16 bytes and whose members / params base
 * addresses are 16-byte aligned, one launch does both: each tile fits its
 * vertices and their one-vertex halo from the members into on-chip memory
 * and integrates from there, so the HBM-bound fit and the arithmetic-bound
 * forward overlap and the parameters are not read back.  Other fields run
 * the two calls' launches in order.
 *   members  [n_members][H][row_stride]; params [n_param][H][row_stride];
 *   p_min, p_max [H][row_stride]; opts as cpu_fit_params
 * Argument errors are those of the two calls.
 */
cp_status_t cp_fit_forward(const cp_field_desc_t* desc, const void* members, int32_t n_members,
                           const cp_fit_opts_t* opts, void* params, void* p_min, void* p_max, void* stream);

/*
 * Uniform model of a field reconstructed by an error-bounded lossy compressor
 * (Sec. 5.3, climate data): each vertex value lies in
 *     [d' - eb/2, d' + eb/2],
 * d' the decompressed value, and with no knowledge of the error distribution
 * it is modelled as uniform on that range.
 *   desc->model  CP_UNIFORM (else CP_EUNSUPPORTED)
 *   decompressed [H][row_stride], desc->dtype
 *   eb           the bound in data units (a relative bound is converted by the
 *                caller), > 0 and finite, else CP_EDOMAIN
 *   params       output [2][H][row_stride]: lo = d' - h, hi = d' + h with
 *                h = eb/2 rounded to desc->dtype, each end rounded once
 */
cp_status_t cp_fit_error_bound(const cp_field_desc_t* desc, const void* decompressed, double eb, void* params,
                               void* stream);

/*
 * Forward: P_min and P_max of every vertex (Eq. 3 and its negation).
 *   params  [n_param][H][row_stride] (layout above)
 *   p_min, p_max  [H][row_stride] outputs
 * CP_MVGAUSS: desc->estimator selects the estimator; sample i of vertex
 * (y, x) uses Philox4x32-10 counters (i, y*W+x, field_id, 0/1) under key
 * seed, so results do not depend on the launch configuration.
 */
cp_status_t cp_prob_forward(const cp_field_desc_t* desc, const void* params, void* p_min, void* p_max,
                            void* stream);

/*
 * Adjoint: grad_params[k][u] = sum over the stencils v that contain u of
 *   g_min(v) * dP_min(v)/dtheta_k(u) + g_max(v) * dP_max(v)/dtheta_k(u).
 * Parameters differentiated: uniform (lo, hi); Epanechnikov (m, w);
 * histogram masses, taken as free variables (no renormalisation; the lo/hi
 * planes of grad_params receive 0); independent Gaussian (mu, sigma), by
 * the forward's quadrature applied to the differentiated integrand (the
 * vertex's own slot through the translation and scale invariances of P);
 * multivariate Gaussian: mean plane
 * (gathered over stencils) and the Cholesky factor of each vertex, through
 * the conditional estimator (desc->estimator is ignored).
 * Contributions are gathered, not scattered: no atomics, and the result is
 * bit-reproducible.
 * The histogram and multivariate Gaussian adjoints pass per-stencil
 * partials through a library-owned device buffer, one per (device, stream),
 * allocated with hipMalloc on first use and replaced by a larger one when a
 * call needs more (the replaced buffer is kept, not freed, since a graph
 * captured from an earlier call may still write it); calls on different
 * streams never share one, and a stream being captured into a graph must
 * have made an uncaptured call of at least the same size first.
 * cp_release() frees all of them.
 *   g_min, g_max  [H][row_stride]; grad_params [n_param][H][row_stride]
 */
cp_status_t cp_prob_backward(const cp_field_desc_t* desc, const void* params, const void* g_min,
                             const void* g_max, void* grad_params, void* stream);

/*
 * cp_prob_backward without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, serving loops that must not call
 * hipMalloc, harnesses that forbid it.  Same arguments, kernels and results
 * (bit for bit) as cp_prob_backward.  The per-stencil partials of the
 * histogram and multivariate Gaussian adjoints go to one fixed device array
 * of 64 MiB per GPU (2^26 bytes; it exists on every GPU the library's code is
 * loaded on until the process ends), found on the first call on each device;
 * no call allocates, frees or grows device memory.
 *   Scratch needed: histogram (5 * nbins + 4) * H * W * sizeof(dtype) bytes,
 *   multivariate Gaussian 40 * H * W bytes, other models none.  A field that
 *   needs more than 64 MiB returns CP_EINVAL before anything is launched
 *   (cp_last_error gives both sizes).
 *   Every call on one GPU uses the same array: calls that may overlap in time
 *   on one GPU (on streams without ordering between them) race and must not
 *   be issued; calls ordered on one stream are safe.  Each call writes every
 *   scratch entry it later reads, so nothing needs clearing between calls.
 */
cp_status_t cp_prob_backward_noalloc(const cp_field_desc_t* desc, const void* params, const void* g_min,
                                     const void* g_max, void* grad_params, void* stream);

/*
 * Classification of every vertex into minimum, maximum, saddle or regular
 * point, for the closed-form models (uniform, Epanechnikov, histogram) and
 * the independent Gaussian.
 * Besides P_min and P_max (as cp_prob_forward), the saddle probability of
 * Eq. 2 (one dimension) / Eq. 4 (the 4-neighbour stencil): with independent
 * vertex values (Sec. 3) and S = 1 - CDF, F = CDF of a neighbour,
 *     t1 = Pr[X_v < X_e, X_v > X_n, X_v < X_w, X_v > X_s]
 *        = integral pdf_v(x) S_e(x) F_n(x) S_w(x) F_s(x) dx,
 *     t2 = Pr[X_v > X_e, X_v < X_n, X_v > X_w, X_v < X_s]
 *        = integral pdf_v(x) F_e(x) S_n(x) F_w(x) S_s(x) dx,
 *     P_saddle = t1 + t2,
 * integrated exactly over the pieces of [max(a_v, a of the F neighbours),
 * min(b_v, b of the S neighbours)] (Task 1 of Sec. 4.1.1 with mixed
 * factors; CP_GAUSSIAN: by the quadrature described with its layout), and
 * P_regular = 1 - P_min - P_max - P_saddle.  The saddle
 * pattern needs all four neighbours, so P_saddle = 0 on the grid boundary.
 *   params     [n_param][H][row_stride]
 *   p_min, p_max, p_saddle, p_regular  [H][row_stride] outputs
 *   terms      [2][H][row_stride] output: t1, t2
 * Every output pointer may be NULL (then it is not written); at least one
 * must be given.  A vertex with an invalid distribution in its stencil gets
 * NaN in every output.  CP_MVGAUSS: CP_EUNSUPPORTED.
 */
cp_status_t cp_prob_classify(const cp_field_desc_t* desc, const void* params, void* p_min, void* p_max,
                             void* p_saddle, void* p_regular, void* terms, void* stream);

/*
 * Semianalytical histogram estimator (Sec. 4.4.2): desc->nsamples samples c
 * are drawn from each vertex histogram by its inverse CDF; for each sample the
 * probabilities that the neighbours lie above / below it are closed-form
 * (bin lookup plus cumulative masses), and their products are averaged:
 *     P_min ~ T (1/c) sum_i prod_n S_n(x_i),  P_max ~ T (1/c) sum_i prod_n F_n(x_i),
 *     t1, t2 (Eq. 4) likewise with mixed S / F factors (0 on the boundary),
 * T = the vertex's total mass, so the expectation is the closed-form value of
 * cp_prob_forward / cp_prob_classify.  Sample i of vertex (y, x) uses word
 * i mod 4 of Philox4x32-10 with counter (i / 4, y*W + x, desc->field_id, 2)
 * under key desc->seed; u = ((word >> 8) + 1/2) 2^-24, r = u T, bin
 * j = #{k in 1..h-1 : m_0 + ... + m_{k-1} <= r}, x = lo + Delta (j + f) with
 * f = (r - m_0 - ... - m_{j-1}) / m_j clamped to [0, 1] (0 for an empty bin).
 *   desc->model   CP_HISTOGRAM (else CP_EUNSUPPORTED); desc->nsamples >= 1
 *   params        [2 + nbins][H][row_stride]
 *   p_min, p_max  [H][row_stride] outputs; terms [2][H][row_stride] (t1, t2)
 * Any output may be NULL; at least one must be given.  Invalid histograms in
 * a stencil give NaN in its outputs.
 */
cp_status_t cp_prob_semianalytical(const cp_field_desc_t* desc, const void* params, void* p_min, void* p_max,
                                   void* terms, void* stream);

/* cp_prob_batched flags */
#define CP_BATCH_FWD 1u       /* write p_min / p_max */
#define CP_BATCH_BWD 2u       /* write grad_params (needs g_min / g_max) */
#define CP_BATCH_GRAPH 4u     /* replay a cached HIP graph of the plan's launches */
#define CP_BATCH_PER_FIELD 8u /* reference mode: one forward / backward launch per field */
#define CP_BATCH_TUNE 16u     /* autotune the plan's tile shapes and claim chunks (first call) */

/*
 * Many independent fields (mixed sizes, closed-form models, one dtype) in one
 * launch per pass over a device-side table of field descriptors and tiles
 * (one tile per block, or a persistent grid claiming tiles from a queue).
 * Arrays of n pointers index the fields; p_min/p_max may be NULL unless
 * CP_BATCH_FWD, g_min/g_max/grad_params unless CP_BATCH_BWD.  Results equal
 * those of cp_prob_forward / cp_prob_backward on each field.  The graph cache
 * is keyed by the field shapes; each call refreshes the descriptor table
 * (pointers may change between calls).  Calls with the same shapes share one
 * plan, including its device-side tile queue and histogram workspace: a call
 * on another stream than the plan's last uncaptured call is ordered after
 * that call on the device (a stream wait), and such a call while its stream
 * is being captured into a graph returns CP_EINVAL; replays of graphs that
 * the caller captured must not overlap other calls with the same shapes.
 * Gaussian fields (CP_MVGAUSS, CP_GAUSSIAN) are not accepted here
 * (CP_EUNSUPPORTED).
 * CP_BATCH_TUNE: the first call with these shapes and flags times, for every
 * pass of the plan, each tile shape the library offers (uniform /
 * Epanechnikov forward: 64 x 4, 64 x 8 or 64 x 16 vertices; histogram
 * passes: 64 x 4 or 64 x 8; uniform / Epanechnikov adjoint: FP32 30x30,
 * 14x14 or 62x30 outputs, FP64 14x14, 30x14 or 30x30)
 * with each claim chunk (1, 2, 4, 8 tiles) of the persistent launch and with
 * one tile per block (a grid of all the pass's tiles, most expensive first),
 * on the caller's own buffers, and keeps the fastest for every later call;
 * the call then blocks until the trials are done, and fails (CP_EINVAL)
 * while the stream is being captured.  The trials write the outputs, with
 * the same values: no tile shape or launch form changes a result.  Without
 * the flag a plan uses the first shape and one tile per block.
 * Tuning table: if the environment variable CPCRIT_TUNE_CACHE names a file,
 * every plan the tuner times appends its choices there (one text line keyed
 * by the GPU architecture, its CU count and the field shapes), and a later
 * CP_BATCH_TUNE call with the same key (in any process) takes them instead
 * of timing; cp_batched_describe then reports "tuned (table)".
 */
cp_status_t cp_prob_batched(int32_t n, const cp_field_desc_t* descs, const void* const* params,
                            void* const* p_min, void* const* p_max, const void* const* g_min,
                            const void* const* g_max, void* const* grad_params, uint32_t flags,
                            void* stream);

/* Passes of a batched plan (index of the arrays of cp_batched_pin). */
typedef enum {
  CP_PASS_FORWARD = 0,        /* uniform / Epanechnikov forward */
  CP_PASS_HIST_FORWARD = 1,   /* histogram forward */
  CP_PASS_ADJOINT = 2,        /* uniform / Epanechnikov adjoint */
  CP_PASS_HIST_ADJOINT = 3,   /* histogram adjoint sweep (per-stencil Jacobians) */
  CP_PASS_HIST_GATHER = 4,    /* histogram adjoint gather */
  CP_NUM_PASSES = 5
} cp_batch_pass_t;

/*
 * Fix the tile shape and claim chunk of each pass of the plan that
 * cp_prob_batched uses for these descriptors and flags (building the plan if
 * no call has yet): shape[p] indexes the shapes listed under CP_BATCH_TUNE
 * for pass p (0 = the default), chunk[p] >= 1 tiles per claim of the
 * persistent launch or -1 for one tile per block; entries < 0 (shape) or of
 * any other value (chunk) keep the current choice, entries of passes the
 * plan lacks are ignored.  For callers that tuned offline and want the result
 * without timing, or that want one shape.  A pinned plan is not re-tuned.
 * CP_EINVAL: a shape index out of range; CP_EUNSUPPORTED: the shape does not
 * fit a workgroup for these fields.
 */
cp_status_t cp_batched_pin(int32_t n, const cp_field_desc_t* descs, uint32_t flags, const int32_t* shape,
                           const int32_t* chunk);

/*
 * The plan a cp_prob_batched call with these descriptors and flags uses, as
 * text: "tuned", "pinned" or "default", then per pass its shape index and
 * tile, claim chunk and resident grid (or "one tile per block"), tile count
 * and (tuned) launch time.  Returns NULL when no
 * call has built that plan yet.  The string is thread-local, valid until
 * the next call of this function on the thread.
 */
const char* cp_batched_describe(int32_t n, const cp_field_desc_t* descs, uint32_t flags);

/* Number of parameter planes of a model (histogram: 2 + nbins; Gaussian: 16). */
int32_t cp_n_params(int32_t model, int32_t nbins);

/* Text for a status code (static storage). */
const char* cp_status_string(cp_status_t status);

/* Thread-local description of the last non-OK status of this thread. */
const char* cp_last_error(void);

/* Free the library's own device tables, adjoint buffers and cached graphs
 * (optional); no call may be running on any stream. */
cp_status_t cp_release(void);

/*
 * Raw Philox4x32-10 words for n counters on the device (the generator the
 * Gaussian path uses): counters [n][4] uint32, out [n][4] uint32, key = seed.
 */
cp_status_t cp_philox4x32_10(int64_t n, const uint32_t* counters, uint64_t seed, uint32_t* out,
                             void* stream);

/*
 * Gauss-Legendre rule the closed-form kernels use for an n-point piece
 * (n in {1, 2, 3, 4, 5, 6, 7, 8, 10}): host copies of the device tables, for checking.
 * Returns CP_EINVAL for other n.
 */
cp_status_t cp_gauss_legendre(int32_t n, double* nodes, double* weights);

#ifdef __cplusplus
}
#endif

#endif /* CPCRIT_H */
