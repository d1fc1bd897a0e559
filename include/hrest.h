/*
 * hrest.h -- C ABI of the MI355X (gfx950) library that estimates gradients,
 * Hessians and Hessian-vector products of a Gaussian-smoothed rendering loss
 * by importance-sampled Monte Carlo, and takes Newton-CG steps with them.
 *
 * Method: Z. Wang, M. Fischer, T. Ritschel, "Stochastic Gradient Estimation
 * for Higher-order Differentiable Rendering", ICCV 2025 (arXiv 2412.03489).
 *   - problem statement and smoothing by convolution: section "Our approach",
 *     "Background" (D S R = integral of D kappa(tau) R(theta - tau));
 *   - gradient kernel and its lobe sampler: section "Gradients";
 *   - Hessian kernel, diagonal CDF and off-diagonal product sampler:
 *     section "Hessians";
 *   - Hessian-vector product by central differences of gradient estimators:
 *     section "Hessian-vector product";
 *   - aggregate importance sampling and the evaluation-count table:
 *     section "Aggregate";
 *   - Newton-CG with Fletcher-Reeves and trust truncation: section
 *     "Previous Work", and the appendix on non-PSD Hessians;
 *   - antithetic pairs: appendix "Hyperparameters".
 *
 * Conventions (every entry point):
 *   - returns hr_status: 0 on success, negative on failure; no C++ exception
 *     crosses the ABI; hr_last_error() returns a thread-local message for the
 *     last failure on the calling thread;
 *   - "host" pointers are plain CPU memory owned by the caller and never
 *     retained after the call returns; "_dev" entry points take device
 *     pointers (HBM of the context's GPU), owned by the caller, and enqueue
 *     their work asynchronously on the context's stream;
 *   - all parameter vectors are FP64; images are FP32, row-major
 *     (y, x, channel), y pointing down;
 *   - theta layout of a disk scene: per disk (cx, cy) or (cx, cy, r),
 *     interleaved, in image-normalised coordinates; of a path-traced scene:
 *     (light centre x, y, z, sphere-0 centre x, y, z);
 *   - estimates use N draws tau_s, s = 0..N-1, from one Philox4x32-10 stream
 *     keyed by `seed`; with antithetic pairs every draw is rendered at
 *     theta - tau and theta + tau.  Results at N' < N are the estimates over
 *     the first N' draws (counter-based random numbers).
 *   - invalid input (sigma <= 0 or non-finite, N == 0 or N >= 2^32, non-finite
 *     theta or v, NULL pointers, unsupported option) returns HR_EINVAL and
 *     writes nothing; a request larger than the context's memory budget
 *     returns HR_ENOMEM; a HIP runtime failure returns HR_EDEVICE.
 */
#ifndef HREST_H
#define HREST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HR_OK = 0,
  HR_EINVAL = -1,
  HR_ENOMEM = -2,
  HR_EDEVICE = -3,
  HR_EUNSUPPORTED = -4,
  HR_EBUSY = -5,          /* nothing completed within the wait's time limit, or
                             another thread already waits on the ticket       */
} hr_status;

/* Sampler (section "Aggregate", table of evaluations per draw).
 *   HR_AIS  : aggregate importance sampling -- draw the element uniformly, draw
 *             tau from that element's lobe density, weight every element by
 *             d_m(tau) / q(tau) with q the mixture of all element densities;
 *             one render per draw.
 *   HR_IS   : per-element importance sampling, one stream of N draws per
 *             element (K renders per draw), weight sgn(d_m) Z_m.
 *   HR_GAUSS: plain Gaussian draws, weight d_m(tau) ("no IS" column).
 *   HR_FR22 : comparator of the gradient-derivation appendix: per-element
 *             streams like HR_IS but only the differentiated dimension is
 *             blurred (all other components of tau are 0); gradient and HVP
 *             only (HR_EUNSUPPORTED for Hessians). */
typedef enum { HR_AIS = 0, HR_IS = 1, HR_GAUSS = 2, HR_FR22 = 3 } hr_sampler;

typedef struct hr_ctx hr_ctx;      /* one per GPU: stream, workspace, timers   */
typedef struct hr_scene hr_scene;  /* device-resident scene and target image   */

typedef struct {
  int sampler;          /* hr_sampler; default HR_AIS                                 */
  int antithetic;       /* 1 (default): pair tau with -tau; 0: single draws             */
  double hvp_rel_step;  /* HVP central-difference step h = hvp_rel_step * sigma (0.1) */
  int accum_fp64;       /* 0 (default): compensated-FP32 lobe sums; 1: FP64 sums        */
  int samples_per_block;/* renders per raster/path-tracer block (raster: at most 256);
                           0 = library choice (raster: the largest of 256,
                           128, 64 and 32 that still gives at least 128 * S
                           blocks)                                            */
  int raster_tile;      /* raster block of 16x16 wave tiles: 1 = 32x32,
                           2 = 64x16, 3 = 16x64; 0 = library choice: the shape
                           that covers the image with the fewest blocks, ties
                           going to 16x64, then 32x32.  Neither this nor
                           samples_per_block changes any result bit: every wave
                           tile's loss partial is summed in a fixed order.          */
  double* dbg_loss;     /* optional host buffer receiving every render's loss, in the
                           order ((stream*N + s)*A + a)*S + shift, with a = 0 for
                           theta - tau, 1 for theta + tau, shift = 0 for +h, 1 for -h
                           (S = 2 for the HVP, else 1); NULL = not wanted           */
  double* dbg_tau;      /* optional host buffer receiving the draws tau, streams*N*n
                           doubles in the order (stream*N + s)*n + j; NULL = not wanted */
  int hess_mix_n2;      /* aggregate sampler with Hessian-kernel draws (Hessian, limit
                           HVP), section "Aggregate": 0 (default) mixes over the
                           n(n+1)/2 unique elements i <= j, 1 over all n^2 ordered
                           pairs (an off-diagonal element drawn twice as often);
                           ignored by the other samplers and estimators; other
                           values are HR_EINVAL                                    */
  int hvp_per_render;   /* HVP on a disk scene of at most 64 disks and W + H <= 2048,
                           0 (default): the two shifted scenes of a draw are taken
                           as a pair that yields their loss difference f(+h) - f(-h)
                           directly (only the pixels along the disks' edges whose
                           top disk can differ between the shifts are visited, and
                           decided per shift in FP64); then dbg_loss receives one
                           difference per (stream, draw, a), in the order
                           (stream*N + s)*A + a.  1: every shifted scene rendered
                           and its loss taken separately (always so for larger
                           scenes).  Other values are HR_EINVAL                     */
} hr_opts;

/* Fills the defaults listed above. */
void hr_opts_default(hr_opts* o);

/* ---- context ------------------------------------------------------------ */
/* Creates a context on HIP device `device`: one stream of default priority and
 * an empty workspace.  Errors: HR_EINVAL (bad device), HR_EDEVICE. */
hr_status hr_ctx_create(int device, hr_ctx** out);
void hr_ctx_destroy(hr_ctx* ctx);
/* Makes `stream` (a hipStream_t of the context's device, e.g. a torch stream)
 * the stream all "_dev" calls enqueue on; NULL restores the context's own. */
hr_status hr_ctx_set_stream(hr_ctx* ctx, void* stream);
/* Upper bound on workspace bytes one call may hold (default: 64 GiB). */
hr_status hr_ctx_set_memory_budget(hr_ctx* ctx, uint64_t bytes);
/* Waits for all work enqueued by the context. */
hr_status hr_ctx_synchronize(hr_ctx* ctx);
/* Kernel timing: when enabled, HIP events bracket every launch of the named
 * kernel on the stream it is launched on; stats report launch count and the
 * summed event time in milliseconds.  Names: "raster_loss", "pt_loss",
 * "tile_reduce", "sample", "records", "accumulate"; batches (eager runs):
 * "batch_sample", "batch_records", "batch_analytic", "batch_raster",
 * "batch_pt", "batch_reduce", "batch_prep", "batch_accum", "batch_finalize". */
hr_status hr_ctx_enable_timing(hr_ctx* ctx, int enable);
hr_status hr_ctx_kernel_stats(hr_ctx* ctx, const char* name, uint64_t* launches,
                              double* total_ms);
hr_status hr_ctx_reset_stats(hr_ctx* ctx);
const char* hr_last_error(void);

/* ---- device memory for the "_dev" entry points ---------------------------
 * Plain HBM allocations on the context's device, so callers need no other GPU
 * runtime in the process.  hr_memcpy copies `bytes` between host and device
 * (kind 0: host -> device, 1: device -> host, 2: device -> device) in order on
 * the context stream and returns when the copy is complete. */
hr_status hr_dev_alloc(hr_ctx* ctx, size_t bytes, void** out);
hr_status hr_dev_free(hr_ctx* ctx, void* ptr);
hr_status hr_memcpy(hr_ctx* ctx, void* dst, const void* src, size_t bytes, int kind);

/* ---- scenes (copied to the device at creation; immutable) ---------------- */
/* Disks in painter's order on a black background (the plateau tasks of
 * section "Methods", with disks for squares).  A pixel centre
 * ((x + 1/2)/W, (y + 1/2)/H) takes the colour of the last disk with positive
 * radius whose squared distance to it is below r^2.
 *   params_per_disk 2: theta = (cx, cy) per disk, radii from `radius` (D floats);
 *   params_per_disk 3: theta = (cx, cy, r) per disk, `radius` ignored.
 *   colors: D*C floats; target: H*W*C floats.  C in 1..4, D in 1..1024. */
hr_status hr_scene_disks(hr_ctx* ctx, int W, int H, int C, int n_disks, int params_per_disk,
                         const float* radius, const float* colors, const float* target,
                         hr_scene** out);
/* Path-traced scene (section "Background": Monte Carlo light transport).
 * Diffuse spheres on the ground plane y = 0, one square light facing -y,
 * pinhole camera; per pixel `spp` jittered paths with next-event estimation at
 * the first two surface hits and one cosine-weighted bounce; black background.
 * desc (FP64): eye[3], look_at[3], vfov_deg, light_side, Le, ground_albedo[3],
 * then per sphere centre[3], radius, albedo[3] (sphere 0's centre comes from
 * theta).  Pixel randomness of draw s is shared by all renders of that draw.
 * nspheres in 1..16; target H*W*3 floats. */
hr_status hr_scene_pt(hr_ctx* ctx, int W, int H, int spp, int nspheres, const double* desc,
                      const float* target, hr_scene** out);
/* Analytic test scenes: f = 1/2 theta^T A theta + b^T theta + c (the quadratic
 * task of section "Methods"), and f = -N(theta; 0, s1^2 I) (appendix on
 * non-PSD Hessians).  n in 1..128. */
hr_status hr_scene_quad(hr_ctx* ctx, int n, const double* A, const double* b, double c,
                        hr_scene** out);
hr_status hr_scene_neggauss(hr_ctx* ctx, int n, double s1, hr_scene** out);
/* Frees a scene.  A scene belongs to its context: destroying the context
 * first releases the scene's device memory and orphans it -- every later call
 * with it returns HR_EINVAL, and hr_scene_destroy still frees the handle.
 * Queries a server holds on the scene (submitted, not yet finished) complete
 * first: the call blocks until they have. */
void hr_scene_destroy(hr_scene* sc);
int hr_scene_nparams(const hr_scene* sc);

/* Renders an image scene at theta (host FP64) into `image` (host, H*W*C
 * floats).  For the path tracer, `s` selects the draw's pixel randomness and
 * `spp` > 0 overrides the scene's samples per pixel. */
hr_status hr_render(hr_scene* sc, const double* theta, uint64_t seed, uint32_t s, int spp,
                    float* image);

/* ---- estimators (host pointers; synchronous) ---------------------------- */
/* g (n doubles) of the smoothed loss: gradient kernel -tau_i/sigma^2 N(tau)
 * (section "Gradients"). */
hr_status hr_est_grad(hr_scene* sc, const double* theta, double sigma, uint64_t N,
                      uint64_t seed, const hr_opts* opts, double* g);
/* H (n*n doubles, row-major, symmetric): Hessian kernel (section "Hessians");
 * only the n(n+1)/2 elements i <= j are estimated, then mirrored. */
hr_status hr_est_hessian(hr_scene* sc, const double* theta, double sigma, uint64_t N,
                         uint64_t seed, const hr_opts* opts, double* H);
/* Hv (n doubles): |v| (g(theta + h u) - g(theta - h u)) / (2h), u = v/|v|,
 * h = hvp_rel_step * sigma, both gradients from the same draws (section
 * "Hessian-vector product").  v = 0 returns 0 without rendering. */
hr_status hr_est_hvp(hr_scene* sc, const double* theta, double sigma, uint64_t N,
                     uint64_t seed, const double* v, const hr_opts* opts, double* Hv);
/* Hv through the sampled Hessian kernel applied to v (the epsilon -> 0 limit of
 * the central difference): one render per draw, linear in v.  HR_AIS or
 * HR_GAUSS only (HR_EUNSUPPORTED for HR_IS). */
hr_status hr_est_hvp_limit(hr_scene* sc, const double* theta, double sigma, uint64_t N,
                           uint64_t seed, const double* v, const hr_opts* opts, double* Hv);

/* Smoothed loss F(theta) = E f(theta - tau), tau ~ N(0, sigma^2 I) (section
 * "Background"): mean of the renders over N plain Gaussian draws (antithetic
 * pairs as set in opts; opts->sampler is ignored).  sigma = 0 returns the plain
 * loss f(theta) of one render.  F: one double (host). */
hr_status hr_est_loss(hr_scene* sc, const double* theta, double sigma, uint64_t N,
                      uint64_t seed, const hr_opts* opts, double* F);

/* ---- grey-box composition (appendix "Grey-box differentials") -----------
 * The scene's parameters y = g(x) come from a caller-side inner map with known
 * Jacobian J = dg/dx: n rows (scene parameters) x n_in columns, row-major,
 * host FP64.  The outer derivatives are sampled at y exactly as by the plain
 * estimators and composed in FP64 on the GPU:
 *   gx  = J^T g_y                          (n_in doubles)
 *   Hx  = J^T H_y J (inner second derivatives dropped, as in the appendix)
 *                                           (n_in * n_in doubles, row-major)
 *   Hvx = J^T H_y (J vx)  with H_y (J vx) by hr_est_hvp's central difference
 * n_in in 1..4096; errors as for the plain estimators. */
hr_status hr_est_grad_greybox(hr_scene* sc, const double* y, const double* J, int n_in,
                              double sigma, uint64_t N, uint64_t seed, const hr_opts* opts,
                              double* gx);
hr_status hr_est_hessian_greybox(hr_scene* sc, const double* y, const double* J, int n_in,
                                 double sigma, uint64_t N, uint64_t seed, const hr_opts* opts,
                                 double* Hx);
hr_status hr_est_hvp_greybox(hr_scene* sc, const double* y, const double* J, int n_in,
                             double sigma, uint64_t N, uint64_t seed, const double* vx,
                             const hr_opts* opts, double* Hvx);

/* ---- estimators (device pointers; asynchronous on the context stream) ---- */
/* Same results as the host versions.  d_theta, d_v: n FP64 on the device;
 * outputs n (grad, HVP) or n*n (Hessian) FP64 on the device.  d_v == 0 gives
 * a zero result.  dbg_loss is ignored. */
hr_status hr_est_grad_dev(hr_scene* sc, const double* d_theta, double sigma, uint64_t N,
                          uint64_t seed, const hr_opts* opts, double* d_g);
hr_status hr_est_hessian_dev(hr_scene* sc, const double* d_theta, double sigma, uint64_t N,
                             uint64_t seed, const hr_opts* opts, double* d_H);
hr_status hr_est_hvp_dev(hr_scene* sc, const double* d_theta, double sigma, uint64_t N,
                         uint64_t seed, const double* d_v, const hr_opts* opts, double* d_Hv);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * HVP as hr_est_hvp_dev -- same kernels, same result bits -- with its
 * workspace in a fixed array of 64 MiB that every GPU the library runs on
 * holds from context creation until the process ends; the call makes no
 * allocation.  The caller passes inputs and output as for hr_est_hvp_dev.
 * Requests whose workspace exceeds 64 MiB return HR_ENOMEM (on the 256x256
 * RGB, 32-disk scene: about 79k draws by render pairs, 9.5k with
 * hvp_per_render).  Every call on one GPU uses the
 * same array: calls that overlap on one GPU (other streams, other contexts
 * of the device) race and must be ordered by the caller. */
hr_status hr_est_hvp_dev_noalloc(hr_scene* sc, const double* d_theta, double sigma, uint64_t N,
                                 uint64_t seed, const double* d_v, const hr_opts* opts,
                                 double* d_Hv);

/* ---- Newton-CG step (section "Previous Work") ---------------------------- */
typedef struct {
  int cg_iters;          /* maximum inner CG iterations (default 10)                 */
  double trust_radius;   /* Delta: each CG step length alpha <= Delta/|v| (default 1) */
  int use_full_hessian;  /* 1: modified Newton on the estimated H (eigenvalues
                            clamped to max(|lambda|, eig_floor)), step scaled into
                            Delta; 0: Newton-CG with HVPs (default)                  */
  double eig_floor;      /* default 1e-6                                             */
  int hvp_limit;         /* 1: CG products through hr_est_hvp_limit                  */
  int modified;          /* 0 (default): Steihaug exits above; 1: Hessian modification
                            inside CG -- v^T H v replaced by max(|v^T H v|,
                            eig_floor |v|^2), truncated steps continue, so all
                            cg_iters products are made unless |r| <= 1e-10 |g|   */
} hr_ncg_opts;

typedef struct {
  int iters_done;        /* HVP products used (1 in full-Hessian mode)               */
  int hit_trust;         /* a step was truncated at Delta                            */
  int neg_curv;          /* v^T H v <= 0 was met                                     */
  double step_norm;      /* |theta_new - theta|                                      */
  double g_norm;         /* |g(theta)|                                               */
} hr_ncg_report;

void hr_ncg_opts_default(hr_ncg_opts* o);
/* One step: g = est_grad(theta); inner Fletcher-Reeves CG on H d = -g at the
 * fixed theta with HVPs from the same seed; alpha = r^T r / v^T H v truncated
 * to Delta/|v| (then the loop ends); v^T H v <= 0 moves to the trust boundary
 * along v and ends; |r| <= 1e-10 |g| ends.  theta (host, n) is updated in
 * place.  All vector arithmetic of the solve runs in FP64 on the GPU. */
hr_status hr_newton_cg_step(hr_scene* sc, double* theta, double sigma, uint64_t N,
                            uint64_t seed, const hr_ncg_opts* ncg, const hr_opts* opts,
                            hr_ncg_report* report);
/* Same with theta in device memory (updated in place). */
hr_status hr_newton_cg_step_dev(hr_scene* sc, double* d_theta, double sigma, uint64_t N,
                                uint64_t seed, const hr_ncg_opts* ncg, const hr_opts* opts,
                                hr_ncg_report* report);

/* ---- optimiser loop (appendix "Hyperparameters") --------------------------
 * sigma annealed linearly from sigma_start to sigma_end over the iterations;
 * the step of each iteration comes from Newton-CG, modified Newton on the full
 * estimated H, or gradient descent; an optional line search halves alpha from
 * 1 up to ls_iters times until the smoothed loss (N_loss draws, the
 * iteration's seed for every trial) drops by ls_tol |F|, else alpha = 0;
 * "recompute" reads as the number of iterations an accepted alpha is reused
 * before a fresh search.  Iteration t uses draws keyed by seed + t. */
typedef enum { HR_OPT_NEWTON_CG = 0, HR_OPT_NEWTON_FULL = 1, HR_OPT_GD = 2 } hr_optim_method;

typedef struct {
  int iters;                       /* outer iterations (default 10)                    */
  double sigma_start, sigma_end;   /* linear schedule (0.1 -> 0.01)                    */
  int method;                      /* hr_optim_method (HR_OPT_NEWTON_CG)               */
  double lr;                       /* gradient-descent step (0.1)                      */
  int ls_iters;                    /* line-search halvings, 0 = none (0)               */
  double ls_tol;                   /* relative decrease demanded (1e-3)                */
  int recompute;                   /* iterations between fresh searches (1)            */
  uint64_t N_loss;                 /* draws per smoothed-loss estimate (1024)          */
  hr_ncg_opts ncg;                 /* inner Newton settings (hr_ncg_opts_default)      */
} hr_optim_opts;

void hr_optim_opts_default(hr_optim_opts* o);
/* theta (host, n) updated in place.  trace: optional host buffer of iters x 5
 * doubles -- sigma_t, alpha, |alpha d|, smoothed loss at the new theta
 * (sigma_t, N_loss draws), plain loss at the new theta. */
hr_status hr_optimize(hr_scene* sc, double* theta, uint64_t N, uint64_t seed,
                      const hr_optim_opts* opts_optim, const hr_opts* opts, double* trace);

/* ---- batched queries ------------------------------------------------------
 * Many independent estimator queries -- any scenes of one context, any kinds,
 * image sizes, parameter counts and sample budgets -- run together: one
 * launch per pipeline step over all queries, and one persistent launch each
 * for the rasteriser and the path tracer that takes (query, chunk, tile) work
 * items from per-XCD queues, longest items first.  The launch sequence is
 * fixed (all per-batch data is in one device table), so it is captured once
 * as a hipGraph and replayed for every later batch.  Each result is the same
 * bits as the single-query entry point returns for the same query, whatever
 * the batch around it and whatever samples_per_block / raster_tile. */
typedef enum {
  HR_QUERY_GRAD = 0,        /* out: n doubles                                   */
  HR_QUERY_HESSIAN = 1,     /* out: n*n doubles                                 */
  HR_QUERY_HVP = 2,         /* out: n doubles; v required                       */
  HR_QUERY_HVP_LIMIT = 3,   /* out: n doubles; v required                       */
  HR_QUERY_LOSS = 4         /* out: 1 double (smoothed loss; sigma = 0: plain)  */
} hr_query_kind;

typedef struct {
  hr_scene* scene;
  int kind;                 /* hr_query_kind                                    */
  double sigma;
  uint64_t N;               /* draws                                            */
  uint64_t seed;
  const double* theta;      /* host, n doubles; read during the call            */
  const double* v;          /* host, n doubles (HVP kinds), else NULL           */
  const hr_opts* opts;      /* NULL = defaults; dbg buffers must be NULL        */
  double* out;              /* host result buffer (see hr_query_kind)           */
} hr_query;

typedef struct {
  int use_graph;            /* 1 (default): replay the launches as a hipGraph   */
  int autotune;             /* 1: before a batch, time samples-per-block
                               (32-256) and block shape (the three) for
                               every not yet tuned class of disk scene
                               (channels, disk count, image size buckets),
                               and draws per block item (2-32) for every not
                               yet tuned class of path-traced query (renders
                               per draw, samples per pixel, sphere count,
                               image size buckets), and keep the fastest in
                               the context; 0 (default): the library's
                               choices (samples_per_block and raster_tile 0;
                               8 draws per path-traced item).  A query's own
                               samples_per_block still comes first.            */
} hr_batch_opts;

typedef struct {
  uint64_t queries;         /* queries in the last run                          */
  uint64_t raster_items;    /* work items of the persistent rasteriser          */
  uint64_t pt_items;        /* work items of the persistent path tracer         */
  int raster_blocks;        /* persistent grid size of the rasteriser (largest
                               over the raster classes launched)              */
  int pt_blocks;            /* persistent grid size of the path tracer         */
  uint64_t workspace_bytes; /* device workspace of the batch                    */
  uint64_t lds_bytes;       /* dynamic LDS of the persistent rasteriser         */
  int graph;                /* 1 if the launches ran as a graph replay; a batch
                               of one query runs the per-query kernels directly
                               (same result bits) and reports 0               */
} hr_batch_report;

typedef struct hr_batch hr_batch;
void hr_batch_opts_default(hr_batch_opts* o);
/* A batch executor of the context (own stream, table, workspace and graph). */
hr_status hr_batch_create(hr_ctx* ctx, const hr_batch_opts* opts, hr_batch** out);
void hr_batch_destroy(hr_batch* b);
/* Runs `count` queries and returns when every out buffer is written.
 * Errors: any query's validation error (HR_EINVAL / HR_EUNSUPPORTED, message
 * names the query), HR_ENOMEM when the summed workspace exceeds the context's
 * memory budget; no query is run then. */
hr_status hr_batch_run(hr_batch* b, const hr_query* queries, int count);
hr_status hr_batch_report_get(const hr_batch* b, hr_batch_report* out);
/* The autotuner's choice for the scene's class (0, 0 if not tuned yet).  For
 * a path-traced scene: the draws per block item tuned for its queries with two
 * renders per draw (gradients and Hessians with antithetic pairs), and 0 as
 * raster_tile. */
hr_status hr_batch_tuned(hr_ctx* ctx, const hr_scene* sc, int* samples_per_block,
                         int* raster_tile);

/* ---- serving: continuous batching ------------------------------------------
 * A server owns a worker thread and `slots` batch executors, each with its own
 * stream.  Queries are submitted asynchronously; whenever a slot is free the
 * worker forms a batch from the waiting queries in arrival order, admitting a
 * query only while the batch's workspace fits the slot's share of
 * memory_bytes, and launches it at once -- so queries arriving while others
 * are on the GPU start in the next free slot and their work overlaps with the
 * batches in flight.  Results are the same bits as the single-query entry
 * points give.  hr_scene_destroy on a scene with queries still held by a
 * server blocks until they have finished. */
typedef struct {
  int slots;                /* batches in flight (default 4)                    */
  int max_batch;            /* queries per batch (default 64)                   */
  double max_batch_ms;      /* predicted device time per batch (default 2 ms;
                               <= 0: no limit).  The prediction is a static
                               cost model (renders x pixels for the
                               rasteriser, x samples per pixel for the path
                               tracer, draws x elements for the lobe sums);
                               a query is always admitted into an empty batch.
                               A query that fills the cap alone runs as a
                               one-query batch on the per-query kernels;
                               smaller ones share the batch's launches.      */
  uint64_t memory_bytes;    /* device workspace across all slots
                               (default: the context's memory budget)           */
  int use_graph;            /* as in hr_batch_opts (default 1)                  */
  int autotune;             /* as in hr_batch_opts (default 0)                  */
  const char* metrics_path; /* per-query metrics as JSON Lines, appended to
                               this file (default NULL: none): one object per
                               completed query with ticket, kind, scene, W, H,
                               params, N, seed, sampler, renders, batch,
                               batch_size, slot, submit_ms, start_ms, end_ms,
                               queue_ms, service_ms and status (times in ms
                               since the server started).  The string is read
                               at creation only; a file that cannot be opened
                               is HR_EINVAL.                                    */
} hr_server_opts;

typedef struct {
  double submit_ms;         /* times since the server started                   */
  double start_ms;          /* its batch was launched                           */
  double end_ms;            /* its batch's results were on the host             */
  int batch_size;           /* queries in its batch                             */
  hr_status status;         /* HR_OK, or the error that failed its batch        */
} hr_query_stats;

typedef struct {
  uint64_t submitted, completed, batches;
  double mean_batch;        /* queries per batch                                */
  double busy_ms;           /* wall time with at least one batch in flight      */
} hr_server_stats;

typedef struct hr_server hr_server;
void hr_server_opts_default(hr_server_opts* o);
hr_status hr_server_create(hr_ctx* ctx, const hr_server_opts* opts, hr_server** out);
/* Waits for every submitted query, then stops the worker. */
void hr_server_destroy(hr_server* s);
/* Validates and enqueues a query; theta and v are copied, q->out is ignored
 * (the result is returned by hr_wait).  Errors: validation errors as in
 * hr_batch_run; HR_ENOMEM if the query alone exceeds a slot's workspace. */
hr_status hr_submit(hr_server* s, const hr_query* q, uint64_t* ticket);
/* Blocks until the query is done, copies its result to `out` (sized as in
 * hr_query_kind) and its timings to `stats` (either may be NULL), and retires
 * the ticket.  Returns the query's status; HR_EINVAL for unknown or retired
 * tickets; HR_EBUSY if another thread is already waiting on the ticket (one
 * waiter per ticket). */
hr_status hr_wait(hr_server* s, uint64_t ticket, double* out, hr_query_stats* stats);
/* Waits up to timeout_ms (< 0: no limit) for any completed, not yet retired
 * query and returns its ticket; HR_EBUSY if none completed in time. */
hr_status hr_wait_any(hr_server* s, double timeout_ms, uint64_t* ticket);
hr_status hr_server_stats_get(hr_server* s, hr_server_stats* out);

#ifdef __cplusplus
}
#endif
#endif /* HREST_H */
