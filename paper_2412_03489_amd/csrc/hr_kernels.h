// hr_kernels.h -- launch interface between the host runtime (hr_api.hip) and
// the device kernels (hr_raster.hip, hr_estim.hip, hr_pt.hip, hr_solve.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hr {

inline __host__ __device__ uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }

enum What { kGrad = 0, kHess = 1, kHvp = 2, kHvpLimit = 3, kLoss = 4 };
enum Sampler { kAIS = 0, kIS = 1, kGauss = 2, kFR22 = 3 };
// per-element streams (one stream of draws per estimated element)
inline __host__ __device__ bool per_element(int sampler) { return sampler == kIS || sampler == kFR22; }

// Shape of one estimator call.  Renders are indexed
//   r = ((stream * N + s) * A + a) * NH + shift
// with a = 0 for theta - tau, 1 for theta + tau; shift = 0 for +h u, 1 for -h u.
struct EstShape {
  int what, sampler, n, K, hessk;   // hessk: draws/weights from the Hessian kernel
  int nout;                          // estimated elements (K for the Hessian, else n)
  uint64_t N, streams;               // streams = K for per-element IS, else 1
  int A, NH;                         // antithetic factor, shifts per render group
  uint64_t R;                        // renders = streams * N * A * NH
  double sigma, h;                   // h: HVP step (0 if none)
  uint64_t seed;
};

// ---- sampling ----
void launch_sample(hipStream_t st, const EstShape& e, double* tau);
void launch_vnorm(hipStream_t st, int n, const double* v, double* u, double* vnorm);

// ---- renders ----
struct DiskScene {
  int W, H, C, D, ppd;
  const float* target;   // H*W*C
  const float* colors;   // D*C
  const float* radius;   // D (ppd == 2)
};
// Unrounded render parameters for the exact FP64 coverage decision:
// disk params of render r = theta (+- h u) - a tau_s (tau == nullptr: theta).
struct RasterExact {
  const double* theta;
  const double* tau;
  const double* u;
  const float* radius;
  int n, ppd, A, NH;
  double h;
};
// One query's raster work: records of renders [0, R) (r_base = global index
// of render 0 for the exact path), 32x32 tiles, S renders per work item.
struct RasterQuery {
  const float4* rec;
  const float* target;
  const float* colors;
  float* partial;
  int W, H, C, D, S, tiles_x, tiles, pad;
  uint64_t R, r_base;
  RasterExact ex;
};
size_t raster_lds_bytes(int D, int S);
int raster_max_samples();
void launch_records(hipStream_t st, const EstShape& e, const DiskScene& s, const double* theta,
                    const double* tau, const double* u, float4* rec);
// number of 32x32 tiles; partial[r * tiles + t]
int raster_tiles(int W, int H);
void launch_raster_loss(hipStream_t st, const DiskScene& s, const float4* rec, uint64_t R,
                        int samples_per_block, const RasterExact& ex, float* partial);
void launch_tile_reduce(hipStream_t st, const float* partial, uint64_t R, int tiles,
                        double inv_count, double* f);
void launch_render_disks(hipStream_t st, const DiskScene& s, const RasterExact& ex, float* image);

struct PTScene {
  int W, H, spp, nspheres;
  const float* target;   // H*W*3
  const float* desc;     // FP32 copy of the scene description
};
int pt_tiles(int W, int H);
void launch_pt_loss(hipStream_t st, const EstShape& e, const PTScene& s, const double* theta,
                    const double* tau, const double* u, int samples_per_block, float* partial);
void launch_pt_render(hipStream_t st, const PTScene& s, const double* theta, uint64_t seed,
                      uint32_t sidx, int spp, float* image);

struct AnalyticScene {
  int kind;              // 0 quadratic, 1 negated Gaussian
  int n;
  const double* A;       // n*n
  const double* b;       // n
  double c, s1;
};
void launch_analytic(hipStream_t st, const EstShape& e, const AnalyticScene& s,
                     const double* theta, const double* tau, const double* u, double* f);

// ---- weights and accumulation ----
void launch_prep(hipStream_t st, const EstShape& e, const double* f, const double* tau,
                 const double* vnorm, const double* v, double* Fq, double* vt);
int accum_chunk(const EstShape& e);
void launch_accum(hipStream_t st, const EstShape& e, const double* tau, const double* Fq,
                  const double* vt, const double* v, int fp64, void* part, int chunk);
void launch_finalize(hipStream_t st, const EstShape& e, const void* part, int fp64, int chunk,
                     double* out);

// ---- solver ----
struct CgState {
  int stop, iters, hit_trust, neg_curv, modified, pad;
  double rr, gnorm, delta, step_norm, eig_floor;
};
void launch_cg_init(hipStream_t st, int n, const double* g, double delta, int modified,
                    double eig_floor, double* r, double* p, double* d, CgState* cs);
void launch_cg_update(hipStream_t st, int n, const double* Hp, double* r, double* p, double* d,
                      CgState* cs);
void launch_cg_apply(hipStream_t st, int n, const double* d, double* theta, CgState* cs);
void launch_newton_full(hipStream_t st, int n, const double* H, const double* g, double delta,
                        double eig_floor, double* work, double* d, CgState* cs);

// ---- grey-box composition (FP64) ----
// J: n rows (scene parameters) x n_in columns, row-major
void launch_jt_vec(hipStream_t st, int n, int n_in, const double* J, const double* a, double* out);
void launch_j_vec(hipStream_t st, int n, int n_in, const double* J, const double* v, double* out);
void launch_jt_h_j(hipStream_t st, int n, int n_in, const double* J, const double* H, double* T,
                   double* out);

}  // namespace hr
