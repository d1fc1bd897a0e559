// hr_kernels.h -- launch interface between the host runtime (hr_api.hip) and
// the device kernels (hr_raster.hip, hr_estim.hip, hr_pt.hip, hr_solve.hip).
#pragma once
#include <type_traits>
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
  int mix_n2;                        // aggregate Hessian mixture over the n^2 ordered pairs
  int nout;                          // estimated elements (K for the Hessian, else n)
  uint64_t N, streams;               // streams = K for per-element IS, else 1
  int A, NH;                         // antithetic factor, shifts per render group
  uint64_t R;                        // renders = streams * N * A * NH
  int pair;                          // 1: an HVP on a disk scene whose +-h renders come as
                                     //    pairs, one loss difference per (draw, a)
  int pad_;
  uint64_t L;                        // loss outputs: R / 2 pairs (pair), else R
  // device flag: when it reads nonzero at launch, every kernel of the query
  // returns at once (a Newton-CG product after the inner loop stopped);
  // nullptr: never
  const int* skip;
  double sigma, h;                   // h: HVP step (0 if none)
  uint64_t seed;
};

// ---- sampling ----
void launch_sample(hipStream_t st, const EstShape& e, double* tau);
// sampling with |v| and v / |v| of an HVP query computed by block 0; with
// draws false only |v| and v / |v| (tau already holds the query's draws)
void launch_sample_vnorm(hipStream_t st, const EstShape& e, double* tau, const double* v,
                         double* u, double* vnorm, bool draws = true);

// ---- renders ----
// Half-width of the band around r^2 outside which the FP32 and the FP64
// decision of (px - cx)^2 + (py - cy)^2 < r^2 provably agree.  FP32 rounding
// of the pixel centre, of the disk centre and of the products moves
// d^2 - r^2 by at most about 2^-21 r (1 + |cx| + |cy|) + 2^-22 r^2 near the
// circle (|dx|, |dy| <= r there); the band is 4-8x that.
__host__ __device__ inline double ambiguity_band(double cx, double cy, double r) {
  return 0x1p-19 * (r * (1.0 + fabs(cx) + fabs(cy)) + r * r);
}

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
// of render 0 for the exact path).  A block covers bwx x bwy wave tiles of
// 16x16 pixels and S renders per work item; the loss partial of every wave
// tile is written to partial[part_index(r, wave tile, subs)], so neither the
// block shape nor S changes any result bit.
// Largest parameter count of any scene (1024 disks x 3); the lobe
// accumulation stages at least one draw of that many doubles in LDS.
constexpr int kMaxParams = 3072;

// Loss partials of a query, (render r, tile t) of `tiles` per render: groups
// of 16 renders, tile-major inside a group, so one tile's partials of 16
// consecutive renders fill one 64-byte line (a wave writes them at once, and
// the loss pass reads them coalesced).
__host__ __device__ inline uint64_t part_index(uint64_t r, uint64_t t, uint64_t tiles) {
  return ((r >> 4) * tiles + t) * 16u + (r & 15u);
}
inline uint64_t part_floats(uint64_t R, uint64_t tiles) { return ((R + 15) / 16) * 16 * tiles; }

struct RasterQuery {
  const float4* rec;
  const float* target;
  const float* colors;
  float* partial;
  int W, H, C, D, S;
  int bwx, bwy;          // wave tiles per block along x and y (bwx * bwy == 4)
  int tiles_x, tiles;    // blocks per row, per image
  int subs_x, subs;      // wave tiles per row, per image
  int pad;
  uint64_t R, r_base;
  RasterExact ex;
  const int* skip;       // as EstShape::skip
};
// the per-query raster kernel finds `ex` in its kernel arguments by offsetof
static_assert(std::is_standard_layout<RasterQuery>::value, "RasterQuery is read by offsetof");
// block shapes: 1 = 32x32, 2 = 64x16, 3 = 16x64, 0 = the fewest blocks for a
// W x H image (ties: 16x64, then 32x32)
void raster_block_shape(int shape, int W, int H, int* bwx, int* bwy);
size_t raster_lds_bytes(int D, int S);
int raster_max_samples();
int raster_auto_samples(int W, int H, uint64_t R, int shape);
// fills the geometry fields of a RasterQuery (W, H must be set)
void raster_geometry(RasterQuery& a, int shape);
void launch_records(hipStream_t st, const EstShape& e, const DiskScene& s, const double* theta,
                    const double* tau, const double* u, float4* rec);
// HVP render pairs (e.pair) on a disk scene: pair p = (stream * N + s) * A +
// a stands for the renders at theta + h u - a tau_s and theta - h u - a tau_s;
// f[p] = scale * (sum over pixels of (I+ - T)^2 - (I- - T)^2), decided with
// exact coverage along the disks' edges (hr_edges.hip)
struct PairQuery {
  const double* theta;
  const double* tau;
  const double* u;           // v / |v|
  const float* radius;       // D (ppd == 2)
  const float* colors;       // D x C
  const float* target;       // H x W x C
  double* f;                 // L loss differences
  int W, H, C, D, ppd, n, A, S;   // S: pairs per batch item
  double h, scale;           // shift; 1 / (W H C)
  uint64_t L;                // pairs
  const int* skip;           // as EstShape::skip
};
void launch_raster_dloss(hipStream_t st, const PairQuery& a);
size_t raster_pair_lds_bytes(int W, int H, int D);
// largest disk count, and largest W + H, of the pair path (larger scenes
// render the HVP per render)
int raster_pair_max_disks();
int raster_pair_max_side_sum();
// number of 16x16 wave tiles of the image: the partial stride per render
int raster_subtiles(int W, int H);
void launch_raster_loss(hipStream_t st, const DiskScene& s, const float4* rec, uint64_t R,
                        int samples_per_block, int shape, const RasterExact& ex, float* partial,
                        const int* skip = nullptr);
void launch_tile_reduce(hipStream_t st, const float* partial, uint64_t R, int tiles,
                        double inv_count, double* f, const int* skip = nullptr);
void launch_render_disks(hipStream_t st, const DiskScene& s, const RasterExact& ex, float* image);

struct PTScene {
  int W, H, spp, nspheres;
  const float* target;   // H*W*3
  const float* desc;     // FP32 copy of the scene description (host)
  const void* ptc;       // device copy of the tracer's constants (pt_fill_const)
};
int pt_tiles(int W, int H);
int pt_tiles_x(int W);
int pt_max_samples();
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

// ---- batched execution ----
// A batch runs many queries through one launch per phase.  Each phase kernel
// walks a task list: the tasks of query q are [off[phase][q], off[phase][q+1]);
// a task is either a run of kBatchElems consecutive elements of a per-element
// step or one block of a per-block step, with the same arithmetic as the
// single-query kernels (so every output is the same bits).  Renders come from
// two persistent kernels that pull work items from eight queues, one per XCD.
constexpr int kBatchElems = 2048;    // elements per task of an elementwise step
constexpr int kBatchHeavyElems = 256; // per task where an element costs O(n) or more
                                      // (per-draw prep, analytic renders): one per thread
constexpr int kBatchRenders = 64;    // renders per task of the tile reduction

enum SceneKind { kDisks = 0, kPT = 1, kQuad = 2, kNegGauss = 3 };

struct WorkSeg {           // one query's items in one work queue
  uint64_t item0;          // first item of the segment within its queue
  int q;                   // query
  int c0;                  // first chunk; the segment holds chunks c0, c0 + 8, ...
  int tiles;               // items per chunk (blocks of the image)
  int pad;
};
struct WorkQueues {
  const WorkSeg* seg;
  unsigned long long* ctr;   // 8 item counters, zeroed by the sampling phase
  uint64_t seg_off[9];       // queue x owns seg[seg_off[x] .. seg_off[x + 1])
  uint64_t items[8];
};
struct BatchQuery {
  EstShape e;
  int scene, fp64, chunk, pt_S;
  int pt_tiles_x, pt_tiles, part_stride, pad;
  uint64_t nchunks;
  double inv_count;          // 1 / (pixels * channels) of a render's loss
  const double* theta;
  const double* v;
  double* out;
  double* tau;
  double* u;                 // n entries, then |v|
  float4* rec;
  float* partial;
  double* f;
  double* Fq;
  double* vt;
  void* acc;
  DiskScene ds;
  RasterQuery rq;
  AnalyticScene as;
  const void* ptc;           // device copy of the path tracer's constants
  const float* pt_target;
};
enum BatchPhase { kPhSample = 0, kPhRecords, kPhAnalytic, kPhReduce, kPhPrep, kPhAccum,
                  kPhFinalize, kNumPhases };
// Raster items are queued by class -- channel count and whether all disks
// fit one wavefront -- and each class has its own persistent kernel, which
// holds only that variant's registers.
constexpr int kRasterClasses = 16;
__host__ __device__ inline int raster_class(int C, int D) { return (C - 1) * 2 + (D > 64 ? 1 : 0); }
// HVP render pairs (at most 64 disks) by channel count and LDS layout:
// 8..11 the 64-disk layout, 12..15 the 32-disk one, which serves scenes of up
// to 32 disks only
__host__ __device__ constexpr int raster_pair_class(int C, int D) { return (D <= 32 ? 12 : 8) + (C - 1); }
__host__ __device__ constexpr bool raster_is_pair_class(int cls) { return cls >= 8; }
constexpr int kWorkCounters = 8 * (kRasterClasses + 3);   // 8 per queue set

struct BatchTable {
  int nq, pad;
  const BatchQuery* q;
  const uint64_t* off;       // [kNumPhases][nq + 1]
  WorkQueues raster[kRasterClasses];
  WorkQueues pt[3];          // path-traced items by renders per draw: 1, 2, 4
  unsigned long long* ctr;   // kWorkCounters item counters, zeroed by the sampling phase
};
// device-side lookup: the query owning task t of a phase (t < off[nq])
__device__ __forceinline__ int batch_find(const uint64_t* off, int nq, uint64_t t) {
  int lo = 0, hi = nq - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}
// Copy of a small table entry whose address is the same for the whole block,
// taken word by word through readfirstlane so that the compiler keeps it in
// scalar registers (a plain load after the block's own stores would be a
// vector load).
template <class Ty>
__device__ __forceinline__ Ty uniform_copy(const Ty* p) {
  static_assert(sizeof(Ty) % 4 == 0, "word-sized table entries only");
  Ty v;
  const uint32_t* src = (const uint32_t*)p;
  uint32_t* dst = (uint32_t*)&v;
#pragma unroll
  for (int i = 0; i < (int)(sizeof(Ty) / 4); ++i) dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
  return v;
}
// tasks per phase of one query (host planning)
uint64_t batch_tasks(const BatchQuery& q, int phase);
void launch_batch_sample(hipStream_t st, const BatchTable* T, int blocks);
void launch_batch_records(hipStream_t st, const BatchTable* T, int blocks);
void launch_batch_analytic(hipStream_t st, const BatchTable* T, int blocks);
void launch_batch_raster(hipStream_t st, const BatchTable* T, int cls, int blocks, size_t lds);
// path-traced items with nr renders per draw (1, 2 or 4)
void launch_batch_pt(hipStream_t st, const BatchTable* T, int nr, int blocks);
void launch_batch_reduce(hipStream_t st, const BatchTable* T, int blocks);
void launch_batch_prep(hipStream_t st, const BatchTable* T, int blocks);
void launch_batch_accum(hipStream_t st, const BatchTable* T, int blocks);
void launch_batch_finalize(hipStream_t st, const BatchTable* T, int blocks);
// occupancy of the persistent raster kernel (blocks per CU) for a given LDS size
int batch_raster_blocks_per_cu(int cls, size_t lds);
// the persistent form of the render-pair kernel, by channel count C
void launch_batch_dloss(hipStream_t st, const BatchTable* T, int cls, int blocks, size_t lds);
int batch_dloss_blocks_per_cu(int cls, size_t lds);
int batch_pt_blocks_per_cu(int nr);
// path tracer constants for device-resident scenes
size_t pt_const_bytes();
void pt_fill_const(const PTScene& s, void* host_out);

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
