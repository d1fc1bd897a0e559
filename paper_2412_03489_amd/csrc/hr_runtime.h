// hr_runtime.h -- host-side state shared by the library's translation units:
// contexts, device-resident scenes, error reporting, and the planning of one
// estimator query (validation, shape, workspace layout) used alike by the
// single-query entry points, the batch executor and the server.
#pragma once
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cmath>
#include <condition_variable>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "hrest.h"
#include "hr_kernels.h"

// A roctx range over a host-side call (estimates, solver steps, batches),
// shown by rocprofv3 --marker-trace; nearly free when no tool listens.
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

// The captured launch sequence of a repeated Newton-CG step and the
// arguments it was captured for.
struct NewtonGraph {
  hipGraphExec_t exec = nullptr;
  std::vector<char> key;
  int runs = 0;              // eager runs with this key (-1: does not capture)
};

struct hr_ctx {
  int device = 0;
  hipStream_t own = nullptr;
  hipStream_t stream = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  void* stage = nullptr;      // host-call staging: theta, v, outputs
  size_t stage_bytes = 0;
  void* hstage = nullptr;     // pinned host mirror of the staging (async copies)
  size_t hstage_bytes = 0;
  void* cg = nullptr;         // Newton-CG vectors and state
  size_t cg_bytes = 0;
  uint64_t budget = 64ull << 30;
  bool timing = false;
  struct Pending { std::string name; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::map<std::string, std::pair<uint64_t, double>> stats;
  std::set<hr_scene*> scenes;   // released (and orphaned) with the context
  // samples-per-block / block-shape choices of the raster autotuner, by class
  std::map<uint64_t, std::pair<int, int>> tuned;
  std::mutex tuned_mu;   // a server's worker and the caller's thread share it
  NewtonGraph newton_graph;
};

uint64_t next_scene_uid();

struct hr_scene {
  hr_ctx* ctx = nullptr;
  uint64_t uid = next_scene_uid();   // distinct for every scene of the process
  int kind = hr::kDisks;
  int n = 0;
  int W = 0, H = 0, C = 0;
  float* target = nullptr;
  int D = 0, ppd = 0;
  float* colors = nullptr;
  float* radius = nullptr;
  std::vector<float> hradius;
  int spp = 0, nspheres = 0;
  std::vector<float> pt_desc;   // FP32 description + derived camera basis
  void* ptc = nullptr;          // device copy of the path tracer's constants
  double* A = nullptr;
  double* b = nullptr;
  double c = 0.0, s1 = 1.0;
  // queries a server holds on this scene (waiting or on the device);
  // hr_scene_destroy waits for them to finish
  std::mutex hold_mu;
  std::condition_variable hold_cv;
  int held = 0;
};

namespace hr {
namespace rt {

// the calling thread's last error message (read by hr_last_error)
std::string& error_slot();

inline hr_status fail(hr_status st, const std::string& msg) {
  error_slot() = msg;
  return st;
}

#define HR_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return ::hr::rt::fail(HR_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

inline bool finite_all(const double* x, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

hr_opts resolve(const hr_opts* o);

// Grows a device buffer to at least `need` bytes (synchronising the context
// stream before freeing the old one).
hr_status ensure(hr_ctx* ctx, void** buf, size_t* have, size_t need);
// grow-only pinned host buffer (hipHostMalloc)
hr_status ensure_host(hr_ctx* ctx, void** buf, size_t* have, size_t need);

// Records `fn`'s launches between two events on the context stream when
// timing is enabled.
template <class F>
void timed(hr_ctx* ctx, const char* name, F&& fn) {
  if (!ctx->timing) {
    fn();
    return;
  }
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) { fn(); return; }
  if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); fn(); return; }
  (void)hipEventRecord(a, ctx->stream);
  fn();
  (void)hipEventRecord(b, ctx->stream);
  ctx->pending.push_back({name, a, b});
}
hr_status drain_timers(hr_ctx* ctx);

// One estimator query, validated and sized.
struct QueryPlan {
  hr_scene* sc = nullptr;
  hr_opts o{};                 // resolved options (the smoothed loss forces GAUSS)
  EstShape e{};
  int chunk = 0;               // draws per accumulation chunk
  uint64_t nchunks = 0;
  int stride = 0;              // loss partials per render (0: analytic scene)
  size_t b_tau = 0, b_u = 0, b_rec = 0, b_part = 0, b_f = 0, b_Fq = 0, b_vt = 0, b_acc = 0;
  size_t total = 0;            // workspace bytes
  size_t nout = 0;             // output doubles (n, n*n or 1)
};
hr_status plan_query(hr_scene* sc, int what, double sigma, uint64_t N, uint64_t seed, bool has_v,
                     const hr_opts& o_in, QueryPlan* p);

struct QueryBufs {
  double* tau;
  double* u;
  double* vnorm;
  float4* rec;
  float* partial;
  double* f;
  double* Fq;
  double* vt;
  void* acc;
};
QueryBufs carve(const QueryPlan& p, void* base);
// The kernels of one planned query on stream s, its workspace carved as qb;
// theta, v (or nullptr) and the output are device pointers.  S and shape pick
// the raster configuration (0: library choice).  With timing, the launches
// are timed under the per-query kernel names (ctx->stream must be s).  With
// keep_draws an HVP query does not sample: qb.tau already holds its draws (a
// query of the same plan, seed included, wrote them into this workspace).
void launch_query(hr_ctx* ctx, hipStream_t s, const QueryPlan& pl, const QueryBufs& qb,
                  const double* d_theta, const double* d_v, double* d_out, int S, int shape,
                  bool timing, bool keep_draws = false);

}  // namespace rt
}  // namespace hr
