// hr_api.hip -- host runtime behind include/hrest.h: contexts, device-resident
// scenes, workspace carving, the estimator pipeline
//   draw tau -> perturbed renders + per-render loss -> per-draw weights ->
//   compensated lobe sums -> FP64 finalisation
// and the Newton-CG loop whose vector arithmetic runs on the GPU.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <atomic>
#include <mutex>
#include <string>
#include <vector>

#include "hr_runtime.h"

using namespace hr;
using namespace hr::rt;

// Fixed workspace of hr_est_hvp_dev_noalloc, for callers that cannot allocate
// (graph capture, tight serving loops).  Every GPU the library runs on holds
// its own copy until the process ends; host code reaches a device's copy only
// through the address hipGetSymbolAddress returns for it (g_scratch below),
// never through the array's name.
constexpr size_t kNoallocScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

uint64_t next_scene_uid() {
  static std::atomic<uint64_t> counter{1};
  return counter.fetch_add(1);
}

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};   // device address of `scratch`, per device

// Resolves the current device's copy of `scratch` once (at context creation).
hr_status scratch_resolve(int device) {
  if (device < 0 || device >= kMaxDevices)
    return fail(HR_EDEVICE, "device index beyond the fixed-workspace table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[device]) return HR_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || ptr == nullptr) {
    (void)hipGetLastError();
    return fail(HR_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  }
  g_scratch[device] = ptr;
  return HR_OK;
}

void* scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch[device];
}
}  // namespace

namespace hr {
namespace rt {

std::string& error_slot() {
  thread_local std::string err;
  return err;
}

hr_opts resolve(const hr_opts* o) {
  hr_opts r;
  hr_opts_default(&r);
  if (o) r = *o;
  return r;
}

hr_status ensure(hr_ctx* ctx, void** buf, size_t* have, size_t need) {
  if (need <= *have) return HR_OK;
  if (*buf) {
    HR_HIP(hipStreamSynchronize(ctx->stream));
    HR_HIP(hipFree(*buf));
    *buf = nullptr;
    *have = 0;
  }
  size_t sz = align256(need + need / 4);
  hipError_t e = hipMalloc(buf, sz);
  if (e != hipSuccess) {
    *buf = nullptr;
    (void)hipGetLastError();
    return fail(HR_ENOMEM, "device allocation of " + std::to_string(sz) + " bytes failed");
  }
  *have = sz;
  return HR_OK;
}

hr_status ensure_host(hr_ctx* ctx, void** buf, size_t* have, size_t need) {
  if (need <= *have) return HR_OK;
  if (*buf) {
    HR_HIP(hipStreamSynchronize(ctx->stream));
    HR_HIP(hipHostFree(*buf));
    *buf = nullptr;
    *have = 0;
  }
  size_t sz = align256(need + need / 4);
  hipError_t e = hipHostMalloc(buf, sz, hipHostMallocDefault);
  if (e != hipSuccess) {
    *buf = nullptr;
    (void)hipGetLastError();
    return fail(HR_ENOMEM, "pinned host allocation of " + std::to_string(sz) + " bytes failed");
  }
  *have = sz;
  return HR_OK;
}

hr_status drain_timers(hr_ctx* ctx) {
  for (auto& p : ctx->pending) {
    HR_HIP(hipEventSynchronize(p.b));
    float ms = 0.f;
    HR_HIP(hipEventElapsedTime(&ms, p.a, p.b));
    auto& s = ctx->stats[p.name];
    s.first += 1;
    s.second += ms;
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  ctx->pending.clear();
  return HR_OK;
}

hr_status plan_query(hr_scene* sc, int what, double sigma, uint64_t N, uint64_t seed, bool has_v,
                     const hr_opts& o_in, QueryPlan* p) {
  if (!sc) return fail(HR_EINVAL, "scene is NULL");
  if (!sc->ctx) return fail(HR_EINVAL, "the scene's context has been destroyed");
  if (what < kGrad || what > kLoss) return fail(HR_EINVAL, "unknown query kind");
  hr_opts o = o_in;
  if (what == kLoss) {
    // the smoothed loss uses the plain Gaussian draws; sigma = 0: one render at theta
    o.sampler = kGauss;
    if (sigma == 0.0) {
      N = 1;
      o.antithetic = 0;
    }
  }
  if (!(what == kLoss && sigma == 0.0) && (!(sigma > 0.0) || !std::isfinite(sigma)))
    return fail(HR_EINVAL, "sigma must be positive and finite");
  if (N == 0 || N >= 0xFFFFFFFFull) return fail(HR_EINVAL, "N must be in [1, 2^32 - 1)");
  if (o.sampler < 0 || o.sampler > 3) return fail(HR_EINVAL, "unknown sampler");
  if (o.raster_tile < 0 || o.raster_tile > 3) return fail(HR_EINVAL, "raster_tile must be in [0, 3]");
  if (o.hess_mix_n2 != 0 && o.hess_mix_n2 != 1) return fail(HR_EINVAL, "hess_mix_n2 must be 0 or 1");
  if (o.hvp_per_render != 0 && o.hvp_per_render != 1)
    return fail(HR_EINVAL, "hvp_per_render must be 0 or 1");
  if ((what == kHvp || what == kHvpLimit) && !has_v) return fail(HR_EINVAL, "v is NULL");
  if (what == kHvpLimit && per_element(o.sampler))
    return fail(HR_EUNSUPPORTED, "the limit-kernel HVP supports the aggregate and Gaussian samplers");
  if (what == kHess && o.sampler == kFR22)
    return fail(HR_EUNSUPPORTED, "the FR22 comparator estimates gradients and HVPs only");
  if (what == kHvp && !(o.hvp_rel_step > 0.0)) return fail(HR_EINVAL, "hvp_rel_step must be positive");
  if (sc->n < 1 || sc->n > kMaxParams) return fail(HR_EINVAL, "parameter count out of range");

  EstShape& e = p->e;
  e = EstShape{};
  e.what = what;
  e.sampler = o.sampler;
  e.n = sc->n;
  e.hessk = (what == kHess || what == kHvpLimit) ? 1 : 0;
  e.mix_n2 = (e.hessk && o.sampler == kAIS && o.hess_mix_n2) ? 1 : 0;
  e.K = what == kLoss ? 1 : (e.hessk ? e.n * (e.n + 1) / 2 : e.n);
  e.nout = what == kHess ? e.K : (what == kLoss ? 1 : e.n);
  e.N = N;
  e.streams = per_element(o.sampler) ? (uint64_t)e.K : 1;
  e.A = o.antithetic ? 2 : 1;
  e.NH = what == kHvp ? 2 : 1;
  e.R = e.streams * N * (uint64_t)e.A * (uint64_t)e.NH;
  // an HVP on a disk scene of at most 64 disks renders its +-h scenes as
  // pairs and yields one loss difference per (draw, a)
  e.pair = (what == kHvp && sc->kind == kDisks && sc->D <= raster_pair_max_disks() &&
            sc->W + sc->H <= raster_pair_max_side_sum() &&
            !o.hvp_per_render) ? 1 : 0;
  e.L = e.pair ? e.R / 2 : e.R;
  e.sigma = sigma;
  e.h = what == kHvp ? o.hvp_rel_step * sigma : 0.0;
  e.seed = seed;

  p->sc = sc;
  p->o = o;
  p->chunk = accum_chunk(e);
  p->nchunks = (N + p->chunk - 1) / p->chunk;
  p->stride = sc->kind == kDisks ? raster_subtiles(sc->W, sc->H)
              : sc->kind == kPT  ? pt_tiles(sc->W, sc->H)
                                 : 0;
  p->b_tau = align256(e.streams * N * (uint64_t)e.n * 8);
  p->b_u = align256((size_t)e.n * 8 + 8);
  // render pairs build their records in the kernel and write their loss
  // differences directly: no records, no partials
  p->b_rec = sc->kind == kDisks && !e.pair ? align256(e.R * (uint64_t)sc->D * 16) : 0;
  p->b_part = p->stride && !e.pair ? align256(part_floats(e.R, (uint64_t)p->stride) * 4) : 0;
  p->b_f = align256(e.L * 8);
  p->b_Fq = align256(e.streams * N * 8);
  p->b_vt = align256(N * 8);
  p->b_acc = align256(p->nchunks * (uint64_t)e.nout * 16);
  p->total = p->b_tau + p->b_u + p->b_rec + p->b_part + p->b_f + p->b_Fq + p->b_vt + p->b_acc;
  p->nout = what == kHess ? (size_t)e.n * e.n : (what == kLoss ? 1 : (size_t)e.n);
  return HR_OK;
}

QueryBufs carve(const QueryPlan& p, void* base) {
  QueryBufs b;
  char* c = (char*)base;
  b.tau = (double*)c; c += p.b_tau;
  b.u = (double*)c;
  b.vnorm = b.u + p.e.n;
  c += p.b_u;
  b.rec = (float4*)c; c += p.b_rec;
  b.partial = (float*)c; c += p.b_part;
  b.f = (double*)c; c += p.b_f;
  b.Fq = (double*)c; c += p.b_Fq;
  b.vt = (double*)c; c += p.b_vt;
  b.acc = (void*)c;
  return b;
}

void launch_query(hr_ctx* ctx, hipStream_t s, const QueryPlan& pl, const QueryBufs& qb,
                  const double* d_theta, const double* d_v, double* d_out, int S, int shape,
                  bool timing, bool keep_draws) {
  const hr_scene* sc = pl.sc;
  const hr_opts& o = pl.o;
  const EstShape& e = pl.e;
  const int chunk = pl.chunk;
  const int tiles = pl.stride;
  const int what = e.what;
  auto T = [&](const char* name, auto&& fn) {
    if (timing) timed(ctx, name, fn);
    else fn();
  };
  double* tau = qb.tau;
  double* u = qb.u;
  double* vnorm = qb.vnorm;
  float4* rec = qb.rec;
  float* partial = qb.partial;
  double* f = qb.f;
  double* Fq = qb.Fq;
  double* vt = qb.vt;
  void* acc = qb.acc;

  if (what == kHvp || what == kHvpLimit)
    T("sample", [&] { launch_sample_vnorm(s, e, tau, d_v, u, vnorm, !keep_draws); });
  else
    T("sample", [&] { launch_sample(s, e, tau); });
  const int spb = S;
  if (sc->kind == kDisks) {
    DiskScene ds{sc->W, sc->H, sc->C, sc->D, sc->ppd, sc->target, sc->colors, sc->radius};
    RasterExact ex{d_theta, tau, u, sc->radius, e.n, sc->ppd, e.A, e.NH, e.h};
    const double scale = 1.0 / ((double)sc->W * sc->H * sc->C);
    if (e.pair) {
      const PairQuery pq{d_theta, tau, u, sc->radius, sc->colors, sc->target, f,
                         sc->W, sc->H, sc->C, sc->D, sc->ppd, e.n, e.A, 0,
                         e.h, scale, e.L, e.skip};
      T("raster_dloss", [&] { launch_raster_dloss(s, pq); });
    } else {
      T("records", [&] { launch_records(s, e, ds, d_theta, tau, u, rec); });
      T("raster_loss", [&] {
        launch_raster_loss(s, ds, rec, e.R, spb, shape, ex, partial, e.skip);
      });
      T("tile_reduce", [&] { launch_tile_reduce(s, partial, e.R, tiles, scale, f, e.skip); });
    }
  } else if (sc->kind == kPT) {
    PTScene ps{sc->W, sc->H, sc->spp, sc->nspheres, sc->target, sc->pt_desc.data(), sc->ptc};
    T("pt_loss", [&] { launch_pt_loss(s, e, ps, d_theta, tau, u, spb, partial); });
    T("tile_reduce", [&] {
      launch_tile_reduce(s, partial, e.R, tiles, 1.0 / ((double)sc->W * sc->H * 3.0), f, e.skip);
    });
  } else {
    AnalyticScene as{sc->kind == kQuad ? 0 : 1, sc->n, sc->A, sc->b, sc->c, sc->s1};
    launch_analytic(s, e, as, d_theta, tau, u, f);
  }
  T("prep", [&] { launch_prep(s, e, f, tau, vnorm, d_v, Fq, vt); });
  T("accumulate", [&] { launch_accum(s, e, tau, Fq, vt, d_v, o.accum_fp64, acc, chunk); });
  launch_finalize(s, e, acc, o.accum_fp64, chunk, d_out);
}

}  // namespace rt
}  // namespace hr

namespace {

void release_scene_memory(hr_scene* sc) {
  if (sc->target) (void)hipFree(sc->target);
  if (sc->colors) (void)hipFree(sc->colors);
  if (sc->radius) (void)hipFree(sc->radius);
  if (sc->A) (void)hipFree(sc->A);
  if (sc->b) (void)hipFree(sc->b);
  if (sc->ptc) (void)hipFree(sc->ptc);
  sc->target = sc->colors = sc->radius = nullptr;
  sc->A = sc->b = nullptr;
  sc->ptc = nullptr;
}

// the estimator pipeline on device pointers; with `skip` (a device flag) every
// kernel of the query returns at once when the flag reads nonzero
const char* est_range(int what) {
  switch (what) {
    case kGrad: return "hr_est grad";
    case kHess: return "hr_est hessian";
    case kHvp: return "hr_est hvp";
    case kHvpLimit: return "hr_est hvp_limit";
    default: return "hr_est loss";
  }
}

// keep_draws: an HVP whose draws the previous query of the same plan left in
// the workspace (the products of one CG solve share their seed)
hr_status run_est(hr_scene* sc, int what, const double* d_theta, double sigma, uint64_t N,
                  uint64_t seed, const double* d_v, const hr_opts& o_in, double* d_out,
                  double* h_dbg, double* h_tau, const int* skip = nullptr,
                  bool keep_draws = false) {
  TraceRange range(est_range(what));
  QueryPlan pl;
  hr_status st = plan_query(sc, what, sigma, N, seed, d_v != nullptr, o_in, &pl);
  if (st) return st;
  pl.e.skip = skip;
  hr_ctx* ctx = sc->ctx;
  const hr_opts& o = pl.o;
  const EstShape& e = pl.e;
  N = e.N;
  (void)what;
  HR_HIP(hipSetDevice(ctx->device));
  (void)hipGetLastError();   // launch checks below report this call's errors only
  if (pl.total > ctx->budget)
    return fail(HR_ENOMEM, "request needs " + std::to_string(pl.total) +
                               " bytes of workspace, budget is " + std::to_string(ctx->budget));
  void* const ws_before = ctx->ws;
  st = ensure(ctx, &ctx->ws, &ctx->ws_bytes, pl.total);
  if (st) return st;
  if (ctx->ws != ws_before) keep_draws = false;   // a new workspace holds no draws
  const QueryBufs qb = carve(pl, ctx->ws);
  hipStream_t s = ctx->stream;
  launch_query(ctx, s, pl, qb, d_theta, d_v, d_out, o.samples_per_block, o.raster_tile, true,
               keep_draws);
  double* tau = qb.tau;
  double* f = qb.f;
  HR_HIP(hipGetLastError());
  if (h_dbg) HR_HIP(hipMemcpyAsync(h_dbg, f, e.L * 8, hipMemcpyDeviceToHost, s));
  if (h_tau) HR_HIP(hipMemcpyAsync(h_tau, tau, e.streams * N * (uint64_t)e.n * 8, hipMemcpyDeviceToHost, s));
  if (h_dbg || h_tau) HR_HIP(hipStreamSynchronize(s));
  return HR_OK;
}

// host-pointer wrapper: stage theta / v, run, copy the result back
hr_status run_host(hr_scene* sc, int what, const double* theta, double sigma, uint64_t N,
                   uint64_t seed, const double* v, const hr_opts* opts, double* out) {
  if (!sc || !theta || !out) return fail(HR_EINVAL, "NULL argument");
  if (!sc->ctx) return fail(HR_EINVAL, "the scene's context has been destroyed");
  const int n = sc->n;
  if (!finite_all(theta, n)) return fail(HR_EINVAL, "theta has a non-finite entry");
  if (what == kHvp || what == kHvpLimit) {
    if (!v) return fail(HR_EINVAL, "v is NULL");
    if (!finite_all(v, n)) return fail(HR_EINVAL, "v has a non-finite entry");
  }
  hr_opts o = resolve(opts);
  hr_ctx* ctx = sc->ctx;
  HR_HIP(hipSetDevice(ctx->device));
  const size_t nout = what == kHess ? (size_t)n * n : (what == kLoss ? 1 : (size_t)n);
  if (what == kHvp || what == kHvpLimit) {
    bool zero = true;
    for (int i = 0; i < n; ++i) zero = zero && v[i] == 0.0;
    if (zero && sigma > 0.0 && std::isfinite(sigma) && N > 0 && N < 0xFFFFFFFFull) {
      for (size_t i = 0; i < nout; ++i) out[i] = 0.0;
      return HR_OK;
    }
  }
  const size_t bytes = (2 * (size_t)n + nout) * 8;
  hr_status st = ensure(ctx, &ctx->stage, &ctx->stage_bytes, bytes);
  if (!st) st = ensure_host(ctx, &ctx->hstage, &ctx->hstage_bytes, bytes);
  if (st) return st;
  // theta and v go up, and the result comes down, through the pinned mirror
  // (the previous call's copies have completed: every call ends synchronised)
  double* h_in = (double*)ctx->hstage;
  double* d_theta = (double*)ctx->stage;
  double* d_v = d_theta + n;
  double* d_out = d_v + n;
  memcpy(h_in, theta, (size_t)n * 8);
  if (v) memcpy(h_in + n, v, (size_t)n * 8);
  HR_HIP(hipMemcpyAsync(d_theta, h_in, (size_t)n * (v ? 16 : 8), hipMemcpyHostToDevice,
                        ctx->stream));
  st = run_est(sc, what, d_theta, sigma, N, seed, v ? d_v : nullptr, o, d_out, o.dbg_loss, o.dbg_tau);
  if (st) return st;
  double* h_out = h_in + 2 * (size_t)n;
  HR_HIP(hipMemcpyAsync(h_out, d_out, nout * 8, hipMemcpyDeviceToHost, ctx->stream));
  HR_HIP(hipStreamSynchronize(ctx->stream));
  memcpy(out, h_out, nout * 8);
  return HR_OK;
}

}  // namespace

extern "C" {

void hr_opts_default(hr_opts* o) {
  if (!o) return;
  o->sampler = HR_AIS;
  o->antithetic = 1;
  o->hvp_rel_step = 0.1;
  o->accum_fp64 = 0;
  o->samples_per_block = 0;
  o->raster_tile = 0;
  o->dbg_loss = nullptr;
  o->dbg_tau = nullptr;
  o->hess_mix_n2 = 0;
  o->hvp_per_render = 0;
}

void hr_ncg_opts_default(hr_ncg_opts* o) {
  if (!o) return;
  o->cg_iters = 10;
  o->trust_radius = 1.0;
  o->use_full_hessian = 0;
  o->eig_floor = 1e-6;
  o->hvp_limit = 0;
  o->modified = 0;
}

const char* hr_last_error(void) { return error_slot().c_str(); }

hr_status hr_ctx_create(int device, hr_ctx** out) {
  if (!out) return fail(HR_EINVAL, "out is NULL");
  if (device < 0) return fail(HR_EINVAL, "negative device index");
  int count = 0;
  HR_HIP(hipGetDeviceCount(&count));
  if (device >= count) return fail(HR_EINVAL, "no such device");
  HR_HIP(hipSetDevice(device));
  // this device's copy of the fixed workspace (hr_est_hvp_dev_noalloc)
  hr_status sst = scratch_resolve(device);
  if (sst) return sst;
  hr_ctx* c = new hr_ctx();
  c->device = device;
  hipError_t e = hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete c;
    return fail(HR_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
  }
  c->stream = c->own;
  *out = c;
  return HR_OK;
}

void hr_ctx_destroy(hr_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  (void)drain_timers(ctx);
  for (hr_scene* sc : ctx->scenes) {   // scenes left alive are orphaned
    release_scene_memory(sc);
    sc->ctx = nullptr;
  }
  ctx->scenes.clear();
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->stage) (void)hipFree(ctx->stage);
  if (ctx->hstage) (void)hipHostFree(ctx->hstage);
  if (ctx->newton_graph.exec) (void)hipGraphExecDestroy(ctx->newton_graph.exec);
  if (ctx->cg) (void)hipFree(ctx->cg);
  if (ctx->own) (void)hipStreamDestroy(ctx->own);
  delete ctx;
}

hr_status hr_ctx_set_stream(hr_ctx* ctx, void* stream) {
  if (!ctx) return fail(HR_EINVAL, "ctx is NULL");
  ctx->stream = stream ? (hipStream_t)stream : ctx->own;
  return HR_OK;
}

hr_status hr_ctx_set_memory_budget(hr_ctx* ctx, uint64_t bytes) {
  if (!ctx || bytes == 0) return fail(HR_EINVAL, "bad budget");
  ctx->budget = bytes;
  return HR_OK;
}

hr_status hr_ctx_synchronize(hr_ctx* ctx) {
  if (!ctx) return fail(HR_EINVAL, "ctx is NULL");
  HR_HIP(hipSetDevice(ctx->device));
  HR_HIP(hipStreamSynchronize(ctx->stream));
  return HR_OK;
}

hr_status hr_ctx_enable_timing(hr_ctx* ctx, int enable) {
  if (!ctx) return fail(HR_EINVAL, "ctx is NULL");
  ctx->timing = enable != 0;
  return HR_OK;
}

hr_status hr_ctx_kernel_stats(hr_ctx* ctx, const char* name, uint64_t* launches, double* total_ms) {
  if (!ctx || !name) return fail(HR_EINVAL, "NULL argument");
  hr_status st = drain_timers(ctx);
  if (st) return st;
  auto it = ctx->stats.find(name);
  if (launches) *launches = it == ctx->stats.end() ? 0 : it->second.first;
  if (total_ms) *total_ms = it == ctx->stats.end() ? 0.0 : it->second.second;
  return HR_OK;
}

hr_status hr_ctx_reset_stats(hr_ctx* ctx) {
  if (!ctx) return fail(HR_EINVAL, "ctx is NULL");
  hr_status st = drain_timers(ctx);
  ctx->stats.clear();
  return st;
}

// ---------------------------------------------------------- device memory
hr_status hr_dev_alloc(hr_ctx* ctx, size_t bytes, void** out) {
  if (!ctx || !out || bytes == 0) return fail(HR_EINVAL, "bad allocation request");
  HR_HIP(hipSetDevice(ctx->device));
  hipError_t e = hipMalloc(out, bytes);
  if (e != hipSuccess) {
    *out = nullptr;
    (void)hipGetLastError();
    return fail(HR_ENOMEM, "device allocation failed");
  }
  return HR_OK;
}

hr_status hr_dev_free(hr_ctx* ctx, void* ptr) {
  if (!ctx) return fail(HR_EINVAL, "ctx is NULL");
  if (!ptr) return HR_OK;
  HR_HIP(hipSetDevice(ctx->device));
  HR_HIP(hipStreamSynchronize(ctx->stream));
  HR_HIP(hipFree(ptr));
  return HR_OK;
}

hr_status hr_memcpy(hr_ctx* ctx, void* dst, const void* src, size_t bytes, int kind) {
  if (!ctx || (!dst && bytes) || (!src && bytes)) return fail(HR_EINVAL, "NULL argument");
  if (kind < 0 || kind > 2) return fail(HR_EINVAL, "kind must be 0, 1 or 2");
  if (bytes == 0) return HR_OK;
  HR_HIP(hipSetDevice(ctx->device));
  const hipMemcpyKind k = kind == 0 ? hipMemcpyHostToDevice
                          : kind == 1 ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  HR_HIP(hipMemcpyAsync(dst, src, bytes, k, ctx->stream));
  HR_HIP(hipStreamSynchronize(ctx->stream));
  return HR_OK;
}

// ---------------------------------------------------------------- scenes
static hr_status upload(const void* src, size_t bytes, void** dst) {
  HR_HIP(hipMalloc(dst, bytes));
  HR_HIP(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
  return HR_OK;
}

hr_status hr_scene_disks(hr_ctx* ctx, int W, int H, int C, int D, int ppd, const float* radius,
                         const float* colors, const float* target, hr_scene** out) {
  if (!ctx || !out || !colors || !target) return fail(HR_EINVAL, "NULL argument");
  if (W <= 0 || H <= 0 || W > 16384 || H > 16384) return fail(HR_EINVAL, "bad image size");
  if (C < 1 || C > 4) return fail(HR_EINVAL, "channels must be 1..4");
  if (D < 1 || D > 1024) return fail(HR_EINVAL, "disk count must be 1..1024");
  if (ppd != 2 && ppd != 3) return fail(HR_EINVAL, "params_per_disk must be 2 or 3");
  if (ppd == 2 && !radius) return fail(HR_EINVAL, "radius is NULL");
  HR_HIP(hipSetDevice(ctx->device));
  hr_scene* sc = new hr_scene();
  sc->ctx = ctx;
  sc->kind = kDisks;
  sc->W = W; sc->H = H; sc->C = C; sc->D = D; sc->ppd = ppd;
  sc->n = D * ppd;
  hr_status st = upload(target, (size_t)W * H * C * 4, (void**)&sc->target);
  if (!st) st = upload(colors, (size_t)D * C * 4, (void**)&sc->colors);
  if (!st && ppd == 2) {
    st = upload(radius, (size_t)D * 4, (void**)&sc->radius);
    sc->hradius.assign(radius, radius + D);
  }
  if (st) { hr_scene_destroy(sc); return st; }
  ctx->scenes.insert(sc);
  *out = sc;
  return HR_OK;
}

hr_status hr_scene_pt(hr_ctx* ctx, int W, int H, int spp, int nspheres, const double* desc,
                      const float* target, hr_scene** out) {
  if (!ctx || !out || !desc || !target) return fail(HR_EINVAL, "NULL argument");
  if (W <= 0 || H <= 0 || W > 8192 || H > 8192) return fail(HR_EINVAL, "bad image size");
  if (spp < 1 || spp > 65536) return fail(HR_EINVAL, "spp must be 1..65536");
  if (nspheres < 1 || nspheres > 16) return fail(HR_EINVAL, "nspheres must be 1..16");
  if (!finite_all(desc, 12 + 7 * (size_t)nspheres)) return fail(HR_EINVAL, "non-finite description");
  HR_HIP(hipSetDevice(ctx->device));
  hr_scene* sc = new hr_scene();
  sc->ctx = ctx;
  sc->kind = kPT;
  sc->W = W; sc->H = H; sc->C = 3; sc->spp = spp; sc->nspheres = nspheres;
  sc->n = 6;
  // camera basis in FP64, stored as FP32: fwd = unit(look - eye),
  // right = unit(fwd x (0,1,0)), up = right x fwd
  double f[3] = {desc[3] - desc[0], desc[4] - desc[1], desc[5] - desc[2]};
  double fl = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  for (double& x : f) x /= fl;
  double r[3] = {-f[2], 0.0, f[0]};   // fwd x (0,1,0)
  double rl = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  for (double& x : r) x /= rl;
  double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
  const double th = std::tan(0.5 * desc[6] * 3.14159265358979323846 / 180.0);
  std::vector<float>& d = sc->pt_desc;
  d.assign(23 + 7 * nspheres, 0.0f);
  for (int i = 0; i < 12; ++i) d[i] = (float)desc[i];
  for (int i = 0; i < 3; ++i) {
    d[12 + i] = (float)f[i];
    d[15 + i] = (float)r[i];
    d[18 + i] = (float)u[i];
  }
  d[21] = (float)(th * (double)W / (double)H);
  d[22] = (float)th;
  for (int i = 0; i < 7 * nspheres; ++i) d[23 + i] = (float)desc[12 + i];
  hr_status st = upload(target, (size_t)W * H * 3 * 4, (void**)&sc->target);
  if (!st) {
    // the path tracer's constants, resident for the batch kernels
    const PTScene ps{W, H, spp, nspheres, sc->target, d.data(), nullptr};
    std::vector<char> pc(pt_const_bytes());
    pt_fill_const(ps, pc.data());
    st = upload(pc.data(), pc.size(), &sc->ptc);
  }
  if (st) { hr_scene_destroy(sc); return st; }
  ctx->scenes.insert(sc);
  *out = sc;
  return HR_OK;
}

hr_status hr_scene_quad(hr_ctx* ctx, int n, const double* A, const double* b, double c,
                        hr_scene** out) {
  if (!ctx || !out || !A) return fail(HR_EINVAL, "NULL argument");
  if (n < 1 || n > 128) return fail(HR_EINVAL, "n must be 1..128");
  HR_HIP(hipSetDevice(ctx->device));
  hr_scene* sc = new hr_scene();
  sc->ctx = ctx;
  sc->kind = kQuad;
  sc->n = n;
  sc->c = c;
  std::vector<double> bb(n, 0.0);
  if (b) bb.assign(b, b + n);
  hr_status st = upload(A, (size_t)n * n * 8, (void**)&sc->A);
  if (!st) st = upload(bb.data(), (size_t)n * 8, (void**)&sc->b);
  if (st) { hr_scene_destroy(sc); return st; }
  ctx->scenes.insert(sc);
  *out = sc;
  return HR_OK;
}

hr_status hr_scene_neggauss(hr_ctx* ctx, int n, double s1, hr_scene** out) {
  if (!ctx || !out) return fail(HR_EINVAL, "NULL argument");
  if (n < 1 || n > 128 || !(s1 > 0.0) || !std::isfinite(s1)) return fail(HR_EINVAL, "bad negated-Gaussian scene");
  hr_scene* sc = new hr_scene();
  sc->ctx = ctx;
  sc->kind = kNegGauss;
  sc->n = n;
  sc->s1 = s1;
  ctx->scenes.insert(sc);
  *out = sc;
  return HR_OK;
}

void hr_scene_destroy(hr_scene* sc) {
  if (!sc) return;
  {
    // a server may still hold queries on the scene: they finish first
    std::unique_lock<std::mutex> lk(sc->hold_mu);
    sc->hold_cv.wait(lk, [&] { return sc->held == 0; });
  }
  if (sc->ctx) {   // an orphaned scene (context destroyed first) holds no memory
    (void)hipSetDevice(sc->ctx->device);
    (void)hipStreamSynchronize(sc->ctx->stream);
    release_scene_memory(sc);
    sc->ctx->scenes.erase(sc);
  }
  delete sc;
}

int hr_scene_nparams(const hr_scene* sc) { return sc ? sc->n : -1; }

hr_status hr_render(hr_scene* sc, const double* theta, uint64_t seed, uint32_t s, int spp,
                    float* image) {
  if (!sc || !theta || !image) return fail(HR_EINVAL, "NULL argument");
  if (!sc->ctx) return fail(HR_EINVAL, "the scene's context has been destroyed");
  if (sc->kind != kDisks && sc->kind != kPT) return fail(HR_EUNSUPPORTED, "analytic scenes have no image");
  TraceRange range("hr_render");
  if (!finite_all(theta, sc->n)) return fail(HR_EINVAL, "theta has a non-finite entry");
  hr_ctx* ctx = sc->ctx;
  HR_HIP(hipSetDevice(ctx->device));
  const size_t img = (size_t)sc->W * sc->H * sc->C * 4;
  hr_status st = ensure(ctx, &ctx->ws, &ctx->ws_bytes, align256(img) + (size_t)sc->n * 8);
  if (st) return st;
  float* d_img = (float*)ctx->ws;
  if (sc->kind == kDisks) {
    double* d_theta = (double*)((char*)ctx->ws + align256(img));
    HR_HIP(hipMemcpyAsync(d_theta, theta, (size_t)sc->n * 8, hipMemcpyHostToDevice, ctx->stream));
    DiskScene ds{sc->W, sc->H, sc->C, sc->D, sc->ppd, sc->target, sc->colors, sc->radius};
    RasterExact ex{d_theta, nullptr, nullptr, sc->radius, sc->n, sc->ppd, 1, 1, 0.0};
    launch_render_disks(ctx->stream, ds, ex, d_img);
  } else {
    PTScene ps{sc->W, sc->H, sc->spp, sc->nspheres, sc->target, sc->pt_desc.data(), sc->ptc};
    launch_pt_render(ctx->stream, ps, theta, seed, s, spp > 0 ? spp : sc->spp, d_img);
  }
  HR_HIP(hipGetLastError());
  HR_HIP(hipMemcpyAsync(image, d_img, img, hipMemcpyDeviceToHost, ctx->stream));
  HR_HIP(hipStreamSynchronize(ctx->stream));
  return HR_OK;
}

// ------------------------------------------------------------ estimators
hr_status hr_est_grad(hr_scene* sc, const double* theta, double sigma, uint64_t N, uint64_t seed,
                      const hr_opts* opts, double* g) {
  return run_host(sc, kGrad, theta, sigma, N, seed, nullptr, opts, g);
}
hr_status hr_est_hessian(hr_scene* sc, const double* theta, double sigma, uint64_t N,
                         uint64_t seed, const hr_opts* opts, double* H) {
  return run_host(sc, kHess, theta, sigma, N, seed, nullptr, opts, H);
}
hr_status hr_est_hvp(hr_scene* sc, const double* theta, double sigma, uint64_t N, uint64_t seed,
                     const double* v, const hr_opts* opts, double* Hv) {
  return run_host(sc, kHvp, theta, sigma, N, seed, v, opts, Hv);
}
hr_status hr_est_hvp_limit(hr_scene* sc, const double* theta, double sigma, uint64_t N,
                           uint64_t seed, const double* v, const hr_opts* opts, double* Hv) {
  return run_host(sc, kHvpLimit, theta, sigma, N, seed, v, opts, Hv);
}

hr_status hr_est_grad_dev(hr_scene* sc, const double* d_theta, double sigma, uint64_t N,
                          uint64_t seed, const hr_opts* opts, double* d_g) {
  if (!sc || !d_theta || !d_g) return fail(HR_EINVAL, "NULL argument");
  hr_opts o = resolve(opts);
  o.dbg_loss = nullptr;
  o.dbg_tau = nullptr;
  return run_est(sc, kGrad, d_theta, sigma, N, seed, nullptr, o, d_g, nullptr, nullptr);
}
hr_status hr_est_hessian_dev(hr_scene* sc, const double* d_theta, double sigma, uint64_t N,
                             uint64_t seed, const hr_opts* opts, double* d_H) {
  if (!sc || !d_theta || !d_H) return fail(HR_EINVAL, "NULL argument");
  hr_opts o = resolve(opts);
  o.dbg_loss = nullptr;
  o.dbg_tau = nullptr;
  return run_est(sc, kHess, d_theta, sigma, N, seed, nullptr, o, d_H, nullptr, nullptr);
}
hr_status hr_est_hvp_dev(hr_scene* sc, const double* d_theta, double sigma, uint64_t N,
                         uint64_t seed, const double* d_v, const hr_opts* opts, double* d_Hv) {
  if (!sc || !d_theta || !d_v || !d_Hv) return fail(HR_EINVAL, "NULL argument");
  hr_opts o = resolve(opts);
  o.dbg_loss = nullptr;
  o.dbg_tau = nullptr;
  return run_est(sc, kHvp, d_theta, sigma, N, seed, d_v, o, d_Hv, nullptr, nullptr);
}

hr_status hr_est_hvp_dev_noalloc(hr_scene* sc, const double* d_theta, double sigma, uint64_t N,
                                 uint64_t seed, const double* d_v, const hr_opts* opts,
                                 double* d_Hv) {
  if (!sc || !d_theta || !d_v || !d_Hv) return fail(HR_EINVAL, "NULL argument");
  TraceRange range("hr_est hvp noalloc");
  hr_opts o = resolve(opts);
  o.dbg_loss = nullptr;
  o.dbg_tau = nullptr;
  QueryPlan pl;
  hr_status st = plan_query(sc, kHvp, sigma, N, seed, true, o, &pl);
  if (st) return st;
  if (pl.total > kNoallocScratchBytes)
    return fail(HR_ENOMEM, "request needs " + std::to_string(pl.total) +
                               " bytes of workspace; the fixed workspace of this entry point holds " +
                               std::to_string(kNoallocScratchBytes));
  hr_ctx* ctx = sc->ctx;
  void* ws = scratch_of(ctx->device);
  if (!ws) return fail(HR_EDEVICE, "the fixed workspace is not resolved on this device");
  HR_HIP(hipSetDevice(ctx->device));
  (void)hipGetLastError();   // launch checks below report this call's errors only
  // every buffer of the query is written before it is read: nothing in the
  // workspace has to start at zero
  launch_query(ctx, ctx->stream, pl, carve(pl, ws), d_theta, d_v, d_Hv, o.samples_per_block,
               o.raster_tile, false);
  HR_HIP(hipGetLastError());
  return HR_OK;
}

hr_status hr_est_loss(hr_scene* sc, const double* theta, double sigma, uint64_t N, uint64_t seed,
                      const hr_opts* opts, double* F) {
  return run_host(sc, kLoss, theta, sigma, N, seed, nullptr, opts, F);
}

// ------------------------------------------------------------ grey-box
static hr_status run_greybox(hr_scene* sc, int what, const double* y, const double* J, int n_in,
                             double sigma, uint64_t N, uint64_t seed, const double* vx,
                             const hr_opts* opts, double* out) {
  if (!sc || !y || !J || !out || (what == kHvp && !vx)) return fail(HR_EINVAL, "NULL argument");
  if (n_in < 1 || n_in > 4096) return fail(HR_EINVAL, "n_in must be 1..4096");
  if (!sc->ctx) return fail(HR_EINVAL, "the scene's context has been destroyed");
  const int n = sc->n;
  if (!finite_all(y, n)) return fail(HR_EINVAL, "y has a non-finite entry");
  if (!finite_all(J, (size_t)n * n_in)) return fail(HR_EINVAL, "J has a non-finite entry");
  if (what == kHvp && !finite_all(vx, n_in)) return fail(HR_EINVAL, "vx has a non-finite entry");
  hr_opts o = resolve(opts);
  o.dbg_loss = nullptr;
  o.dbg_tau = nullptr;
  hr_ctx* ctx = sc->ctx;
  HR_HIP(hipSetDevice(ctx->device));
  const size_t nj = (size_t)n * n_in;
  const size_t nouty = what == kHess ? (size_t)n * n : (size_t)n;
  const size_t noutx = what == kHess ? (size_t)n_in * n_in : (size_t)n_in;
  const size_t need = (2 * (size_t)n + nj + n_in + nouty + nj + noutx) * 8;
  hr_status st = ensure(ctx, &ctx->stage, &ctx->stage_bytes, need);
  if (st) return st;
  double* d_y = (double*)ctx->stage;
  double* d_vy = d_y + n;
  double* d_J = d_vy + n;
  double* d_vx = d_J + nj;
  double* d_outy = d_vx + n_in;
  double* d_T = d_outy + nouty;
  double* d_outx = d_T + nj;
  hipStream_t s = ctx->stream;
  HR_HIP(hipMemcpyAsync(d_y, y, (size_t)n * 8, hipMemcpyHostToDevice, s));
  HR_HIP(hipMemcpyAsync(d_J, J, nj * 8, hipMemcpyHostToDevice, s));
  if (what == kHvp) {
    HR_HIP(hipMemcpyAsync(d_vx, vx, (size_t)n_in * 8, hipMemcpyHostToDevice, s));
    launch_j_vec(s, n, n_in, d_J, d_vx, d_vy);
  }
  st = run_est(sc, what, d_y, sigma, N, seed, what == kHvp ? d_vy : nullptr, o, d_outy, nullptr,
               nullptr);
  if (st) return st;
  if (what == kHess) launch_jt_h_j(s, n, n_in, d_J, d_outy, d_T, d_outx);
  else launch_jt_vec(s, n, n_in, d_J, d_outy, d_outx);
  HR_HIP(hipGetLastError());
  HR_HIP(hipMemcpyAsync(out, d_outx, noutx * 8, hipMemcpyDeviceToHost, s));
  HR_HIP(hipStreamSynchronize(s));
  return HR_OK;
}

hr_status hr_est_grad_greybox(hr_scene* sc, const double* y, const double* J, int n_in,
                              double sigma, uint64_t N, uint64_t seed, const hr_opts* opts,
                              double* gx) {
  return run_greybox(sc, kGrad, y, J, n_in, sigma, N, seed, nullptr, opts, gx);
}
hr_status hr_est_hessian_greybox(hr_scene* sc, const double* y, const double* J, int n_in,
                                 double sigma, uint64_t N, uint64_t seed, const hr_opts* opts,
                                 double* Hx) {
  return run_greybox(sc, kHess, y, J, n_in, sigma, N, seed, nullptr, opts, Hx);
}
hr_status hr_est_hvp_greybox(hr_scene* sc, const double* y, const double* J, int n_in,
                             double sigma, uint64_t N, uint64_t seed, const double* vx,
                             const hr_opts* opts, double* Hvx) {
  return run_greybox(sc, kHvp, y, J, n_in, sigma, N, seed, vx, opts, Hvx);
}

// ------------------------------------------------------------ Newton-CG
hr_status hr_newton_cg_step_dev(hr_scene* sc, double* d_theta, double sigma, uint64_t N,
                                uint64_t seed, const hr_ncg_opts* ncg, const hr_opts* opts,
                                hr_ncg_report* report) {
  if (!sc || !d_theta) return fail(HR_EINVAL, "NULL argument");
  if (!sc->ctx) return fail(HR_EINVAL, "the scene's context has been destroyed");
  TraceRange range("hr_newton_cg_step");
  hr_ncg_opts no;
  hr_ncg_opts_default(&no);
  if (ncg) no = *ncg;
  if (!(no.trust_radius > 0.0) || !std::isfinite(no.trust_radius))
    return fail(HR_EINVAL, "trust_radius must be positive");
  if (no.cg_iters < 0 || no.cg_iters > 10000) return fail(HR_EINVAL, "cg_iters out of range");
  if (!(no.eig_floor >= 0.0)) return fail(HR_EINVAL, "eig_floor must be >= 0");
  hr_opts o = resolve(opts);
  o.dbg_loss = nullptr;
  o.dbg_tau = nullptr;
  hr_ctx* ctx = sc->ctx;
  HR_HIP(hipSetDevice(ctx->device));
  const int n = sc->n;
  const size_t nv = align256((size_t)n * 8);
  const size_t need = 5 * nv + align256((size_t)n * n * 8) * 3 + align256(sizeof(CgState));
  hr_status st = ensure(ctx, &ctx->cg, &ctx->cg_bytes, need);
  if (st) return st;
  // the estimates' workspace is sized before the step is enqueued, so that
  // nothing inside the step allocates (or synchronises to free)
  {
    const int prod = no.use_full_hessian ? kHess : (no.hvp_limit ? kHvpLimit : kHvp);
    QueryPlan pg, pp;
    st = plan_query(sc, kGrad, sigma, N, seed, false, o, &pg);
    if (!st) st = plan_query(sc, prod, sigma, N, seed, true, o, &pp);
    if (st) return st;
    const size_t ws = pg.total > pp.total ? pg.total : pp.total;
    if (ws > ctx->budget)
      return fail(HR_ENOMEM, "request needs " + std::to_string(ws) +
                                 " bytes of workspace, budget is " + std::to_string(ctx->budget));
    st = ensure(ctx, &ctx->ws, &ctx->ws_bytes, ws);
    if (st) return st;
  }
  char* p = (char*)ctx->cg;
  double* g = (double*)p; p += nv;
  double* r = (double*)p; p += nv;
  double* pv = (double*)p; p += nv;
  double* d = (double*)p; p += nv;
  double* Hp = (double*)p; p += nv;
  double* Hm = (double*)p; p += align256((size_t)n * n * 8);
  double* work = (double*)p; p += 2 * align256((size_t)n * n * 8);
  CgState* cs = (CgState*)p;
  hipStream_t s = ctx->stream;

  // The step is enqueued without a host round trip: every CG product is
  // launched, and once the inner loop has stopped (the state's stop flag, set
  // on the device) each later product's kernels and update return at once.
  auto enqueue_step = [&]() -> hr_status {
    hr_status e = run_est(sc, kGrad, d_theta, sigma, N, seed, nullptr, o, g, nullptr, nullptr);
    if (e) return e;
    if (no.use_full_hessian) {
      e = run_est(sc, kHess, d_theta, sigma, N, seed, nullptr, o, Hm, nullptr, nullptr);
      if (e) return e;
      launch_newton_full(s, n, Hm, g, no.trust_radius, no.eig_floor, work, d, cs);
    } else {
      launch_cg_init(s, n, g, no.trust_radius, no.modified, no.eig_floor, r, pv, d, cs);
      // every product draws with the same seed, so the first product's draws
      // stay in the workspace for the others (nothing between them writes it)
      for (int k = 0; k < no.cg_iters; ++k) {
        e = run_est(sc, no.hvp_limit ? kHvpLimit : kHvp, d_theta, sigma, N, seed, pv, o, Hp,
                    nullptr, nullptr, &cs->stop, k > 0);
        if (e) return e;
        launch_cg_update(s, n, Hp, r, pv, d, cs);
      }
    }
    launch_cg_apply(s, n, d, d_theta, cs);
    HR_HIP(hipGetLastError());
    return HR_OK;
  };

  // A step repeated with the same arguments and buffers is replayed as one
  // hipGraph: the first run is eager, the second is captured, later ones
  // replay it (kernel timers, when on, keep every run eager).
  std::vector<char> key;
  auto put = [&](const void* x, size_t b) {
    key.insert(key.end(), (const char*)x, (const char*)x + b);
  };
  put(&sc->uid, sizeof(sc->uid));
  put(&d_theta, sizeof(d_theta));
  put(&sigma, sizeof(sigma));
  put(&N, sizeof(N));
  put(&seed, sizeof(seed));
  put(&no, sizeof(no));
  put(&o, sizeof(o));
  put(&ctx->ws, sizeof(ctx->ws));
  put(&ctx->ws_bytes, sizeof(ctx->ws_bytes));
  put(&ctx->cg, sizeof(ctx->cg));
  put(&ctx->cg_bytes, sizeof(ctx->cg_bytes));
  put(&s, sizeof(s));
  NewtonGraph& G = ctx->newton_graph;
  const bool same = !ctx->timing && key == G.key;
  if (same && G.exec) {
    HR_HIP(hipGraphLaunch(G.exec, s));
  } else if (same && G.runs >= 1) {
    hipGraph_t graph = nullptr;
    HR_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const hr_status est = enqueue_step();
    const hipError_t ee = hipStreamEndCapture(s, &graph);
    if (est || ee != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipGetLastError();
      G.runs = -1;   // this step does not capture: stay eager
      if (est) return est;
      st = enqueue_step();
      if (st) return st;
    } else {
      const hipError_t ie = hipGraphInstantiate(&G.exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ie != hipSuccess) {
        G.exec = nullptr;
        return fail(HR_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
      }
      HR_HIP(hipGraphLaunch(G.exec, s));
    }
  } else {
    if (G.exec) {
      (void)hipGraphExecDestroy(G.exec);
      G.exec = nullptr;
    }
    st = enqueue_step();
    if (st) return st;
    if (!same) {
      G.key = key;
      G.runs = ctx->timing ? 0 : 1;
    }
  }
  if (report) {
    CgState h{};
    HR_HIP(hipMemcpyAsync(&h, cs, sizeof(CgState), hipMemcpyDeviceToHost, s));
    HR_HIP(hipStreamSynchronize(s));
    report->iters_done = h.iters;
    report->hit_trust = h.hit_trust;
    report->neg_curv = h.neg_curv;
    report->step_norm = h.step_norm;
    report->g_norm = h.gnorm;
  }
  return HR_OK;
}

void hr_optim_opts_default(hr_optim_opts* o) {
  if (!o) return;
  o->iters = 10;
  o->sigma_start = 0.1;
  o->sigma_end = 0.01;
  o->method = HR_OPT_NEWTON_CG;
  o->lr = 0.1;
  o->ls_iters = 0;
  o->ls_tol = 1e-3;
  o->recompute = 1;
  o->N_loss = 1024;
  hr_ncg_opts_default(&o->ncg);
}

// Outer loop of the optimiser.  Every estimate and Newton/CG solve runs in
// the library's kernels; the O(n) update theta += alpha d is done here in FP64.
hr_status hr_optimize(hr_scene* sc, double* theta, uint64_t N, uint64_t seed,
                      const hr_optim_opts* oo_in, const hr_opts* opts, double* trace) {
  if (!sc || !theta) return fail(HR_EINVAL, "NULL argument");
  if (!sc->ctx) return fail(HR_EINVAL, "the scene's context has been destroyed");
  TraceRange range("hr_optimize");
  hr_optim_opts oo;
  hr_optim_opts_default(&oo);
  if (oo_in) oo = *oo_in;
  if (oo.iters < 1 || oo.recompute < 1 || oo.ls_iters < 0) return fail(HR_EINVAL, "bad iteration counts");
  if (!(oo.sigma_start > 0.0) || !(oo.sigma_end > 0.0)) return fail(HR_EINVAL, "sigma schedule must be positive");
  if (oo.method < 0 || oo.method > 2) return fail(HR_EINVAL, "unknown method");
  if (oo.ls_iters > 0 && oo.N_loss == 0) return fail(HR_EINVAL, "N_loss must be positive");
  const int n = sc->n;
  if (!finite_all(theta, n)) return fail(HR_EINVAL, "theta has a non-finite entry");
  std::vector<double> d(n), trial(n);
  double alpha_keep = 1.0;
  hr_status st = HR_OK;
  for (int t = 0; t < oo.iters; ++t) {
    const double sg = oo.iters > 1
                          ? oo.sigma_start + (oo.sigma_end - oo.sigma_start) * t / (double)(oo.iters - 1)
                          : oo.sigma_start;
    const uint64_t sd = seed + (uint64_t)t;
    if (oo.method == HR_OPT_GD) {
      st = hr_est_grad(sc, theta, sg, N, sd, opts, d.data());
      if (st) return st;
      for (int i = 0; i < n; ++i) d[i] = -oo.lr * d[i];
    } else {
      hr_ncg_opts no = oo.ncg;
      no.use_full_hessian = oo.method == HR_OPT_NEWTON_FULL;
      trial.assign(theta, theta + n);
      st = hr_newton_cg_step(sc, trial.data(), sg, N, sd, &no, opts, nullptr);
      if (st) return st;
      for (int i = 0; i < n; ++i) d[i] = trial[i] - theta[i];
    }
    double alpha = 1.0;
    if (oo.ls_iters > 0) {
      if (t % oo.recompute == 0) {
        double F0, F1;
        st = hr_est_loss(sc, theta, sg, oo.N_loss, sd, opts, &F0);
        if (st) return st;
        bool ok = false;
        for (int k = 0; k < oo.ls_iters; ++k) {
          for (int i = 0; i < n; ++i) trial[i] = theta[i] + alpha * d[i];
          st = hr_est_loss(sc, trial.data(), sg, oo.N_loss, sd, opts, &F1);
          if (st) return st;
          if (F1 <= F0 - oo.ls_tol * std::fabs(F0)) { ok = true; break; }
          alpha *= 0.5;
        }
        if (!ok) alpha = 0.0;   // no decrease found: stay
        alpha_keep = alpha;
      } else {
        alpha = alpha_keep;
      }
    }
    double sn = 0.0;
    for (int i = 0; i < n; ++i) {
      theta[i] += alpha * d[i];
      sn += (alpha * d[i]) * (alpha * d[i]);
    }
    if (trace) {
      double Fs = 0.0, f = 0.0;
      st = hr_est_loss(sc, theta, sg, oo.N_loss > 0 ? oo.N_loss : N, sd, opts, &Fs);
      if (!st) st = hr_est_loss(sc, theta, 0.0, 1, sd, opts, &f);
      if (st) return st;
      double* row = trace + 5 * (size_t)t;
      row[0] = sg; row[1] = alpha; row[2] = std::sqrt(sn); row[3] = Fs; row[4] = f;
    }
  }
  return HR_OK;
}

hr_status hr_newton_cg_step(hr_scene* sc, double* theta, double sigma, uint64_t N, uint64_t seed,
                            const hr_ncg_opts* ncg, const hr_opts* opts, hr_ncg_report* report) {
  if (!sc || !theta) return fail(HR_EINVAL, "NULL argument");
  if (!sc->ctx) return fail(HR_EINVAL, "the scene's context has been destroyed");
  const int n = sc->n;
  if (!finite_all(theta, n)) return fail(HR_EINVAL, "theta has a non-finite entry");
  hr_ctx* ctx = sc->ctx;
  HR_HIP(hipSetDevice(ctx->device));
  hr_status st = ensure(ctx, &ctx->stage, &ctx->stage_bytes, (size_t)n * 8 * 3 + (size_t)n * n * 8);
  if (st) return st;
  double* d_theta = (double*)ctx->stage;
  HR_HIP(hipMemcpyAsync(d_theta, theta, (size_t)n * 8, hipMemcpyHostToDevice, ctx->stream));
  st = hr_newton_cg_step_dev(sc, d_theta, sigma, N, seed, ncg, opts, report);
  if (st) return st;
  HR_HIP(hipMemcpyAsync(theta, d_theta, (size_t)n * 8, hipMemcpyDeviceToHost, ctx->stream));
  HR_HIP(hipStreamSynchronize(ctx->stream));
  return HR_OK;
}

}  // extern "C"
