// hr_batch.hip -- batched execution of uneven estimator queries.
//
// A batch of queries (any mix of scenes, kinds, sizes and sample budgets)
// runs as one fixed sequence of launches: one phase kernel per pipeline step
// (draws, disk records, analytic renders, tile reduction, per-draw weights,
// lobe accumulation, finalisation), each walking a task list built on the
// host, and two persistent render kernels (rasteriser and path tracer) that
// pull (query, chunk, tile) items from eight per-XCD work queues.  All
// per-batch data -- the task lists, the queue segments, every query's shape
// and buffers, theta and v -- lives in one device table uploaded with one
// copy, so the launch sequence never changes and is replayed as a hipGraph.
//
// Every kernel body is the one the single-query entry points use, so a
// query's result is the same bits alone and in any batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "hr_batch.h"

using namespace hr;
using namespace hr::rt;

namespace hr {
namespace rt {

namespace {

constexpr int kPhaseBlocksPerCU = 8;
constexpr int kDefaultPtSamples = 8;

uint64_t lg2(int v) {
  uint64_t b = 0;
  while ((1 << (b + 1)) <= v) ++b;
  return b;
}

// class of a raster query for the autotuner: channels, disk-count bucket,
// image-size buckets
uint64_t tune_key(const hr_scene* sc) {
  return ((uint64_t)sc->C << 24) | (lg2(sc->D) << 16) | (lg2(sc->W) << 8) | lg2(sc->H);
}

// class of a path-traced query: renders per draw, samples per pixel, sphere
// count, image-size buckets (bit 40 keeps it apart from the raster classes)
uint64_t pt_tune_key(const hr_scene* sc, int nr) {
  return (1ull << 40) | ((uint64_t)nr << 32) | ((uint64_t)sc->spp << 24) |
         ((uint64_t)sc->nspheres << 16) | (lg2(sc->W) << 8) | lg2(sc->H);
}

// draws per block item of a path-traced query: the explicit option, then the
// autotuner's choice for its class, then the default
int pt_samples(hr_ctx* ctx, const QueryPlan& p) {
  const hr_scene* sc = p.sc;
  if (p.o.samples_per_block > 0 && p.o.samples_per_block <= pt_max_samples())
    return p.o.samples_per_block;
  std::lock_guard<std::mutex> lk(ctx->tuned_mu);
  auto it = ctx->tuned.find(pt_tune_key(sc, p.e.A * p.e.NH));
  return it != ctx->tuned.end() ? it->second.first : kDefaultPtSamples;
}

}  // namespace

hr_status BatchSlot::init(hr_ctx* c) {
  ctx = c;
  HR_HIP(hipSetDevice(ctx->device));
  HR_HIP(hipStreamCreateWithFlags(&stream, hipStreamNonBlocking));
  HR_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
  hipDeviceProp_t prop;
  HR_HIP(hipGetDeviceProperties(&prop, ctx->device));
  cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
  phase_blocks = cus * kPhaseBlocksPerCU;
  for (int c = 0; c < 3; ++c) pt_blocks[c] = cus * batch_pt_blocks_per_cu(1 << c);
  return HR_OK;
}

void BatchSlot::release() {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  if (stream) (void)hipStreamSynchronize(stream);
  if (exec) (void)hipGraphExecDestroy(exec);
  if (dev) (void)hipFree(dev);
  if (host) (void)hipHostFree(host);
  if (ws) (void)hipFree(ws);
  if (done) (void)hipEventDestroy(done);
  if (stream) (void)hipStreamDestroy(stream);
  exec = nullptr;
  dev = host = ws = nullptr;
  done = nullptr;
  stream = nullptr;
  ctx = nullptr;
}

hr_status BatchSlot::reserve_workspace(size_t bytes) {
  if (bytes <= ws_bytes) return HR_OK;
  HR_HIP(hipSetDevice(ctx->device));
  if (ws) {
    HR_HIP(hipStreamSynchronize(stream));
    HR_HIP(hipFree(ws));
    ws = nullptr;
    ws_bytes = 0;
  }
  const size_t sz = align256(bytes);
  if (hipMalloc(&ws, sz) != hipSuccess) {
    ws = nullptr;
    (void)hipGetLastError();
    return fail(HR_ENOMEM, "batch workspace of " + std::to_string(sz) + " bytes");
  }
  ws_bytes = sz;
  return HR_OK;
}

hr_status BatchSlot::reserve_table(size_t bytes) {
  if (bytes <= table_bytes) return HR_OK;
  HR_HIP(hipSetDevice(ctx->device));
  HR_HIP(hipStreamSynchronize(stream));
  if (exec) {   // the captured launches point at the old table
    (void)hipGraphExecDestroy(exec);
    exec = nullptr;
  }
  if (dev) HR_HIP(hipFree(dev));
  if (host) HR_HIP(hipHostFree(host));
  dev = host = nullptr;
  table_bytes = 0;
  const size_t sz = align256(bytes + bytes / 2 + 4096);
  if (hipMalloc(&dev, sz) != hipSuccess) {
    dev = nullptr;
    (void)hipGetLastError();
    return fail(HR_ENOMEM, "batch table of " + std::to_string(sz) + " bytes");
  }
  if (hipHostMalloc(&host, sz, hipHostMallocDefault) != hipSuccess) {
    host = nullptr;
    (void)hipGetLastError();
    return fail(HR_ENOMEM, "pinned batch table of " + std::to_string(sz) + " bytes");
  }
  table_bytes = sz;
  return HR_OK;
}

// The raster configuration a query runs with: explicit options first, then
// the autotuner's choice for its class, then the defaults.
static void raster_config(hr_ctx* ctx, const hr_scene* sc, const hr_opts& o, uint64_t R,
                          int* S, int* shape) {
  *S = o.samples_per_block;
  *shape = o.raster_tile;
  {
    std::lock_guard<std::mutex> lk(ctx->tuned_mu);
    auto it = ctx->tuned.find(tune_key(sc));
    if (it != ctx->tuned.end()) {
      if (*S <= 0) *S = it->second.first;
      if (*shape <= 0) *shape = it->second.second;
    }
  }
  if (*shape < 0 || *shape > 3) *shape = 0;
  if (*S <= 0) *S = raster_auto_samples(sc->W, sc->H, R, *shape);
  if (*S > raster_max_samples()) *S = raster_max_samples();
}

hr_status BatchSlot::build(std::vector<BatchItem>& items) {
  const int nq = (int)items.size();
  nq_ = nq;
  // workspace: queries back to back
  size_t ws_need = 0;
  for (auto& it : items) {
    it.ws_off = ws_need;
    ws_need += align256(it.plan.total);
  }
  hr_status st = reserve_workspace(ws_need > 0 ? ws_need : 256);
  if (st) return st;

  // render work queues, items in decreasing cost (longest first)
  std::vector<int> order(nq);
  std::iota(order.begin(), order.end(), 0);
  std::vector<double> cost(nq, 0.0);
  std::vector<int> qS(nq, 0), qshape(nq, 0);
  lds = 0;
  lds_pair = 0;
  lds_pair32 = 0;
  for (int q = 0; q < nq; ++q) {
    const QueryPlan& p = items[q].plan;
    const hr_scene* sc = p.sc;
    if (sc->kind == kDisks) {
      raster_config(ctx, sc, p.o, p.e.R, &qS[q], &qshape[q]);
      cost[q] = (double)qS[q] * (double)(sc->D + 16);
      if (p.e.pair) {
        // pairs per block item: the block's four waves take one pair each at
        // a time; a few per wave for large queries, one for small ones, so
        // that every query spreads over many blocks
        qS[q] = p.o.samples_per_block > 0
                    ? std::max(4, p.o.samples_per_block / 2)
                    : (int)std::min<uint64_t>(32, std::max<uint64_t>(4, 4 * (p.e.L / 16384)));
        size_t& lp = sc->D <= 32 ? lds_pair32 : lds_pair;
        lp = std::max(lp, raster_pair_lds_bytes(sc->W, sc->H, sc->D));
      } else {
        lds = std::max(lds, raster_lds_bytes(sc->D, qS[q]));
      }
    } else if (sc->kind == kPT) {
      qS[q] = pt_samples(ctx, p);
      cost[q] = (double)qS[q] * p.e.A * p.e.NH * sc->spp;
    }
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });

  struct Q8 { std::vector<WorkSeg> seg[8]; uint64_t items[8] = {0, 0, 0, 0, 0, 0, 0, 0}; };
  Q8 rq[kRasterClasses], pq[3];   // raster queues by class, path-traced by renders per draw
  uint64_t rchunks[kRasterClasses] = {}, pchunks[3] = {0, 0, 0};
  auto add_segments = [](Q8& Qs, uint64_t& cbase, int q, uint64_t chunks, int tiles) {
    for (int x = 0; x < 8; ++x) {
      const int c0 = (int)(((uint64_t)x + 8u - (cbase & 7u)) & 7u);
      if ((uint64_t)c0 >= chunks) continue;
      const uint64_t nch = (chunks - 1 - (uint64_t)c0) / 8 + 1;
      WorkSeg s{Qs.items[x], q, c0, tiles, 0};
      Qs.seg[x].push_back(s);
      Qs.items[x] += nch * (uint64_t)tiles;
    }
    cbase += chunks;
  };

  // geometry of every query first (queue segments need the tile counts)
  std::vector<RasterQuery> rqs(nq);
  for (int q : order) {
    const QueryPlan& p = items[q].plan;
    const hr_scene* sc = p.sc;
    if (sc->kind == kDisks) {
      RasterQuery& a = rqs[q];
      a = RasterQuery{};
      a.W = sc->W; a.H = sc->H; a.C = sc->C; a.D = sc->D; a.S = qS[q];
      raster_geometry(a, qshape[q]);
      const int cls = p.e.pair ? raster_pair_class(sc->C, sc->D) : raster_class(sc->C, sc->D);
      // a pair item covers the whole image
      add_segments(rq[cls], rchunks[cls], q, (p.e.L + qS[q] - 1) / qS[q], p.e.pair ? 1 : a.tiles);
    } else if (sc->kind == kPT) {
      const uint64_t draws = p.e.streams * p.e.N;
      const int nr = p.e.A * p.e.NH;
      const int c = nr == 1 ? 0 : (nr == 2 ? 1 : 2);
      add_segments(pq[c], pchunks[c], q, (draws + qS[q] - 1) / qS[q], pt_tiles(sc->W, sc->H));
    }
  }
  raster_items_ = pt_items_ = 0;
  for (int c = 0; c < kRasterClasses; ++c) raster_class_items[c] = 0;
  for (int c = 0; c < 3; ++c) pt_class_items[c] = 0;
  for (int x = 0; x < 8; ++x) {
    for (int c = 0; c < kRasterClasses; ++c) raster_class_items[c] += rq[c].items[x];
    for (int c = 0; c < 3; ++c) pt_class_items[c] += pq[c].items[x];
  }
  for (int c = 0; c < kRasterClasses; ++c) raster_items_ += raster_class_items[c];
  for (int c = 0; c < 3; ++c) pt_items_ += pt_class_items[c];

  // table layout
  size_t nrs[kRasterClasses] = {}, nps[3] = {0, 0, 0}, nin = 0, nout = 0;
  for (int x = 0; x < 8; ++x) {
    for (int c = 0; c < kRasterClasses; ++c) nrs[c] += rq[c].seg[x].size();
    for (int c = 0; c < 3; ++c) nps[c] += pq[c].seg[x].size();
  }
  for (auto& it : items) {
    nin += (size_t)it.plan.e.n * (it.v ? 2 : 1);
    nout += it.plan.nout;
  }
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off = align256(off + bytes); return o; };
  const size_t o_hdr = take(sizeof(BatchTable));
  const size_t o_q = take((size_t)nq * sizeof(BatchQuery));
  const size_t o_off = take((size_t)kNumPhases * (nq + 1) * 8);
  size_t o_rs[kRasterClasses], o_ps[3];
  for (int c = 0; c < kRasterClasses; ++c) o_rs[c] = take(std::max<size_t>(nrs[c], 1) * sizeof(WorkSeg));
  for (int c = 0; c < 3; ++c) o_ps[c] = take(std::max<size_t>(nps[c], 1) * sizeof(WorkSeg));
  const size_t o_ctr = take(kWorkCounters * 8);
  const size_t o_in = take(nin * 8);
  upload_bytes_ = off;
  const size_t o_out = take(nout * 8);
  st = reserve_table(off);
  if (st) return st;
  out_off_ = o_out;
  out_doubles_ = nout;
  char* H = (char*)host;
  char* Dv = (char*)dev;
  memset(H, 0, upload_bytes_);

  BatchTable* T = (BatchTable*)(H + o_hdr);
  T->nq = nq;
  T->q = (const BatchQuery*)(Dv + o_q);
  T->off = (const uint64_t*)(Dv + o_off);
  T->ctr = (unsigned long long*)(Dv + o_ctr);
  auto fill_queues = [&](WorkQueues& W, Q8& Qs, size_t o_seg, size_t ctr_index) {
    WorkSeg* hs = (WorkSeg*)(H + o_seg);
    uint64_t k = 0;
    for (int x = 0; x < 8; ++x) {
      W.seg_off[x] = k;
      W.items[x] = Qs.items[x];
      for (const WorkSeg& s : Qs.seg[x]) hs[k++] = s;
    }
    W.seg_off[8] = k;
    W.seg = (const WorkSeg*)(Dv + o_seg);
    W.ctr = (unsigned long long*)(Dv + o_ctr) + ctr_index;
  };
  for (int c = 0; c < kRasterClasses; ++c) fill_queues(T->raster[c], rq[c], o_rs[c], 8 * c);
  for (int c = 0; c < 3; ++c) fill_queues(T->pt[c], pq[c], o_ps[c], 8 * (kRasterClasses + c));

  BatchQuery* HQ = (BatchQuery*)(H + o_q);
  double* hin = (double*)(H + o_in);
  const double* din = (const double*)(Dv + o_in);
  double* dout = (double*)(Dv + o_out);
  size_t kin = 0, kout = 0;
  for (int q = 0; q < nq; ++q) {
    BatchItem& it = items[q];
    const QueryPlan& p = it.plan;
    const hr_scene* sc = p.sc;
    const int n = p.e.n;
    BatchQuery& b = HQ[q];
    b = BatchQuery{};
    b.e = p.e;
    b.scene = sc->kind;
    b.fp64 = p.o.accum_fp64 ? 1 : 0;
    b.chunk = p.chunk;
    b.nchunks = p.nchunks;
    b.part_stride = p.stride;
    b.inv_count = sc->kind == kDisks ? 1.0 / ((double)sc->W * sc->H * sc->C)
                  : sc->kind == kPT  ? 1.0 / ((double)sc->W * sc->H * 3.0)
                                     : 0.0;
    memcpy(hin + kin, it.theta, (size_t)n * 8);
    b.theta = din + kin;
    kin += n;
    if (it.v) {
      memcpy(hin + kin, it.v, (size_t)n * 8);
      b.v = din + kin;
      kin += n;
    }
    b.out = dout + kout;
    it.out_off = kout;
    kout += p.nout;
    const QueryBufs qb = carve(p, (char*)ws + it.ws_off);
    b.tau = qb.tau;
    b.u = qb.u;
    b.rec = qb.rec;
    b.partial = qb.partial;
    b.f = qb.f;
    b.Fq = qb.Fq;
    b.vt = qb.vt;
    b.acc = qb.acc;
    if (sc->kind == kDisks) {
      b.ds = DiskScene{sc->W, sc->H, sc->C, sc->D, sc->ppd, sc->target, sc->colors, sc->radius};
      RasterQuery a = rqs[q];
      a.rec = qb.rec;
      a.target = sc->target;
      a.colors = sc->colors;
      a.partial = qb.partial;
      a.R = p.e.L;
      a.r_base = 0;
      a.ex = RasterExact{b.theta, qb.tau, qb.u, sc->radius, n, sc->ppd, p.e.A, p.e.NH, p.e.h};
      b.rq = a;
    } else if (sc->kind == kPT) {
      b.ptc = sc->ptc;
      b.pt_target = sc->target;
      b.pt_S = qS[q];
      b.pt_tiles_x = pt_tiles_x(sc->W);
      b.pt_tiles = pt_tiles(sc->W, sc->H);
    } else {
      b.as = AnalyticScene{sc->kind == kQuad ? 0 : 1, n, sc->A, sc->b, sc->c, sc->s1};
    }
  }
  single_ = nq == 1;
  if (single_) {
    single_plan_ = items[0].plan;
    single_bufs_ = carve(single_plan_, (char*)ws + items[0].ws_off);
    single_theta_ = HQ[0].theta;
    single_v_ = HQ[0].v;
    single_out_ = HQ[0].out;
    single_S_ = single_plan_.e.pair ? 2 * qS[0] : qS[0];   // renders per block
    single_shape_ = qshape[0];
  }
  uint64_t* ho = (uint64_t*)(H + o_off);
  for (int ph = 0; ph < kNumPhases; ++ph) {
    uint64_t acc = 0;
    for (int q = 0; q < nq; ++q) {
      ho[(size_t)ph * (nq + 1) + q] = acc;
      acc += batch_tasks(HQ[q], ph);
    }
    ho[(size_t)ph * (nq + 1) + nq] = acc;
  }
  lds = std::max(lds, (size_t)1024);
  lds = (lds + 4095) & ~size_t(4095);   // LDS classes of 4 KiB keep the graph reusable
  lds_pair = (std::max(lds_pair, (size_t)1024) + 4095) & ~size_t(4095);
  lds_pair32 = (std::max(lds_pair32, (size_t)1024) + 4095) & ~size_t(4095);
  return HR_OK;
}

void BatchSlot::launches(hipStream_t st, bool time_phases) {
  const BatchTable* T = (const BatchTable*)dev;
  if (single_) {
    hipStream_t keep = ctx->stream;
    if (time_phases) ctx->stream = st;
    launch_query(ctx, st, single_plan_, single_bufs_, single_theta_, single_v_, single_out_,
                 single_S_, single_shape_, time_phases);
    if (time_phases) ctx->stream = keep;
    return;
  }
  auto run = [&](const char* name, auto&& fn) {
    if (time_phases) {
      hipStream_t keep = ctx->stream;
      ctx->stream = st;
      timed(ctx, name, fn);
      ctx->stream = keep;
    } else {
      fn();
    }
  };
  run("batch_sample", [&] { launch_batch_sample(st, T, phase_blocks); });
  run("batch_records", [&] { launch_batch_records(st, T, phase_blocks); });
  run("batch_analytic", [&] { launch_batch_analytic(st, T, phase_blocks); });
  // only the render classes with work are launched
  const unsigned cl = classes();
  run("batch_raster", [&] {
    for (int c = 0; c < kRasterClasses; ++c)
      if (cl & (1u << c))
        launch_batch_raster(st, T, c, raster_blocks[c], class_lds(c));
  });
  run("batch_pt", [&] {
    for (int c = 0; c < 3; ++c)
      if (cl & (1u << (16 + c))) launch_batch_pt(st, T, 1 << c, pt_blocks[c]);
  });
  run("batch_reduce", [&] { launch_batch_reduce(st, T, phase_blocks); });
  run("batch_prep", [&] { launch_batch_prep(st, T, phase_blocks); });
  run("batch_accum", [&] { launch_batch_accum(st, T, phase_blocks); });
  run("batch_finalize", [&] { launch_batch_finalize(st, T, phase_blocks); });
}

unsigned BatchSlot::classes() const {
  unsigned m = 0;
  for (int c = 0; c < kRasterClasses; ++c)
    if (raster_class_items[c]) m |= 1u << c;
  for (int c = 0; c < 3; ++c)
    if (pt_class_items[c]) m |= 1u << (16 + c);
  return m;
}

hr_status BatchSlot::enqueue(bool use_graph, bool timing_ok) {
  HR_HIP(hipSetDevice(ctx->device));
  (void)hipGetLastError();
  const unsigned cl = classes();
  for (int c = 0; c < kRasterClasses; ++c)
    if (cl & (1u << c))
      raster_blocks[c] = cus * batch_raster_blocks_per_cu(c, class_lds(c));
  HR_HIP(hipMemcpyAsync(dev, host, upload_bytes_, hipMemcpyHostToDevice, stream));
  graph_used = false;
  const bool timing = allow_timing && timing_ok && ctx->timing;
  // a one-query batch launches its per-query kernels directly: their launch
  // parameters are the query's own, so a captured sequence would not be reusable
  if (use_graph && !timing && !single_) {
    if (exec && (exec_lds != lds || exec_lds_pair != lds_pair || exec_lds_pair32 != lds_pair32 ||
                 exec_classes != cl)) {
      (void)hipGraphExecDestroy(exec);
      exec = nullptr;
    }
    if (!exec) {
      hipGraph_t g = nullptr;
      HR_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
      launches(stream, false);
      HR_HIP(hipStreamEndCapture(stream, &g));
      hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        exec = nullptr;
        return fail(HR_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
      }
      exec_lds = lds;
      exec_lds_pair = lds_pair;
      exec_lds_pair32 = lds_pair32;
      exec_classes = cl;
    }
    HR_HIP(hipGraphLaunch(exec, stream));
    graph_used = true;
  } else {
    launches(stream, timing);
  }
  HR_HIP(hipGetLastError());
  HR_HIP(hipMemcpyAsync((char*)host + out_off_, (char*)dev + out_off_, out_doubles_ * 8,
                        hipMemcpyDeviceToHost, stream));
  HR_HIP(hipEventRecord(done, stream));
  return HR_OK;
}

void BatchSlot::scatter(const std::vector<BatchItem>& items) const {
  const double* ho = (const double*)((const char*)host + out_off_);
  for (const BatchItem& it : items)
    if (it.out) memcpy(it.out, ho + it.out_off, it.plan.nout * 8);
}

// ---------------------------------------------------------------- autotuner
hr_status autotune_raster(BatchSlot& slot, const std::vector<BatchItem>& items) {
  hr_ctx* ctx = slot.ctx;
  // classes present and not yet tuned
  std::map<uint64_t, std::vector<int>> classes, pt_classes;
  {
    std::lock_guard<std::mutex> lk(ctx->tuned_mu);
    for (int i = 0; i < (int)items.size(); ++i) {
      const QueryPlan& p = items[i].plan;
      const hr_scene* sc = p.sc;
      if (sc->kind == kPT) {
        const uint64_t key = pt_tune_key(sc, p.e.A * p.e.NH);
        if (!ctx->tuned.count(key)) pt_classes[key].push_back(i);
        continue;
      }
      if (sc->kind != kDisks) continue;
      if (ctx->tuned.count(tune_key(sc))) continue;
      classes[tune_key(sc)].push_back(i);
    }
  }
  const int Ss[] = {32, 64, 128, 256};
  const int shapes[] = {1, 2, 3};
  hipEvent_t a, b;
  HR_HIP(hipEventCreate(&a));
  HR_HIP(hipEventCreate(&b));
  hr_status st = HR_OK;
  for (auto& kv : classes) {
    std::vector<BatchItem> sub;
    for (int i : kv.second) {
      BatchItem it = items[i];
      it.out = nullptr;
      sub.push_back(it);
    }
    double best = 1e300;
    std::pair<int, int> pick{0, 0};
    for (int S : Ss) {
      for (int shape : shapes) {
        for (auto& it : sub) {
          it.plan.o.samples_per_block = S;
          it.plan.o.raster_tile = shape;
        }
        st = slot.build(sub);
        if (st) break;
        // prepare draws and records (first pass); the tuning launches are
        // never timed into the context's kernel stats
        st = slot.enqueue(false, false);
        if (st) break;
        // time the raster kernel alone, twice, on the prepared records
        const BatchTable* T = (const BatchTable*)slot.dev;
        const unsigned cl = slot.classes();
        float best_ms = 1e30f;
        for (int rep = 0; rep < 2; ++rep) {
          // the work counters restart from zero before each timed launch
          launch_batch_sample(slot.stream, T, slot.phase_blocks);
          if (hipEventRecord(a, slot.stream) != hipSuccess) { st = fail(HR_EDEVICE, "event"); break; }
          for (int c = 0; c < kRasterClasses; ++c) {
            if (!(cl & (1u << c))) continue;
            const size_t l = slot.class_lds(c);
            launch_batch_raster(slot.stream, T, c, slot.cus * batch_raster_blocks_per_cu(c, l), l);
          }
          if (hipEventRecord(b, slot.stream) != hipSuccess) { st = fail(HR_EDEVICE, "event"); break; }
          if (hipEventSynchronize(b) != hipSuccess) { st = fail(HR_EDEVICE, "event sync"); break; }
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, a, b);
          best_ms = std::min(best_ms, ms);
        }
        if (st) break;
        if (best_ms < best) {
          best = best_ms;
          pick = {S, shape};
        }
      }
      if (st) break;
    }
    if (st) break;
    std::lock_guard<std::mutex> lk(ctx->tuned_mu);
    ctx->tuned[kv.first] = pick;
  }
  // path-traced classes: draws per block item, timed on the persistent path
  // tracer of the class's renders per draw
  const int pSs[] = {2, 4, 8, 16, 32};
  for (auto& kv : pt_classes) {
    if (st) break;
    std::vector<BatchItem> sub;
    for (int i : kv.second) {
      BatchItem it = items[i];
      it.out = nullptr;
      sub.push_back(it);
    }
    const int nr = sub[0].plan.e.A * sub[0].plan.e.NH;
    const int c = nr == 1 ? 0 : (nr == 2 ? 1 : 2);
    double best = 1e300;
    int pick = kDefaultPtSamples;
    for (int S : pSs) {
      for (auto& it : sub) it.plan.o.samples_per_block = S;
      st = slot.build(sub);
      if (st) break;
      st = slot.enqueue(false, false);   // draws prepared, never timed into the stats
      if (st) break;
      const BatchTable* T = (const BatchTable*)slot.dev;
      float best_ms = 1e30f;
      for (int rep = 0; rep < 2; ++rep) {
        launch_batch_sample(slot.stream, T, slot.phase_blocks);   // counters back to zero
        if (hipEventRecord(a, slot.stream) != hipSuccess) { st = fail(HR_EDEVICE, "event"); break; }
        launch_batch_pt(slot.stream, T, nr, slot.pt_blocks[c]);
        if (hipEventRecord(b, slot.stream) != hipSuccess) { st = fail(HR_EDEVICE, "event"); break; }
        if (hipEventSynchronize(b) != hipSuccess) { st = fail(HR_EDEVICE, "event sync"); break; }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, a, b);
        best_ms = std::min(best_ms, ms);
      }
      if (st) break;
      if (best_ms < best) {
        best = best_ms;
        pick = S;
      }
    }
    if (st) break;
    std::lock_guard<std::mutex> lk(ctx->tuned_mu);
    ctx->tuned[kv.first] = {pick, 0};
  }
  (void)hipStreamSynchronize(slot.stream);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return st;
}

// validates one public query and plans it
hr_status plan_item(const hr_query& q, BatchItem* it) {
  if (!q.scene || !q.theta) return fail(HR_EINVAL, "query has a NULL scene or theta");
  if (!q.scene->ctx) return fail(HR_EINVAL, "the scene's context has been destroyed");
  const int what = q.kind;
  const bool hv = what == kHvp || what == kHvpLimit;
  hr_opts o = resolve(q.opts);
  if (o.dbg_loss || o.dbg_tau) return fail(HR_EUNSUPPORTED, "debug buffers are not supported in batches");
  hr_status st = plan_query(q.scene, what, q.sigma, q.N, q.seed, !hv || q.v != nullptr, o, &it->plan);
  if (st) return st;
  const int n = q.scene->n;
  if (!finite_all(q.theta, n)) return fail(HR_EINVAL, "theta has a non-finite entry");
  it->theta = q.theta;
  it->v = nullptr;
  it->zero = false;
  if (hv) {
    if (!finite_all(q.v, n)) return fail(HR_EINVAL, "v has a non-finite entry");
    bool zero = true;
    for (int i = 0; i < n; ++i) zero = zero && q.v[i] == 0.0;
    it->zero = zero;   // Hv = 0, no device work
    it->v = q.v;
  }
  it->out = q.out;
  return HR_OK;
}

}  // namespace rt
}  // namespace hr

struct hr_batch {
  hr_ctx* ctx = nullptr;
  hr_batch_opts opts{};
  BatchSlot slot;
  hr_batch_report last{};
};

extern "C" {

void hr_batch_opts_default(hr_batch_opts* o) {
  if (!o) return;
  o->use_graph = 1;
  o->autotune = 0;
}

hr_status hr_batch_create(hr_ctx* ctx, const hr_batch_opts* opts, hr_batch** out) {
  if (!ctx || !out) return fail(HR_EINVAL, "NULL argument");
  hr_batch* b = new hr_batch();
  b->ctx = ctx;
  hr_batch_opts_default(&b->opts);
  if (opts) b->opts = *opts;
  hr_status st = b->slot.init(ctx);
  if (st) {
    b->slot.release();
    delete b;
    return st;
  }
  *out = b;
  return HR_OK;
}

void hr_batch_destroy(hr_batch* b) {
  if (!b) return;
  b->slot.release();
  delete b;
}

hr_status hr_batch_run(hr_batch* b, const hr_query* queries, int count) {
  if (!b || (!queries && count > 0)) return fail(HR_EINVAL, "NULL argument");
  if (count < 0) return fail(HR_EINVAL, "count must be >= 0");
  TraceRange range("hr_batch_run");
  hr_ctx* ctx = b->ctx;
  if (!b->slot.ctx) return fail(HR_EINVAL, "batch is not initialised");
  for (int i = 0; i < count; ++i) {
    if (!queries[i].out) return fail(HR_EINVAL, "query " + std::to_string(i) + " has a NULL out");
    if (queries[i].scene && queries[i].scene->ctx != ctx)
      return fail(HR_EINVAL, "query " + std::to_string(i) + " uses a scene of another context");
  }
  std::vector<BatchItem> items;
  items.reserve(count);
  size_t ws = 0;
  for (int i = 0; i < count; ++i) {
    BatchItem it;
    hr_status st = plan_item(queries[i], &it);
    if (st) return fail(st, "query " + std::to_string(i) + ": " + error_slot());
    if (it.zero) {
      for (size_t k = 0; k < it.plan.nout; ++k) it.out[k] = 0.0;
      continue;
    }
    ws += align256(it.plan.total);
    items.push_back(it);
  }
  if (ws > ctx->budget)
    return fail(HR_ENOMEM, "batch needs " + std::to_string(ws) + " bytes of workspace, budget is " +
                               std::to_string(ctx->budget));
  b->last = hr_batch_report{};
  b->last.queries = (uint64_t)count;
  if (items.empty()) return HR_OK;
  HR_HIP(hipSetDevice(ctx->device));
  hr_status st = HR_OK;
  if (b->opts.autotune) {
    st = autotune_raster(b->slot, items);
    if (st) return st;
  }
  st = b->slot.build(items);
  if (st) return st;
  st = b->slot.enqueue(b->opts.use_graph != 0);
  if (st) return st;
  HR_HIP(hipEventSynchronize(b->slot.done));
  if (ctx->timing) {
    st = drain_timers(ctx);
    if (st) return st;
  }
  b->slot.scatter(items);
  b->last.raster_items = b->slot.raster_items_;
  b->last.pt_items = b->slot.pt_items_;
  {
    int rb = 0;
    const unsigned cl = b->slot.classes();
    for (int c = 0; c < kRasterClasses; ++c)
      if (cl & (1u << c)) rb = std::max(rb, b->slot.raster_blocks[c]);
    b->last.raster_blocks = rb;
  }
  b->last.pt_blocks = b->slot.pt_blocks[0];
  b->last.workspace_bytes = ws;
  b->last.graph = b->slot.graph_used ? 1 : 0;
  b->last.lds_bytes = (uint64_t)b->slot.lds;
  return HR_OK;
}

hr_status hr_batch_report_get(const hr_batch* b, hr_batch_report* out) {
  if (!b || !out) return fail(HR_EINVAL, "NULL argument");
  *out = b->last;
  return HR_OK;
}

hr_status hr_batch_tuned(hr_ctx* ctx, const hr_scene* sc, int* samples_per_block, int* raster_tile) {
  if (!ctx || !sc || !samples_per_block || !raster_tile) return fail(HR_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(ctx->tuned_mu);
  auto it = ctx->tuned.find(sc->kind == kPT ? pt_tune_key(sc, 2) : tune_key(sc));
  if (it == ctx->tuned.end()) {
    *samples_per_block = 0;
    *raster_tile = 0;
    return HR_OK;
  }
  *samples_per_block = it->second.first;
  *raster_tile = it->second.second;
  return HR_OK;
}

}  // extern "C"
