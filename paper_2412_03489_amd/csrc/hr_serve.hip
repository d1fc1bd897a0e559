// hr_serve.hip -- continuous-batching server over the batch executor.
//
// One worker thread owns `slots` BatchSlots (each with its own stream).  Its
// loop: retire every slot whose batch has finished (results scattered to the
// tickets, waiters woken), then fill every free slot with the waiting
// queries in arrival order while their workspace fits the slot's share of
// device memory, and launch it.  A slot's workspace is allocated once at
// start-up, so admission is pure bookkeeping and no allocation or free ever
// stalls the batches in flight.  With two or more slots, queries that
// arrive while a batch runs are launched in the next free slot and overlap
// with it on the device.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hr_batch.h"

using namespace hr;
using namespace hr::rt;

namespace {

constexpr uint64_t kDefaultServerMemory = 8ull << 30;
constexpr size_t kTableReserve = 4u << 20;

// Predicted device milliseconds of one query (batch formation only; results
// never depend on it): rasterised pixel-renders at ~3.3 per ps, path-traced
// pixel samples at ~80 per ns, lobe-sum terms at ~200 per ns, plus a fixed
// 20 us of small launches.
double predict_ms(const QueryPlan& p) {
  const hr_scene* sc = p.sc;
  const double R = (double)p.e.R;
  double ms = 0.02;
  if (sc->kind == kDisks) ms += R * sc->W * sc->H / 3.3e9;
  else if (sc->kind == kPT) ms += R * sc->W * sc->H * sc->spp / 8.0e7;
  else ms += R * p.e.n * p.e.n / 1.0e9;
  ms += (double)p.e.streams * (double)p.e.N * (double)p.e.nout / 2.0e8;
  return ms;
}

struct Ticket {
  uint64_t id = 0;
  BatchItem item;
  double cost_ms = 0.0;   // predicted device time
  std::vector<double> theta, v, result;
  hr_query_stats stats{};
  int state = 0;   // 0 waiting, 1 on the device, 2 done
  bool waited = false;   // a thread is blocked in hr_wait on this ticket
  uint64_t batch = 0;    // the batch it ran in (1, 2, ...; 0: none)
  int slot = -1;         // the slot that ran it
};

const char* what_name(int w) {
  switch (w) {
    case kGrad: return "grad";
    case kHess: return "hess";
    case kHvp: return "hvp";
    case kHvpLimit: return "hvp_limit";
    default: return "loss";
  }
}

const char* scene_name(int k) {
  switch (k) {
    case kDisks: return "disks";
    case kPT: return "pt";
    case kQuad: return "quad";
    default: return "neggauss";
  }
}

// One JSON line per completed query: what it was, where it ran, its times
// (ms since the server started) and its status.
void write_metrics(FILE* f, const Ticket& t) {
  const QueryPlan& p = t.item.plan;
  const hr_scene* sc = p.sc;
  const hr_query_stats& st = t.stats;
  std::fprintf(f,
               "{\"ticket\":%llu,\"kind\":\"%s\",\"scene\":\"%s\",\"W\":%d,\"H\":%d,"
               "\"params\":%d,\"N\":%llu,\"seed\":%llu,\"sampler\":%d,\"renders\":%llu,"
               "\"batch\":%llu,\"batch_size\":%d,\"slot\":%d,\"submit_ms\":%.4f,"
               "\"start_ms\":%.4f,\"end_ms\":%.4f,\"queue_ms\":%.4f,\"service_ms\":%.4f,"
               "\"status\":%d}\n",
               (unsigned long long)t.id, what_name(p.e.what), scene_name(sc->kind), sc->W, sc->H,
               sc->n, (unsigned long long)p.e.N, (unsigned long long)p.e.seed, p.e.sampler,
               (unsigned long long)p.e.R, (unsigned long long)t.batch, st.batch_size, t.slot,
               st.submit_ms, st.start_ms, st.end_ms, st.start_ms - st.submit_ms,
               st.end_ms - st.start_ms, (int)st.status);
}

struct Flight {
  bool busy = false;
  std::vector<BatchItem> items;
  std::vector<Ticket*> tickets;
};

// A query held by a server (waiting or on the device) pins its scene:
// hr_scene_destroy waits until the count drops to zero.
void scene_hold(hr_scene* sc) {
  std::lock_guard<std::mutex> lk(sc->hold_mu);
  ++sc->held;
}
void scene_release(hr_scene* sc) {
  std::lock_guard<std::mutex> lk(sc->hold_mu);
  if (--sc->held == 0) sc->hold_cv.notify_all();
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct hr_server {
  hr_ctx* ctx = nullptr;
  hr_server_opts opts{};
  std::vector<BatchSlot> slots;
  std::vector<Flight> flights;
  size_t capacity = 0;   // workspace bytes per slot
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Ticket*> waiting;
  std::unordered_map<uint64_t, std::unique_ptr<Ticket>> tickets;
  std::deque<uint64_t> completed;   // done, not yet handed out by hr_wait_any
  std::thread worker;
  bool stop = false;
  uint64_t next_id = 1;
  std::chrono::steady_clock::time_point t0;
  hr_server_stats st{};
  int busy_slots = 0;
  double busy_since = 0.0;
  uint64_t launched = 0;   // queries sent to the device in batches
  uint64_t batch_seq = 0;  // batches launched so far
  FILE* metrics = nullptr; // JSON Lines of completed queries (opts.metrics_path)

  void finish_flight(int i, hr_status status) {
    Flight& f = flights[i];
    if (status == HR_OK) slots[i].scatter(f.items);
    const double now = ms_since(t0);
    for (Ticket* t : f.tickets) {
      t->state = 2;
      t->stats.end_ms = now;
      t->stats.status = status;
      completed.push_back(t->id);
      scene_release(t->item.plan.sc);
      if (metrics) write_metrics(metrics, *t);
    }
    if (metrics) std::fflush(metrics);
    st.completed += f.tickets.size();
    f.items.clear();
    f.tickets.clear();
    f.busy = false;
    if (--busy_slots == 0) st.busy_ms += now - busy_since;
    cv_done.notify_all();
  }

  // Forms slot i's batch from the waiting queries (under the lock held by
  // `lk`), then releases the lock while the batch is tuned, laid out and
  // enqueued: the flight is the worker's alone once marked busy, and callers
  // of hr_submit / hr_wait / hr_wait_any are never held up by that host work.
  void launch(int i, std::unique_lock<std::mutex>& lk) {
    Flight& f = flights[i];
    size_t ws = 0;
    double work = 0.0;
    const double cap = opts.max_batch_ms > 0.0 ? opts.max_batch_ms : 1e300;
    while (!waiting.empty() && (int)f.items.size() < opts.max_batch) {
      Ticket* t = waiting.front();
      const size_t need = align256(t->item.plan.total);
      if (!f.items.empty() && (ws + need > capacity || work + t->cost_ms > cap)) break;
      waiting.pop_front();
      ws += need;
      work += t->cost_ms;
      f.items.push_back(t->item);
      f.tickets.push_back(t);
    }
    if (f.items.empty()) return;
    const double now = ms_since(t0);
    ++batch_seq;
    for (Ticket* t : f.tickets) {
      t->state = 1;
      t->stats.start_ms = now;
      t->stats.batch_size = (int)f.tickets.size();
      t->batch = batch_seq;
      t->slot = i;
    }
    f.busy = true;
    if (busy_slots++ == 0) busy_since = now;
    st.batches += 1;
    launched += f.items.size();
    lk.unlock();
    TraceRange range("hr_server batch");
    hr_status s = HR_OK;
    if (opts.autotune) s = autotune_raster(slots[i], f.items);
    if (!s) s = slots[i].build(f.items);
    if (!s) s = slots[i].enqueue(opts.use_graph != 0, false);
    if (s) (void)hipStreamSynchronize(slots[i].stream);
    lk.lock();
    if (s) finish_flight(i, s);
  }

  void run() {
    (void)hipSetDevice(ctx->device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      bool any_busy = false;
      for (int i = 0; i < (int)slots.size(); ++i) {
        if (!flights[i].busy) continue;
        const hipError_t q = hipEventQuery(slots[i].done);
        if (q == hipSuccess) {
          finish_flight(i, HR_OK);
        } else if (q != hipErrorNotReady) {
          fail(HR_EDEVICE, std::string("batch failed: ") + hipGetErrorString(q));
          finish_flight(i, HR_EDEVICE);
        } else {
          any_busy = true;
        }
      }
      for (int i = 0; i < (int)slots.size() && !waiting.empty(); ++i)
        if (!flights[i].busy) {
          launch(i, lk);
          any_busy = any_busy || flights[i].busy;
        }
      if (stop && waiting.empty() && !any_busy) break;
      if (any_busy) cv_work.wait_for(lk, std::chrono::microseconds(50));
      else if (waiting.empty()) cv_work.wait(lk, [&] { return stop || !waiting.empty(); });
    }
  }
};

extern "C" {

void hr_server_opts_default(hr_server_opts* o) {
  if (!o) return;
  o->slots = 4;
  o->max_batch = 64;
  o->max_batch_ms = 2.0;
  o->memory_bytes = 0;
  o->use_graph = 1;
  o->autotune = 0;
  o->metrics_path = nullptr;
}

hr_status hr_server_create(hr_ctx* ctx, const hr_server_opts* opts, hr_server** out) {
  if (!ctx || !out) return fail(HR_EINVAL, "NULL argument");
  hr_server_opts o;
  hr_server_opts_default(&o);
  if (opts) o = *opts;
  if (o.slots < 1 || o.slots > 8) return fail(HR_EINVAL, "slots must be 1..8");
  if (o.max_batch < 1 || o.max_batch > 4096) return fail(HR_EINVAL, "max_batch must be 1..4096");
  if (std::isnan(o.max_batch_ms)) return fail(HR_EINVAL, "max_batch_ms is NaN");
  uint64_t mem = o.memory_bytes ? o.memory_bytes : kDefaultServerMemory;
  if (mem > ctx->budget) mem = ctx->budget;
  auto s = std::make_unique<hr_server>();
  s->ctx = ctx;
  s->opts = o;
  s->capacity = (size_t)(mem / (uint64_t)o.slots) & ~size_t(255);
  s->slots.resize(o.slots);
  s->flights.resize(o.slots);
  HR_HIP(hipSetDevice(ctx->device));
  for (auto& sl : s->slots) {
    hr_status st = sl.init(ctx);
    sl.allow_timing = false;   // the worker never touches the context's timers
    if (!st) st = sl.reserve_workspace(s->capacity);
    if (!st) st = sl.reserve_table(kTableReserve);
    if (st) {
      for (auto& x : s->slots) x.release();
      return st;
    }
  }
  if (o.metrics_path && o.metrics_path[0]) {
    s->metrics = std::fopen(o.metrics_path, "a");
    if (!s->metrics) {
      for (auto& x : s->slots) x.release();
      return fail(HR_EINVAL, std::string("cannot open metrics file ") + o.metrics_path);
    }
  }
  s->opts.metrics_path = nullptr;   // the caller's string is not kept
  s->t0 = std::chrono::steady_clock::now();
  hr_server* raw = s.release();
  raw->worker = std::thread([raw] { raw->run(); });
  *out = raw;
  return HR_OK;
}

void hr_server_destroy(hr_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto& sl : s->slots) sl.release();
  if (s->metrics) std::fclose(s->metrics);
  delete s;
}

hr_status hr_submit(hr_server* s, const hr_query* q, uint64_t* ticket) {
  if (!s || !q || !ticket) return fail(HR_EINVAL, "NULL argument");
  if (q->scene && q->scene->ctx != s->ctx) return fail(HR_EINVAL, "scene of another context");
  auto t = std::make_unique<Ticket>();
  hr_query qq = *q;
  qq.out = nullptr;
  hr_status st = plan_item(qq, &t->item);
  if (st) return st;
  if (align256(t->item.plan.total) > s->capacity)
    return fail(HR_ENOMEM, "query needs " + std::to_string(t->item.plan.total) +
                               " bytes of workspace, a server slot holds " +
                               std::to_string(s->capacity));
  const int n = q->scene->n;
  t->theta.assign(q->theta, q->theta + n);
  t->item.theta = t->theta.data();
  if (t->item.v) {
    t->v.assign(q->v, q->v + n);
    t->item.v = t->v.data();
  }
  t->result.assign(t->item.plan.nout, 0.0);
  t->item.out = t->result.data();
  t->cost_ms = predict_ms(t->item.plan);
  std::lock_guard<std::mutex> lk(s->mu);
  t->id = s->next_id++;
  t->item.ticket = t->id;
  t->stats.submit_ms = ms_since(s->t0);
  t->stats.status = HR_OK;
  s->st.submitted += 1;
  *ticket = t->id;
  Ticket* raw = t.get();
  s->tickets.emplace(t->id, std::move(t));
  if (raw->item.zero) {   // Hv = 0: done without device work
    raw->state = 2;
    raw->stats.start_ms = raw->stats.end_ms = raw->stats.submit_ms;
    if (s->metrics) {
      write_metrics(s->metrics, *raw);
      std::fflush(s->metrics);
    }
    s->completed.push_back(raw->id);
    s->st.completed += 1;
    s->cv_done.notify_all();
    return HR_OK;
  }
  scene_hold(raw->item.plan.sc);
  s->waiting.push_back(raw);
  s->cv_work.notify_one();
  return HR_OK;
}

hr_status hr_wait(hr_server* s, uint64_t ticket, double* out, hr_query_stats* stats) {
  if (!s) return fail(HR_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(HR_EINVAL, "unknown or retired ticket");
  Ticket* t = it->second.get();
  // one waiter per ticket: the waiter retires (frees) it when done
  if (t->waited) return fail(HR_EBUSY, "another thread is already waiting on this ticket");
  t->waited = true;
  s->cv_done.wait(lk, [&] { return t->state == 2; });
  if (out) memcpy(out, t->result.data(), t->result.size() * 8);
  if (stats) *stats = t->stats;
  const hr_status status = t->stats.status;
  s->tickets.erase(it);
  if (status) return fail(status, "query failed on the device");
  return HR_OK;
}

hr_status hr_wait_any(hr_server* s, double timeout_ms, uint64_t* ticket) {
  if (!s || !ticket) return fail(HR_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto ready = [&] {
    while (!s->completed.empty() && !s->tickets.count(s->completed.front())) s->completed.pop_front();
    return !s->completed.empty();
  };
  if (timeout_ms < 0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), ready)) {
    return fail(HR_EBUSY, "no query completed in time");
  }
  *ticket = s->completed.front();
  s->completed.pop_front();
  return HR_OK;
}

hr_status hr_server_stats_get(hr_server* s, hr_server_stats* out) {
  if (!s || !out) return fail(HR_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  out->mean_batch = s->st.batches ? (double)s->launched / (double)s->st.batches : 0.0;
  if (s->busy_slots > 0) out->busy_ms += ms_since(s->t0) - s->busy_since;
  return HR_OK;
}

}  // extern "C"
