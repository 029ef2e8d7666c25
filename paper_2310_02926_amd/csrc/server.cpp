// Request server with continuous batching (binsrv_*).
//
// binsrv_submit() may be called from any thread while earlier requests run.
// One dispatcher thread:
//   * polls the in-flight batches (one per stream slot) for completion and
//     stamps their requests done (latency = submit -> completion observed);
//   * whenever a slot is free, admits waiting requests in arrival order as
//     long as their result grids and the batch scratch fit the device-memory
//     budget, and runs them as one batched launch on that slot's stream.
// Slots run concurrently on the device.  Result grids come from a reuse pool
// keyed by size and stay resident until binsrv_release().
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <set>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"

using namespace binimpl;

namespace {

using clk = std::chrono::steady_clock;

double ms_between(clk::time_point a, clk::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

size_t al256(size_t v) { return (v + 255) & ~size_t(255); }

enum ReqState { Q_WAITING = 0, Q_RUNNING = 1, Q_DONE = 2 };

struct SrvReq {
  uint64_t ticket = 0;
  binsrv_request r{};
  std::vector<const void*> coord_cols, attr_cols;
  int state = Q_WAITING;
  int status = BIN_OK;
  clk::time_point t_submit, t_dispatch, t_done;
  bool dispatched = false;
  size_t out_bytes = 0;
  size_t scratch_est = 0;  // library scratch to run it alone
  // resident result grids (device), grouped as one allocation
  void* grids = nullptr;
  size_t grid_bytes = 0;
  uint32_t* count = nullptr;
  void* sum[BIN_MAX_ATTRS] = {};
  void* mn[BIN_MAX_ATTRS] = {};
  void* mx[BIN_MAX_ATTRS] = {};
  void* avg[BIN_MAX_ATTRS] = {};
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  std::vector<uint64_t> tickets;
  size_t scratch_reserved = 0;  // bytes of the library pool this slot may hold
};

// Bytes of the result grids of a request (all requested ops, default precision rules).
size_t grid_bytes_of(const binsrv_request& r) {
  const size_t nb = (size_t)r.nx * r.ny;
  const int k = r.attrs.cols ? r.attrs.ncols : 0;
  const bool f64 = k > 0 && r.attrs.dtype == BIN_F64;
  const size_t mm = f64 ? 8 : 4;
  const size_t sa = (!f64 && (r.ops & BIN_PREC_PLAIN)) ? 4 : 8;
  size_t b = 0;
  if (r.ops & BIN_COUNT) b += al256(4 * nb);
  if (r.ops & BIN_SUM) b += k * al256(sa * nb);
  if (r.ops & BIN_MIN) b += k * al256(mm * nb);
  if (r.ops & BIN_MAX) b += k * al256(mm * nb);
  if (r.ops & BIN_AVG) b += k * al256(sa * nb);
  return std::max<size_t>(b, 256);
}

}  // namespace

struct binsrv {
  binsrv_config cfg{};
  std::mutex mu;
  std::condition_variable cv_work;  // dispatcher wake-up
  std::condition_variable cv_done;  // waiters
  std::thread thr;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, SrvReq> reqs;
  std::vector<Slot> slots;
  std::unordered_map<size_t, std::vector<void*>> pool;  // free result blocks by size
  size_t pool_bytes = 0;       // bytes in free pool blocks
  size_t resident_bytes = 0;   // bytes of blocks held by requests
  binsrv_stats st{};
  int fatal = BIN_OK;
};

namespace {

std::mutex g_live_mu;
std::set<binsrv*> g_live;

bool live(binsrv* s) {
  std::lock_guard<std::mutex> lk(g_live_mu);
  return g_live.count(s) != 0;
}

size_t in_use(const binsrv* s) {
  size_t b = s->pool_bytes + s->resident_bytes;
  for (const Slot& sl : s->slots) b += sl.scratch_reserved;
  return b;
}

// Memory that cannot be reclaimed right now (pooled free blocks can).
size_t committed(const binsrv* s) { return in_use(s) - s->pool_bytes; }

// Take a result block of exactly 'bytes' from the pool or the device.
int take_block(binsrv* s, size_t bytes, void** out) {
  auto it = s->pool.find(bytes);
  if (it != s->pool.end() && !it->second.empty()) {
    *out = it->second.back();
    it->second.pop_back();
    s->pool_bytes -= bytes;
    s->resident_bytes += bytes;
    return BIN_OK;
  }
  // Make room by freeing pooled blocks of other sizes if the budget is tight.
  for (auto& kv : s->pool) {
    while (!kv.second.empty() && in_use(s) + bytes > s->cfg.budget_bytes) {
      (void)hipFree(kv.second.back());
      kv.second.pop_back();
      s->pool_bytes -= kv.first;
    }
  }
  if (fault_injection_hit()) return fail(BIN_ERR_OOM, "injected result-grid allocation failure");
  hipError_t e = hipMalloc(out, bytes);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc(result grids)");
  s->resident_bytes += bytes;
  return BIN_OK;
}

void give_block(binsrv* s, void* p, size_t bytes) {
  if (!p) return;
  s->pool[bytes].push_back(p);
  s->resident_bytes -= bytes;
  s->pool_bytes += bytes;
}

void carve_outputs(SrvReq& q) {
  const binsrv_request& r = q.r;
  const size_t nb = (size_t)r.nx * r.ny;
  const int k = r.attrs.cols ? r.attrs.ncols : 0;
  const bool f64 = k > 0 && r.attrs.dtype == BIN_F64;
  const size_t mm = f64 ? 8 : 4;
  const size_t sa = (!f64 && (r.ops & BIN_PREC_PLAIN)) ? 4 : 8;
  unsigned char* p = static_cast<unsigned char*>(q.grids);
  if (r.ops & BIN_COUNT) {
    q.count = reinterpret_cast<uint32_t*>(p);
    p += al256(4 * nb);
  }
  for (int j = 0; j < k; ++j) {
    if (r.ops & BIN_SUM) { q.sum[j] = p; p += al256(sa * nb); }
    if (r.ops & BIN_MIN) { q.mn[j] = p; p += al256(mm * nb); }
    if (r.ops & BIN_MAX) { q.mx[j] = p; p += al256(mm * nb); }
    if (r.ops & BIN_AVG) { q.avg[j] = p; p += al256(sa * nb); }
  }
}

bin_request as_bin_request(SrvReq& q) {
  bin_request b;
  std::memset(&b, 0, sizeof b);
  b.coords = q.r.coords;
  b.coords.cols = q.coord_cols.data();
  b.attrs = q.r.attrs;
  b.attrs.cols = q.attr_cols.empty() ? nullptr : q.attr_cols.data();
  b.n = q.r.n;
  b.axes[0] = q.r.axes[0];
  b.axes[1] = q.r.axes[1];
  std::memcpy(b.bounds, q.r.bounds, sizeof b.bounds);
  b.nx = q.r.nx;
  b.ny = q.r.ny;
  b.ops = q.r.ops;
  b.out.count = q.count;
  b.out.sum = q.sum;
  b.out.min = q.mn;
  b.out.max = q.mx;
  b.out.avg = q.avg;
  return b;
}

// Completion polling; caller holds the lock.
void poll_slots(binsrv* s) {
  for (Slot& sl : s->slots) {
    if (!sl.busy) continue;
    hipError_t e = hipEventQuery(sl.done);
    if (e == hipErrorNotReady) continue;
    const clk::time_point now = clk::now();
    for (uint64_t t : sl.tickets) {
      auto it = s->reqs.find(t);
      if (it == s->reqs.end()) continue;
      it->second.state = Q_DONE;
      it->second.t_done = now;
      it->second.status = e == hipSuccess ? BIN_OK : BIN_ERR_DEVICE;
      if (e == hipSuccess) s->st.completed++;
      else s->st.failed++;
      s->st.in_flight--;
    }
    if (e != hipSuccess) s->fatal = BIN_ERR_DEVICE;
    sl.tickets.clear();
    sl.busy = false;
    s->cv_done.notify_all();
  }
}

// Admit and launch one micro-batch on a free slot; caller holds the lock.
// Returns true if it launched something.
bool dispatch_one(binsrv* s, std::unique_lock<std::mutex>& lk) {
  int free_slot = -1;
  for (size_t i = 0; i < s->slots.size(); ++i)
    if (!s->slots[i].busy) {
      free_slot = (int)i;
      break;
    }
  if (free_slot < 0 || s->queue.empty()) return false;
  Slot& sl = s->slots[free_slot];
  // Release this slot's previous scratch reservation; re-reserve below.
  const size_t old_reserved = sl.scratch_reserved;
  sl.scratch_reserved = 0;
  std::vector<uint64_t> batch;
  std::vector<bin_request> brs;
  size_t scratch_need = 0;
  while (!s->queue.empty() && (int)batch.size() < s->cfg.max_batch) {
    SrvReq& q = s->reqs[s->queue.front()];
    // Batch scratch is bounded by the sum of the members' own scratch.
    const size_t need = scratch_need + q.scratch_est;
    const size_t reserve = std::max(need, old_reserved);
    // Not admitted now: wait for running work or released grids.
    if (committed(s) + q.out_bytes + reserve > s->cfg.budget_bytes) break;
    void* blk = nullptr;
    int st = take_block(s, q.out_bytes, &blk);
    if (st) {
      q.state = Q_DONE;
      q.status = st;
      q.t_done = clk::now();
      s->st.failed++;
      s->queue.pop_front();
      s->cv_done.notify_all();
      continue;
    }
    q.grids = blk;
    q.grid_bytes = q.out_bytes;
    carve_outputs(q);
    scratch_need = need;
    brs.push_back(as_bin_request(q));
    batch.push_back(q.ticket);
    s->queue.pop_front();
  }
  if (batch.empty()) {
    sl.scratch_reserved = old_reserved;
    return false;
  }
  sl.scratch_reserved = std::max(scratch_need, old_reserved);
  sl.busy = true;
  sl.tickets = batch;
  const clk::time_point now = clk::now();
  for (uint64_t t : batch) {
    SrvReq& q = s->reqs[t];
    q.state = Q_RUNNING;
    q.t_dispatch = now;
    q.dispatched = true;
  }
  s->st.batches++;
  s->st.in_flight += batch.size();
  s->st.queued = s->queue.size();
  s->st.bytes_in_use = in_use(s);
  s->st.peak_bytes = std::max<uint64_t>(s->st.peak_bytes, s->st.bytes_in_use);
  hipStream_t stream = sl.stream;
  hipEvent_t ev = sl.done;
  // Launch outside the lock: submitters and waiters keep going.
  lk.unlock();
  // A lone request takes the single-request kernels (their tuned shapes).
  int st = brs.size() == 1 ? run_request(brs[0], stream, PlanHints{})
                           : run_batch(brs.data(), (int)brs.size(), stream, PlanHints{});
  hipError_t e = hipSuccess;
  if (st == BIN_OK) e = hipEventRecord(ev, stream);
  lk.lock();
  if (st != BIN_OK || e != hipSuccess) {
    // Nothing usable was enqueued: fail the batch now (the slot's stream
    // has no pending work of ours, so the slot is free again).
    (void)hipStreamSynchronize(stream);
    for (uint64_t t : batch) {
      SrvReq& q = s->reqs[t];
      q.state = Q_DONE;
      q.status = st != BIN_OK ? st : BIN_ERR_DEVICE;
      q.t_done = clk::now();
      s->st.failed++;
      s->st.in_flight--;
    }
    sl.busy = false;
    sl.tickets.clear();
    s->cv_done.notify_all();
  }
  return true;
}

void dispatcher(binsrv* s) {
  (void)hipSetDevice(s->cfg.device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    poll_slots(s);
    bool launched = false;
    while (dispatch_one(s, lk)) launched = true;
    bool any_busy = false;
    for (const Slot& sl : s->slots) any_busy |= sl.busy;
    if (s->stop && s->queue.empty() && !any_busy) break;
    if (launched) continue;
    // Sleep until a submission arrives, or briefly while work is in flight
    // (completion is polled).
    if (any_busy) s->cv_work.wait_for(lk, std::chrono::microseconds(20));
    else s->cv_work.wait_for(lk, std::chrono::milliseconds(5));
  }
}

}  // namespace

extern "C" {

int binsrv_create(const binsrv_config* cfg, binsrv** out) {
  clear_error();
  if (!cfg || !out) return fail(BIN_ERR_INVALID_ARG, "cfg or srv is NULL");
  *out = nullptr;
  if (cfg->n_slots < 1 || cfg->n_slots > 64) return fail(BIN_ERR_INVALID_ARG, "n_slots must be in [1, 64]");
  if (cfg->max_batch < 1 || cfg->max_batch > 65535) return fail(BIN_ERR_INVALID_ARG, "max_batch must be in [1, 65535]");
  if (cfg->budget_bytes < (1u << 20)) return fail(BIN_ERR_INVALID_ARG, "budget_bytes must be at least 1 MiB");
  hipError_t e = hipSetDevice(cfg->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  binsrv* s = new binsrv;
  s->cfg = *cfg;
  s->slots.resize(cfg->n_slots);
  for (Slot& sl : s->slots) {
    e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    if (e != hipSuccess) {
      for (Slot& x : s->slots) {
        if (x.done) (void)hipEventDestroy(x.done);
        if (x.stream) (void)hipStreamDestroy(x.stream);
      }
      delete s;
      return hip_fail(e, "server stream setup");
    }
  }
  s->thr = std::thread(dispatcher, s);
  {
    std::lock_guard<std::mutex> lk(g_live_mu);
    g_live.insert(s);
  }
  *out = s;
  return BIN_OK;
}

int binsrv_submit(binsrv* s, const binsrv_request* req, uint64_t* ticket) {
  clear_error();
  if (!live(s)) return fail(BIN_ERR_INVALID_ARG, "not a live server");
  if (!req || !ticket) return fail(BIN_ERR_INVALID_ARG, "req or ticket is NULL");
  bin_output none;
  std::memset(&none, 0, sizeof none);
  // Validate with stand-in outputs (the server owns the real ones).
  void* fake[BIN_MAX_ATTRS];
  for (int j = 0; j < BIN_MAX_ATTRS; ++j) fake[j] = reinterpret_cast<void*>(uintptr_t(256) * (j + 1));
  none.count = reinterpret_cast<uint32_t*>(uintptr_t(4096));
  none.sum = none.min = none.max = none.avg = fake;
  int st = validate(&req->coords, &req->attrs, req->n, req->axes, req->bounds, req->nx, req->ny, req->ops, &none, false);
  if (st) return st;
  SrvReq q;
  q.r = *req;
  q.coord_cols.assign(req->coords.cols, req->coords.cols + req->coords.ncols);
  if (req->attrs.cols && req->attrs.ncols > 0) q.attr_cols.assign(req->attrs.cols, req->attrs.cols + req->attrs.ncols);
  q.out_bytes = grid_bytes_of(*req);
  // Can it ever fit?  Its grids plus the scratch of running it alone.
  bin_request alone = as_bin_request(q);
  void* dummy[BIN_MAX_ATTRS];
  for (int j = 0; j < BIN_MAX_ATTRS; ++j) dummy[j] = fake[j];
  alone.out.count = none.count;
  alone.out.sum = alone.out.min = alone.out.max = alone.out.avg = dummy;
  const size_t need = batch_scratch_bytes(&alone, 1, &st);
  if (st) return st;
  q.scratch_est = need;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return fail(BIN_ERR_INVALID_ARG, "server is shutting down");
  if (q.out_bytes + need > s->cfg.budget_bytes)
    return fail(BIN_ERR_ADMISSION, "request needs %zu bytes, budget is %llu", q.out_bytes + need,
                (unsigned long long)s->cfg.budget_bytes);
  q.ticket = s->next_ticket++;
  q.t_submit = clk::now();
  *ticket = q.ticket;
  s->queue.push_back(q.ticket);
  s->reqs.emplace(q.ticket, std::move(q));
  s->st.submitted++;
  s->st.queued = s->queue.size();
  s->cv_work.notify_one();
  return BIN_OK;
}

int binsrv_wait(binsrv* s, uint64_t ticket, int64_t timeout_ns, bin_result* res) {
  clear_error();
  if (!live(s)) return fail(BIN_ERR_INVALID_ARG, "not a live server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto done = [&] {
    auto it = s->reqs.find(ticket);
    return it == s->reqs.end() || it->second.state == Q_DONE;
  };
  if (timeout_ns < 0) s->cv_done.wait(lk, done);
  else if (!s->cv_done.wait_for(lk, std::chrono::nanoseconds(timeout_ns), done))
    return fail(BIN_ERR_TIMEOUT, "ticket %llu not done after %lld ns", (unsigned long long)ticket, (long long)timeout_ns);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(BIN_ERR_NOT_FOUND, "unknown or released ticket %llu", (unsigned long long)ticket);
  SrvReq& q = it->second;
  if (res) {
    std::memset(res, 0, sizeof *res);
    res->status = q.status;
    res->k = q.r.attrs.cols ? q.r.attrs.ncols : 0;
    res->count = q.count;
    for (int j = 0; j < res->k; ++j) {
      res->sum[j] = q.sum[j];
      res->min[j] = q.mn[j];
      res->max[j] = q.mx[j];
      res->avg[j] = q.avg[j];
    }
    res->submit_to_done_ms = ms_between(q.t_submit, q.t_done);
    res->queue_ms = q.dispatched ? ms_between(q.t_submit, q.t_dispatch) : 0.0;
  }
  return q.status;
}

int binsrv_release(binsrv* s, uint64_t ticket) {
  clear_error();
  if (!live(s)) return fail(BIN_ERR_INVALID_ARG, "not a live server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(BIN_ERR_NOT_FOUND, "unknown or already released ticket %llu", (unsigned long long)ticket);
  if (it->second.state != Q_DONE) return fail(BIN_ERR_INVALID_ARG, "ticket %llu is not finished", (unsigned long long)ticket);
  give_block(s, it->second.grids, it->second.grid_bytes);
  s->reqs.erase(it);
  s->st.released++;
  s->st.bytes_in_use = in_use(s);
  s->cv_work.notify_one();  // released memory may admit waiting requests
  return BIN_OK;
}

int binsrv_get_stats(binsrv* s, binsrv_stats* out) {
  clear_error();
  if (!live(s)) return fail(BIN_ERR_INVALID_ARG, "not a live server");
  if (!out) return fail(BIN_ERR_INVALID_ARG, "stats is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  s->st.queued = s->queue.size();
  s->st.bytes_in_use = in_use(s);
  *out = s->st;
  return BIN_OK;
}

int binsrv_destroy(binsrv* s) {
  clear_error();
  {
    std::lock_guard<std::mutex> lk(g_live_mu);
    if (!g_live.count(s)) return fail(BIN_ERR_INVALID_ARG, "not a live server");
    g_live.erase(s);
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  s->thr.join();  // drains the queue and in-flight batches
  for (Slot& sl : s->slots) {
    (void)hipStreamSynchronize(sl.stream);
    (void)hipEventDestroy(sl.done);
    (void)hipStreamDestroy(sl.stream);
  }
  for (auto& kv : s->reqs)
    if (kv.second.grids) (void)hipFree(kv.second.grids);
  for (auto& kv : s->pool)
    for (void* p : kv.second) (void)hipFree(p);
  delete s;
  return BIN_OK;
}

}  // extern "C"
