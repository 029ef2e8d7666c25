// Request server with continuous batching (binsrv_*).
//
// Requests wait in arrival order.  Work is admitted whenever something can
// make room for it - a submission, a finished batch, a released grid - by
// the thread that caused it: whenever a stream slot is free, the waiting
// requests at the head of the queue whose result grids and scratch fit the
// device-memory budget are launched on that slot's stream as one batch (a
// lone request runs the single-request kernels).  So a request that finds a
// slot free is launched by binsrv_submit itself, and requests that arrive
// while every slot is busy are batched together when the next slot frees.
// Each slot has a waiter thread that blocks on the slot's completion event
// and stamps its requests done the moment the batch finishes.  Result grids
// come from a reuse pool keyed by size class and stay resident until
// binsrv_release(); device memory is allocated and freed outside the lock.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <set>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"
#include "server_admit.h"

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
  size_t scratch_est = 0;   // scratch of running it alone (the plan that runs it)
  hipEvent_t ready = nullptr;  // recorded on the producer stream at submit, or null
  int slot = -1;               // slot running it, and that slot's launch number
  uint64_t slot_seq = 0;
  // resident result grids (device), one allocation
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
  bool launched = false;  // a batch was enqueued and its event recorded; the waiter owns the slot
  uint64_t seq = 0;       // launches so far (tells a batch's event from a later one's)
  std::vector<uint64_t> tickets;
  size_t scratch_reserved = 0;  // bytes of the library pool this slot's stream holds
  std::condition_variable cv;
  std::thread waiter;
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
  // Blocks come in size classes (2^j and 3 * 2^(j-1) bytes, at least
  // 64 KiB), so that released blocks serve later requests of other grid
  // shapes and the pool rarely has to allocate: at most a third is unused.
  size_t c = size_t(1) << 16;
  while (c < b) c = (c & (c - 1)) ? (c / 3) * 4 : c + c / 2;  // 2^j -> 1.5 * 2^j -> 2^(j+1)
  return c;
}

}  // namespace

struct binsrv {
  binsrv_config cfg{};
  std::mutex mu;
  std::condition_variable cv_done;  // waiters
  bool stop = false;      // no more submissions
  bool quit = false;      // slot waiters exit once their slot is idle
  uint64_t next_ticket = 1;
  std::deque<uint64_t> queue;
  std::unordered_map<uint64_t, SrvReq> reqs;
  std::vector<std::unique_ptr<Slot>> slots;
  std::unordered_map<size_t, std::vector<void*>> pool;  // free result blocks by size
  size_t pool_bytes = 0;       // bytes in free pool blocks
  size_t resident_bytes = 0;   // bytes of blocks held (or being allocated) for requests
  int dispatching = 0;         // dispatches between admission and launch
  binsrv_stats st{};
  std::atomic<int> users{0};   // entry points currently using this server
};

namespace {

std::mutex g_live_mu;
std::set<binsrv*> g_live;

// A reference to a live server for the duration of one entry point call:
// binsrv_destroy removes the server from the live set first and then waits
// until no call holds a reference, so a concurrent call either sees it dead
// or keeps it alive until it returns.
struct SrvRef {
  binsrv* s = nullptr;
  explicit SrvRef(binsrv* p) {
    std::lock_guard<std::mutex> lk(g_live_mu);
    if (g_live.count(p)) {
      s = p;
      s->users.fetch_add(1);
    }
  }
  ~SrvRef() {
    if (s) s->users.fetch_sub(1);
  }
  SrvRef(const SrvRef&) = delete;
  SrvRef& operator=(const SrvRef&) = delete;
};

size_t in_use(const binsrv* s) {
  size_t b = s->pool_bytes + s->resident_bytes;
  for (const auto& sl : s->slots) b += sl->scratch_reserved;
  return b;
}

// Memory that cannot be reclaimed right now (pooled free blocks can).
size_t committed(const binsrv* s) { return in_use(s) - s->pool_bytes; }

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

// The request as a bin_request; with stand-in output pointers when the grids
// are not allocated yet (sizing only).
bin_request as_bin_request(SrvReq& q) {
  // stand-ins: non-null, suitably aligned, never dereferenced
  static void* const fake[BIN_MAX_ATTRS] = {
      (void*)0x1000, (void*)0x2000, (void*)0x3000, (void*)0x4000, (void*)0x5000, (void*)0x6000,
      (void*)0x7000, (void*)0x8000, (void*)0x9000, (void*)0xA000, (void*)0xB000, (void*)0xC000,
      (void*)0xD000, (void*)0xE000, (void*)0xF000, (void*)0x10000};
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
  if (q.grids) {
    b.out.count = q.count;
    b.out.sum = q.sum;
    b.out.min = q.mn;
    b.out.max = q.mx;
    b.out.avg = q.avg;
  } else {
    b.out.count = reinterpret_cast<uint32_t*>(uintptr_t(4096));
    b.out.sum = b.out.min = b.out.max = b.out.avg = const_cast<void* const*>(fake);
  }
  return b;
}

// Scratch the batch of these requests needs as it will run: the
// single-request plan for one request, the batch plan for several.
size_t exact_scratch(std::vector<bin_request>& brs, int* status) {
  *status = BIN_OK;
  if (brs.size() == 1) {
    DeviceInfo dev;
    *status = device_info(&dev);
    if (*status) return 0;
    Prepared p;
    *status = prepare(brs[0], dev, PlanHints{}, nullptr, &p);
    return *status ? 0 : p.scratch_bytes;
  }
  return batch_scratch_bytes(brs.data(), (int)brs.size(), status);
}

void fail_request(binsrv* s, SrvReq& q, int status) {
  q.state = Q_DONE;
  q.status = status;
  q.t_done = clk::now();
  s->st.failed++;
}

// Admit and launch one batch on a free slot.  Called with the lock held by
// whichever thread made room (submit, a slot waiter, release); the lock is
// dropped while memory is allocated and kernels are enqueued.  Returns true
// if it launched (or failed) something, so that the caller tries again.
bool dispatch_one(binsrv* s, std::unique_lock<std::mutex>& lk) {
  Slot* sl = nullptr;
  int sl_index = -1;
  for (size_t i = 0; i < s->slots.size(); ++i)
    if (!s->slots[i]->busy) {
      sl = s->slots[i].get();
      sl_index = (int)i;
      break;
    }
  if (!sl || s->queue.empty()) return false;
  // The admission rule (server_admit.h) over the head of the queue; the
  // exact scratch of a candidate batch comes from the plan that will run it.
  const size_t nq = std::min(s->queue.size(), (size_t)std::max(s->cfg.max_batch, 1));
  std::vector<size_t> out_bytes(nq), scratch_est(nq);
  for (size_t i = 0; i < nq; ++i) {
    const SrvReq& q = s->reqs[s->queue[i]];
    out_bytes[i] = q.out_bytes;
    scratch_est[i] = q.scratch_est;
  }
  auto exact = [&](size_t take, int* st) {
    std::vector<bin_request> brs;
    for (size_t i = 0; i < take; ++i) brs.push_back(as_bin_request(s->reqs[s->queue[i]]));
    return exact_scratch(brs, st);
  };
  AdmitDecision d = admit(out_bytes.data(), scratch_est.data(), nq, committed(s) - sl->scratch_reserved,
                          sl->scratch_reserved, s->cfg.budget_bytes, (size_t)s->cfg.max_batch, exact);
  if (d.take == 0) {
    // The scratch pools of idle slots may be what keeps the head out: they
    // are given back (in their streams' order) and the head tried again.
    bool freed = false;
    for (auto& o : s->slots)
      if (!o->busy && o->scratch_reserved) {
        (void)scratch_release(s->cfg.device, o->stream);
        o->scratch_reserved = 0;
        freed = true;
      }
    if (freed)
      d = admit(out_bytes.data(), scratch_est.data(), nq, committed(s), 0, s->cfg.budget_bytes,
                (size_t)s->cfg.max_batch, exact);
    if (d.take == 0) return false;  // wait for running work or released grids
  }
  if (d.status) {  // cannot be planned: fail the head request alone
    SrvReq& q = s->reqs[s->queue.front()];
    s->queue.pop_front();
    fail_request(s, q, d.status);
    s->cv_done.notify_all();
    return true;
  }
  std::vector<uint64_t> batch(s->queue.begin(), s->queue.begin() + (std::ptrdiff_t)d.take);
  const size_t reserve = d.reserve;
  // Commit: the slot, its scratch reservation, the members' grid bytes.
  for (size_t i = 0; i < batch.size(); ++i) s->queue.pop_front();
  sl->busy = true;
  sl->launched = false;
  sl->seq++;
  sl->tickets = batch;
  sl->scratch_reserved = reserve;
  const clk::time_point now = clk::now();
  std::vector<std::pair<SrvReq*, void*>> members;  // request, pooled block (or null: allocate)
  for (uint64_t t : batch) {
    SrvReq& q = s->reqs[t];
    q.state = Q_RUNNING;
    q.t_dispatch = now;
    q.dispatched = true;
    q.slot = sl_index;
    q.slot_seq = sl->seq;
    void* blk = nullptr;
    auto it = s->pool.find(q.out_bytes);
    if (it != s->pool.end() && !it->second.empty()) {
      blk = it->second.back();
      it->second.pop_back();
      s->pool_bytes -= q.out_bytes;
    }
    s->resident_bytes += q.out_bytes;
    members.emplace_back(&q, blk);
  }
  // Pooled blocks of other sizes go back to the device while the budget is
  // tight.
  std::vector<void*> evict;
  for (auto& kv : s->pool)
    while (!kv.second.empty() && in_use(s) > s->cfg.budget_bytes) {
      evict.push_back(kv.second.back());
      kv.second.pop_back();
      s->pool_bytes -= kv.first;
    }
  s->st.batches++;
  s->st.in_flight += batch.size();
  s->st.queued = s->queue.size();
  s->st.bytes_in_use = in_use(s);
  s->st.peak_bytes = std::max<uint64_t>(s->st.peak_bytes, s->st.bytes_in_use);
  s->dispatching++;
  lk.unlock();

  for (void* p : evict) (void)hipFree(p);
  // Grids: pooled blocks, else fresh allocations (a failed one fails only
  // its own request).
  std::vector<int> status(members.size(), BIN_OK);
  std::vector<bin_request> run;
  std::vector<hipEvent_t> ready;
  for (size_t i = 0; i < members.size(); ++i) {
    SrvReq& q = *members[i].first;
    void* blk = members[i].second;
    if (!blk) {
      if (fault_injection_hit()) {
        status[i] = fail(BIN_ERR_OOM, "injected result-grid allocation failure");
      } else {
        const hipError_t e = hipMalloc(&blk, q.out_bytes);
        if (e != hipSuccess) {
          blk = nullptr;
          status[i] = hip_fail(e, "hipMalloc(result grids)");
        }
      }
    }
    if (status[i] != BIN_OK) continue;
    q.grids = blk;
    q.grid_bytes = q.out_bytes;
    carve_outputs(q);
    run.push_back(as_bin_request(q));
    if (q.ready) ready.push_back(q.ready);
  }
  // Inputs written on a producer stream are read only after that work.
  int st = BIN_OK;
  for (hipEvent_t ev : ready) {
    const hipError_t e = hipStreamWaitEvent(sl->stream, ev, 0);
    if (e != hipSuccess && st == BIN_OK) st = hip_fail(e, "hipStreamWaitEvent(producer)");
  }
  if (st == BIN_OK && !run.empty())
    st = run.size() == 1 ? run_request(run[0], sl->stream, PlanHints{})
                         : run_batch(run.data(), (int)run.size(), sl->stream, PlanHints{});
  const hipError_t er = hipEventRecord(sl->done, sl->stream);

  lk.lock();
  s->dispatching--;
  for (size_t i = 0; i < members.size(); ++i) {
    SrvReq& q = *members[i].first;
    if (status[i] != BIN_OK) {  // its grid never existed
      s->resident_bytes -= q.out_bytes;
      fail_request(s, q, status[i]);
      s->st.in_flight--;
    } else if (st != BIN_OK) {  // the launch failed: the batch's requests fail
      fail_request(s, q, st);
      s->st.in_flight--;
    }
  }
  if (st != BIN_OK || er != hipSuccess) {
    std::vector<uint64_t> keep;
    sl->tickets.swap(keep);  // every member is failed above (or below)
    if (er != hipSuccess) {
      for (uint64_t t : keep) {
        SrvReq& q = s->reqs[t];
        if (q.state != Q_DONE) {
          fail_request(s, q, hip_fail(er, "hipEventRecord(slot)"));
          s->st.in_flight--;
        }
      }
      // No event to wait on: drain the stream here, then the slot is free.
      lk.unlock();
      (void)hipStreamSynchronize(sl->stream);
      lk.lock();
      sl->busy = false;
      s->cv_done.notify_all();
      return true;
    }
  } else {
    // drop failed members; the rest complete with the slot's event
    std::vector<uint64_t> keep;
    for (uint64_t t : sl->tickets)
      if (s->reqs[t].state != Q_DONE) keep.push_back(t);
    sl->tickets.swap(keep);
  }
  sl->launched = true;
  sl->cv.notify_one();
  s->cv_done.notify_all();
  return true;
}

void dispatch_all(binsrv* s, std::unique_lock<std::mutex>& lk) {
  while (dispatch_one(s, lk)) {
  }
}

// The slot's batch (launch number seq) has finished with status e at 'now':
// stamp its requests done, free the slot and admit waiting work.  Called
// with the lock held by whichever thread saw the event first - the slot's
// waiter, or a client in binsrv_wait - and a no-op for the other.
void complete_slot(binsrv* s, Slot* sl, uint64_t seq, hipError_t e, clk::time_point now,
                   std::unique_lock<std::mutex>& lk) {
  if (!sl->launched || sl->seq != seq) return;
  for (uint64_t t : sl->tickets) {
    auto it = s->reqs.find(t);
    if (it == s->reqs.end() || it->second.state == Q_DONE) continue;
    it->second.state = Q_DONE;
    it->second.t_done = now;
    it->second.status = e == hipSuccess ? BIN_OK : BIN_ERR_DEVICE;
    if (e == hipSuccess) s->st.completed++;
    else s->st.failed++;
    s->st.in_flight--;
  }
  sl->tickets.clear();
  sl->launched = false;
  sl->busy = false;
  s->cv_done.notify_all();
  dispatch_all(s, lk);
}

// One per slot: waits for the slot's batch to finish (the completion event,
// outside the lock) and completes it.
void slot_waiter(binsrv* s, Slot* sl) {
  (void)hipSetDevice(s->cfg.device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    sl->cv.wait(lk, [&] { return sl->launched || (s->quit && !sl->busy); });
    if (!sl->launched) break;
    hipEvent_t ev = sl->done;
    const uint64_t seq = sl->seq;
    lk.unlock();
    const hipError_t e = hipEventSynchronize(ev);
    const clk::time_point now = clk::now();
    lk.lock();
    complete_slot(s, sl, seq, e, now, lk);
  }
}

int check_request(const binsrv_request* req) {
  bin_output none;
  std::memset(&none, 0, sizeof none);
  // Validate with stand-in outputs (the server owns the real ones).
  void* fake[BIN_MAX_ATTRS];
  for (int j = 0; j < BIN_MAX_ATTRS; ++j) fake[j] = reinterpret_cast<void*>(uintptr_t(256) * (j + 1));
  none.count = reinterpret_cast<uint32_t*>(uintptr_t(4096));
  none.sum = none.min = none.max = none.avg = fake;
  return validate(&req->coords, &req->attrs, req->n, req->axes, req->bounds, req->nx, req->ny, req->ops, &none,
                  false);
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
  for (int i = 0; i < cfg->n_slots; ++i) {
    auto sl = std::make_unique<Slot>();
    e = hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl->done, hipEventDisableTiming);
    if (e != hipSuccess) {
      if (sl->stream) (void)hipStreamDestroy(sl->stream);
      for (auto& x : s->slots) {
        (void)hipEventDestroy(x->done);
        (void)hipStreamDestroy(x->stream);
      }
      delete s;
      return hip_fail(e, "server stream setup");
    }
    s->slots.push_back(std::move(sl));
  }
  for (auto& sl : s->slots) sl->waiter = std::thread(slot_waiter, s, sl.get());
  {
    std::lock_guard<std::mutex> lk(g_live_mu);
    g_live.insert(s);
  }
  *out = s;
  return BIN_OK;
}

int binsrv_submit(binsrv* srv, const binsrv_request* req, uint64_t* ticket) {
  const clk::time_point t_arrival = clk::now();
  clear_error();
  SrvRef ref(srv);
  binsrv* s = ref.s;
  if (!s) return fail(BIN_ERR_INVALID_ARG, "not a live server");
  if (!req || !ticket) return fail(BIN_ERR_INVALID_ARG, "req or ticket is NULL");
  int st = check_request(req);
  if (st) return st;
  SrvReq q;
  q.r = *req;
  q.coord_cols.assign(req->coords.cols, req->coords.cols + req->coords.ncols);
  if (req->attrs.cols && req->attrs.ncols > 0) q.attr_cols.assign(req->attrs.cols, req->attrs.cols + req->attrs.ncols);
  q.out_bytes = grid_bytes_of(*req);
  // Can it ever fit?  Its grids plus the scratch of running it alone (the
  // single-request plan that runs a lone request).
  std::vector<bin_request> alone{as_bin_request(q)};
  const size_t need = exact_scratch(alone, &st);
  if (st) return st;
  q.scratch_est = need;
  if (q.out_bytes + pool_bytes_for(need) > s->cfg.budget_bytes)
    return fail(BIN_ERR_ADMISSION, "request needs %zu bytes, budget is %llu", q.out_bytes + pool_bytes_for(need),
                (unsigned long long)s->cfg.budget_bytes);
  if (req->producer_stream) {
    hipError_t e = hipEventCreateWithFlags(&q.ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(q.ready, static_cast<hipStream_t>(req->producer_stream));
    if (e != hipSuccess) {
      if (q.ready) (void)hipEventDestroy(q.ready);
      return hip_fail(e, "record the producer stream's event");
    }
  }
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->stop) {
    if (q.ready) (void)hipEventDestroy(q.ready);
    return fail(BIN_ERR_INVALID_ARG, "server is shutting down");
  }
  q.ticket = s->next_ticket++;
  q.t_submit = t_arrival;
  *ticket = q.ticket;
  s->queue.push_back(q.ticket);
  s->reqs.emplace(q.ticket, std::move(q));
  s->st.submitted++;
  s->st.queued = s->queue.size();
  dispatch_all(s, lk);  // a free slot takes it at once
  return BIN_OK;
}

int binsrv_wait(binsrv* srv, uint64_t ticket, int64_t timeout_ns, bin_result* res) {
  clear_error();
  SrvRef ref(srv);
  binsrv* s = ref.s;
  if (!s) return fail(BIN_ERR_INVALID_ARG, "not a live server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto done = [&] {
    auto it = s->reqs.find(ticket);
    return it == s->reqs.end() || it->second.state == Q_DONE;
  };
  // A launched request is observed directly: this thread waits on its
  // batch's completion event (as a caller of a plain launch would wait on
  // its stream), so the result is seen without a hand-over between threads.
  if (timeout_ns < 0) {
    auto it = s->reqs.find(ticket);
    if (it != s->reqs.end() && it->second.state == Q_RUNNING && it->second.slot >= 0) {
      Slot* sl = s->slots[it->second.slot].get();
      const uint64_t seq = it->second.slot_seq;
      if (sl->launched && sl->seq == seq) {
        hipEvent_t ev = sl->done;
        lk.unlock();
        const hipError_t e = hipEventSynchronize(ev);
        const clk::time_point now = clk::now();
        lk.lock();
        complete_slot(s, sl, seq, e, now, lk);
      }
    }
  }
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
  if (q.status != BIN_OK) return fail(q.status, "ticket %llu failed", (unsigned long long)ticket);
  return BIN_OK;
}

int binsrv_release(binsrv* srv, uint64_t ticket) {
  clear_error();
  SrvRef ref(srv);
  binsrv* s = ref.s;
  if (!s) return fail(BIN_ERR_INVALID_ARG, "not a live server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(BIN_ERR_NOT_FOUND, "unknown or already released ticket %llu", (unsigned long long)ticket);
  if (it->second.state != Q_DONE) return fail(BIN_ERR_INVALID_ARG, "ticket %llu is not finished", (unsigned long long)ticket);
  give_block(s, it->second.grids, it->second.grid_bytes);
  hipEvent_t ready = it->second.ready;
  s->reqs.erase(it);
  s->st.released++;
  s->st.bytes_in_use = in_use(s);
  dispatch_all(s, lk);  // the released memory may admit waiting requests
  lk.unlock();
  if (ready) (void)hipEventDestroy(ready);
  return BIN_OK;
}

int binsrv_get_stats(binsrv* srv, binsrv_stats* out) {
  clear_error();
  SrvRef ref(srv);
  binsrv* s = ref.s;
  if (!s) return fail(BIN_ERR_INVALID_ARG, "not a live server");
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
    g_live.erase(s);  // no new references from here on
  }
  {
    // Drain: waiting requests still run (a request that can never be
    // admitted is failed), then the slot waiters exit.
    std::unique_lock<std::mutex> lk(s->mu);
    s->stop = true;
    for (;;) {
      dispatch_all(s, lk);
      bool busy = s->dispatching > 0;
      for (auto& sl : s->slots) busy |= sl->busy;
      if (!busy && !s->queue.empty()) {  // nothing running and the head cannot be admitted
        SrvReq& q = s->reqs[s->queue.front()];
        s->queue.pop_front();
        fail_request(s, q, BIN_ERR_ADMISSION);
        s->cv_done.notify_all();
        continue;
      }
      if (!busy) break;
      s->cv_done.wait(lk);
    }
    s->quit = true;
    for (auto& sl : s->slots) sl->cv.notify_one();
  }
  for (auto& sl : s->slots) sl->waiter.join();
  // Calls that took a reference before the server left the live set return
  // promptly now (every request is done); wait for them.
  while (s->users.load() > 0) std::this_thread::yield();
  for (auto& sl : s->slots) {
    (void)hipStreamSynchronize(sl->stream);
    (void)hipEventDestroy(sl->done);
    (void)hipStreamDestroy(sl->stream);
  }
  for (auto& kv : s->reqs) {
    if (kv.second.grids) (void)hipFree(kv.second.grids);
    if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
  }
  for (auto& kv : s->pool)
    for (void* p : kv.second) (void)hipFree(p);
  delete s;
  return BIN_OK;
}

}  // extern "C"
