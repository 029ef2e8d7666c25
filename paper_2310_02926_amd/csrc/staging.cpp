// Staging buffers of the asynchronous in situ mode (bin_particles_async).
//
// A deep copy is written on the simulation's stream and read on the
// analysis stream.  Each (device, source stream, binning stream) triple owns
// a small ring of buffers.  A buffer carries two events: 'copied', recorded
// on the source stream after the copy (the binning stream waits on it), and
// 'done', recorded on the binning stream after the binning.  A buffer is
// reused once its 'done' has completed; when every buffer of a full ring is
// still in use, the source stream waits on the oldest one's 'done' (back
// pressure on the simulation instead of unbounded memory).  Buffers are only
// allocated, grown and freed in the source stream's order, and only while
// idle, so no allocation is ever shared between two streams' free lists.
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "internal.h"

namespace binimpl {

namespace {

constexpr int kRingMax = 4;

struct StageBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  hipEvent_t copied = nullptr;
  hipEvent_t done = nullptr;
  uint64_t last_use = 0;
};

struct Ring {
  std::vector<StageBuf> bufs;
  uint64_t clock = 0;
};

std::mutex g_mu;
std::map<std::tuple<int, void*, void*>, Ring> g_rings;

}  // namespace

int stage_run(int device, hipStream_t src, hipStream_t bs, size_t bytes,
              const std::function<int(void* stage)>& copy, const std::function<int(void* stage)>& bin) {
  std::lock_guard<std::mutex> lk(g_mu);
  Ring& ring = g_rings[std::make_tuple(device, (void*)src, (void*)bs)];
  // An idle buffer (its last binning has completed), the largest first.
  int pick = -1;
  for (int i = 0; i < (int)ring.bufs.size(); ++i) {
    const hipError_t q = hipEventQuery(ring.bufs[i].done);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) return hip_fail(q, "hipEventQuery(staging)");
    if (pick < 0 || ring.bufs[i].bytes > ring.bufs[pick].bytes) pick = i;
  }
  if (pick < 0 && (int)ring.bufs.size() < kRingMax) {
    StageBuf b;
    hipError_t e = hipEventCreateWithFlags(&b.copied, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b.done, hipEventDisableTiming);
    if (e != hipSuccess) {
      if (b.copied) (void)hipEventDestroy(b.copied);
      return hip_fail(e, "hipEventCreate(staging)");
    }
    ring.bufs.push_back(b);
    pick = (int)ring.bufs.size() - 1;
  }
  if (pick < 0) {  // ring full and busy: wait (on the source stream) for the oldest
    pick = 0;
    for (int i = 1; i < (int)ring.bufs.size(); ++i)
      if (ring.bufs[i].last_use < ring.bufs[pick].last_use) pick = i;
    const hipError_t e = hipStreamWaitEvent(src, ring.bufs[pick].done, 0);
    if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent(staging)");
  }
  StageBuf& b = ring.bufs[pick];
  if (b.bytes < bytes) {
    if (b.ptr) {
      const hipError_t e = hipFreeAsync(b.ptr, src);
      b.ptr = nullptr;
      b.bytes = 0;
      if (e != hipSuccess) return hip_fail(e, "hipFreeAsync(staging)");
    }
    if (fault_injection_hit()) return fail(BIN_ERR_OOM, "injected staging allocation failure");
    const hipError_t e = hipMallocAsync(&b.ptr, bytes, src);
    if (e != hipSuccess) {
      b.ptr = nullptr;
      return hip_fail(e, "hipMallocAsync(staging)");
    }
    b.bytes = bytes;
  }
  b.last_use = ++ring.clock;
  int st = copy(b.ptr);
  if (st) return st;
  hipError_t e = hipEventRecord(b.copied, src);
  if (e == hipSuccess) e = hipStreamWaitEvent(bs, b.copied, 0);
  if (e != hipSuccess) return hip_fail(e, "order binning after staging copy");
  st = bin(b.ptr);
  // Recorded whatever the binning returned, so the buffer is reclaimed.
  e = hipEventRecord(b.done, bs);
  if (e != hipSuccess && st == BIN_OK) st = hip_fail(e, "hipEventRecord(staging done)");
  return st;
}

int release_all_staging() {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : g_rings)
    for (StageBuf& b : kv.second.bufs) {
      if (b.ptr) (void)hipFree(b.ptr);
      if (b.copied) (void)hipEventDestroy(b.copied);
      if (b.done) (void)hipEventDestroy(b.done);
    }
  g_rings.clear();
  return BIN_OK;
}

}  // namespace binimpl
