// Admission rule of the request server (binsrv_*), as a pure function: no
// HIP, no server state, so it is tested on the CPU against a simulated
// server whose "device" only counts bytes.
//
// When a stream slot is free, the waiting requests are considered in
// arrival order.  Every byte the server commits is counted against the
// budget: result grids resident on the device, and each slot's scratch
// reservation.  The rule:
//   1. Take the longest prefix of the queue (at most max_batch requests)
//      whose grids plus its estimated scratch fit next to what is
//      committed.  The estimate is the sum of each request's own scratch,
//      as the pool would hold it.  If not even the head fits, nothing is
//      admitted: the server waits for memory to be released.
//   2. Plan the prefix as it will run and take its exact scratch.  If it
//      does not fit, halve the prefix and plan again.  A single request that
//      does not fit waits.
//   3. If a prefix cannot be planned at all, retry the head alone. If the
//      head alone cannot be planned, it is failed on its own.
// A slot's reservation is the scratch pool its stream holds; admission
// never shrinks it.  When nothing fits, the server gives the pools of its
// idle slots back and applies the rule again with those reservations at
// zero, so a request that fits the budget with the grids still resident is
// never kept out by idle scratch.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>

namespace binimpl {

// Bytes the per-stream scratch pool holds after serving a call that needs
// 'bytes': its allocation rounds up to 256 bytes and never goes below 1 MiB.
inline size_t pool_bytes_for(size_t bytes) {
  return bytes ? std::max((bytes + 255) & ~size_t(255), size_t(1) << 20) : 0;
}

struct AdmitDecision {
  size_t take = 0;     // requests admitted from the head of the queue (0: wait)
  size_t reserve = 0;  // the slot's scratch reservation while they run
  int status = 0;      // nonzero: the head request cannot be planned (take == 1): fail it
};

// out_bytes / scratch_est: the first nq waiting requests in arrival order;
// base: bytes committed apart from this slot's reservation; slot_reserved:
// that reservation; exact(take, &status): scratch of running the first
// 'take' requests as one batch (status nonzero if they cannot be planned).
template <class Exact>
AdmitDecision admit(const size_t* out_bytes, const size_t* scratch_est, size_t nq, size_t base,
                    size_t slot_reserved, size_t budget, size_t max_batch, Exact exact) {
  AdmitDecision d;
  size_t take = 0, grids = 0, est = 0;
  while (take < nq && take < max_batch) {
    const size_t scratch = std::max(slot_reserved, pool_bytes_for(est + scratch_est[take]));
    if (base + grids + out_bytes[take] + scratch > budget) break;
    grids += out_bytes[take];
    est += scratch_est[take];
    ++take;
  }
  if (take == 0) return d;
  for (;;) {
    grids = 0;
    for (size_t i = 0; i < take; ++i) grids += out_bytes[i];
    int st = 0;
    const size_t need = exact(take, &st);
    if (st) {
      if (take > 1) {
        take = 1;
        continue;
      }
      d.take = 1;
      d.status = st;
      return d;
    }
    const size_t reserve = std::max(slot_reserved, pool_bytes_for(need));
    if (base + grids + reserve <= budget) {
      d.take = take;
      d.reserve = reserve;
      return d;
    }
    if (take == 1) return d;  // fits once more memory is free
    take /= 2;
  }
}

}  // namespace binimpl
