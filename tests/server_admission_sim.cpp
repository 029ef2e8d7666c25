// CPU test of the request server's admission rule (server_admit.h), with a
// simulated device in place of the GPU: slots that finish after a random
// number of steps, grids and scratch that are only byte counts, and a
// planner double whose batch scratch is a made-up function of its members
// (some requests cannot be planned at all).  Built and run by
// tests/test_server_admission.py; exits nonzero with a message on the first
// broken invariant.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <random>
#include <vector>

#include "../paper_2310_02926_amd/csrc/server_admit.h"

using binimpl::admit;
using binimpl::AdmitDecision;
using binimpl::pool_bytes_for;

namespace {

int g_fail = 0;
#define CHECK(cond, ...)                                   \
  do {                                                     \
    if (!(cond)) {                                         \
      std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
      std::fprintf(stderr, __VA_ARGS__);                   \
      std::fprintf(stderr, "\n");                          \
      ++g_fail;                                            \
      return;                                              \
    }                                                      \
  } while (0)

struct Req {
  size_t out_bytes, scratch_est, alone;  // alone: exact scratch of running it by itself
  bool plannable;
  int state = 0;  // 0 waiting, 1 running, 2 done (resident), 3 released, 4 failed
};

// The planner double: a batch needs its members' scratch plus 64 KiB of
// tables per member; it cannot be planned if any member cannot.
size_t plan(const std::vector<Req>& reqs, const std::deque<int>& q, size_t take, int* st) {
  size_t b = 0;
  for (size_t i = 0; i < take; ++i) {
    const Req& r = reqs[q[i]];
    if (!r.plannable) {
      *st = 7;
      return 0;
    }
    b += take == 1 ? r.alone : r.alone + (64u << 10);
  }
  *st = 0;
  return b;
}

void unit_cases() {
  const size_t M = 1 << 20;
  // nothing fits: the head's grids alone exceed what is left
  {
    size_t ob[] = {10 * M}, se[] = {0};
    auto d = admit(ob, se, 1, 95 * M, 0, 100 * M, 8, [](size_t, int* st) { *st = 0; return size_t(0); });
    CHECK(d.take == 0 && d.status == 0, "take %zu", d.take);
  }
  // the estimate admits four, the exact plan needs more: halved to two
  {
    size_t ob[] = {10 * M, 10 * M, 10 * M, 10 * M}, se[] = {M, M, M, M};
    auto exact = [&](size_t take, int* st) {
      *st = 0;
      return take * 20 * M;
    };
    auto d = admit(ob, se, 4, 0, 0, 100 * M, 8, exact);
    CHECK(d.take == 2 && d.reserve == 40 * M, "take %zu reserve %zu", d.take, d.reserve);
  }
  // a member that cannot be planned: the head is retried alone and runs
  {
    size_t ob[] = {M, M, M}, se[] = {M, M, M};
    auto exact = [&](size_t take, int* st) {
      *st = take > 1 ? 5 : 0;
      return take * M;
    };
    auto d = admit(ob, se, 3, 0, 0, 100 * M, 8, exact);
    CHECK(d.take == 1 && d.status == 0, "take %zu status %d", d.take, d.status);
  }
  // the head alone cannot be planned: it is failed on its own
  {
    size_t ob[] = {M, M}, se[] = {M, M};
    auto d = admit(ob, se, 2, 0, 0, 100 * M, 8, [](size_t, int* st) { *st = 9; return size_t(0); });
    CHECK(d.take == 1 && d.status == 9, "take %zu status %d", d.take, d.status);
  }
  // max_batch caps the prefix; the slot's reservation never shrinks
  {
    size_t ob[] = {M, M, M, M, M}, se[] = {0, 0, 0, 0, 0};
    auto d = admit(ob, se, 5, 0, 8 * M, 100 * M, 3, [](size_t, int* st) { *st = 0; return size_t(0); });
    CHECK(d.take == 3 && d.reserve == 8 * M, "take %zu reserve %zu", d.take, d.reserve);
  }
  // the pool's rounding: a request needing 1 byte of scratch holds 1 MiB
  CHECK(pool_bytes_for(1) == M && pool_bytes_for(0) == 0 && pool_bytes_for(M + 1) == M + 256, "pool rounding");
}

// A whole server on the simulated device: random arrivals, slots that
// finish after a random number of steps, clients that release results.
void simulate(unsigned seed) {
  std::mt19937_64 rng(seed);
  const size_t M = 1 << 20;
  const size_t budget = (64 + rng() % 192) * M;
  const int nslots = 1 + (int)(rng() % 4);
  const size_t max_batch = 1 + rng() % 16;
  std::vector<Req> reqs;
  std::deque<int> queue;
  struct Slot {
    bool busy = false;
    int left = 0;
    size_t reserved = 0;
    std::vector<int> members;
  };
  std::vector<Slot> slots(nslots);
  size_t resident = 0;  // grids of running and finished, unreleased requests
  std::vector<int> finished;
  const int n_req = 400;
  int submitted = 0, steps = 0;
  auto committed = [&] {
    size_t c = resident;
    for (const Slot& sl : slots) c += sl.reserved;
    return c;
  };
  auto dispatch = [&] {
    for (Slot& sl : slots) {
      if (sl.busy || queue.empty()) continue;
      for (;;) {
        if (queue.empty()) break;
        const size_t nq = std::min(queue.size(), max_batch);
        std::vector<size_t> ob(nq), se(nq);
        for (size_t i = 0; i < nq; ++i) {
          ob[i] = reqs[queue[i]].out_bytes;
          se[i] = reqs[queue[i]].scratch_est;
        }
        auto exact = [&](size_t take, int* st) { return plan(reqs, queue, take, st); };
        AdmitDecision d = admit(ob.data(), se.data(), nq, committed() - sl.reserved, sl.reserved, budget,
                                max_batch, exact);
        if (d.take == 0) {  // the server gives idle slots' scratch back and tries again
          bool freed = false;
          for (Slot& o : slots)
            if (!o.busy && o.reserved) {
              o.reserved = 0;
              freed = true;
            }
          if (freed) d = admit(ob.data(), se.data(), nq, committed(), 0, budget, max_batch, exact);
        }
        if (d.take == 0) break;
        if (d.status) {
          CHECK(!reqs[queue.front()].plannable, "a plannable head was failed");
          reqs[queue.front()].state = 4;
          queue.pop_front();
          continue;
        }
        CHECK(d.take <= max_batch, "batch of %zu above max_batch %zu", d.take, max_batch);
        CHECK(d.reserve >= sl.reserved, "admission shrank a reservation");
        sl.reserved = d.reserve;
        sl.busy = true;
        sl.left = 1 + (int)(rng() % 5);
        sl.members.clear();
        for (size_t i = 0; i < d.take; ++i) {
          const int t = queue.front();
          queue.pop_front();
          CHECK(reqs[t].plannable, "an unplannable request was launched");
          reqs[t].state = 1;
          resident += reqs[t].out_bytes;
          sl.members.push_back(t);
        }
        CHECK(committed() <= budget, "committed %zu above budget %zu", committed(), budget);
        break;
      }
    }
  };
  while ((submitted < n_req || !queue.empty() || !finished.empty() ||
          std::any_of(slots.begin(), slots.end(), [](const Slot& s) { return s.busy; })) &&
         steps < 200000) {
    ++steps;
    // arrivals
    for (int a = (int)(rng() % 3); a > 0 && submitted < n_req; --a, ++submitted) {
      Req r;
      r.out_bytes = binimpl::pool_bytes_for((rng() % 24 + 1) * M / (1 + rng() % 4)) / 4;
      r.alone = (rng() % 8) * (budget / 20);  // up to 35% of the budget: idle slots' pools can block
      r.scratch_est = r.alone;
      r.plannable = rng() % 50 != 0;
      // admission at submit: a request that can never fit is refused
      if (r.out_bytes + pool_bytes_for(r.alone) > budget) continue;
      reqs.push_back(r);
      queue.push_back((int)reqs.size() - 1);
    }
    dispatch();
    if (g_fail) return;
    // the device: slots count down, finished batches become resident results
    for (Slot& sl : slots)
      if (sl.busy && --sl.left == 0) {
        sl.busy = false;
        for (int t : sl.members) {
          reqs[t].state = 2;
          finished.push_back(t);
        }
      }
    dispatch();
    if (g_fail) return;
    // clients release some finished results
    while (!finished.empty() && rng() % 2) {
      const size_t i = rng() % finished.size();
      const int t = finished[i];
      finished.erase(finished.begin() + (std::ptrdiff_t)i);
      reqs[t].state = 3;
      resident -= reqs[t].out_bytes;
    }
    dispatch();
    if (g_fail) return;
  }
  CHECK(steps < 200000, "seed %u: no progress (queue %zu)", seed, queue.size());
  // every plannable request ran and was released; the others failed
  for (const Req& r : reqs)
    CHECK(r.plannable ? r.state == 3 : r.state == 4, "seed %u: request ended in state %d", seed, r.state);
  CHECK(resident == 0, "seed %u: %zu bytes still resident", seed, resident);
}

}  // namespace

int main() {
  unit_cases();
  for (unsigned seed = 1; seed <= 300 && !g_fail; ++seed) simulate(seed);
  if (g_fail) return 1;
  std::printf("ok\n");
  return 0;
}
