// Autotuner: times candidate launch configurations for representative
// requests and remembers the fastest per shape class.  The planner looks the
// class up whenever the caller set no explicit override.
//
// Shape class: log2 buckets of n and of the bin count, attribute count,
// coordinate and attribute types, precision and op mask.  The table lives in
// memory and, when the environment variable BIN_TUNE_CACHE names a file, is
// loaded from and saved to that file (one "key value..." line per class).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "internal.h"

namespace binimpl {

namespace {

std::mutex g_tune_mu;
std::map<std::string, PlanHints> g_tune;
bool g_tune_loaded = false;

int log2_bucket(int64_t v) {
  int b = 0;
  while (v > 1) {
    v >>= 1;
    ++b;
  }
  return b;
}

std::string class_key(const bin_request& r) {
  const int k = r.attrs.cols ? r.attrs.ncols : 0;
  char buf[128];
  snprintf(buf, sizeof buf, "n%d_b%d_k%d_c%d_a%d_o%u", log2_bucket(r.n), log2_bucket((int64_t)r.nx * r.ny), k,
           r.coords.dtype, k ? r.attrs.dtype : 0, r.ops);
  return buf;
}

const char* cache_path() { return getenv("BIN_TUNE_CACHE"); }

void load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* p = cache_path();
  if (!p) return;
  std::ifstream f(p);
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    std::string key;
    PlanHints h;
    long long split = 0;
    if (is >> key >> h.force_strategy >> h.block >> h.grid >> h.part_wg >> h.scatter_ppt >> h.scatter_threads >>
        h.tile_shift >> split) {
      h.split_len = split;
      g_tune[key] = h;
    }
  }
}

void save_locked() {
  const char* p = cache_path();
  if (!p) return;
  std::ofstream f(p, std::ios::trunc);
  for (auto& kv : g_tune) {
    const PlanHints& h = kv.second;
    f << kv.first << ' ' << h.force_strategy << ' ' << h.block << ' ' << h.grid << ' ' << h.part_wg << ' '
      << h.scatter_ppt << ' ' << h.scatter_threads << ' ' << h.tile_shift << ' ' << (long long)h.split_len << '\n';
  }
}

bool is_default(const PlanHints& h) {
  return h.force_strategy < 0 && !h.block && !h.grid && !h.part_wg && !h.scatter_ppt && !h.scatter_threads &&
         !h.tile_shift && !h.split_len && !h.quads;
}

}  // namespace

// Hints for a request: the caller's explicit override if any, else the
// tuned entry of its shape class, else defaults.
PlanHints effective_hints(const bin_request& r, const PlanHints& explicit_hints) {
  if (!is_default(explicit_hints)) return explicit_hints;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_locked();
  auto it = g_tune.find(class_key(r));
  return it == g_tune.end() ? explicit_hints : it->second;
}

namespace {

// Median-of-3 time of one configuration, on a private stream.
int time_config(const bin_request& r, const PlanHints& h, hipStream_t s, hipEvent_t e0, hipEvent_t e1, float* ms) {
  int st = run_request(r, s, h);  // warm-up (and validates the configuration)
  if (st) return st;
  float t[3];
  for (int i = 0; i < 3; ++i) {
    hipError_t e = hipEventRecord(e0, s);
    if (e == hipSuccess) st = run_request(r, s, h);
    if (st) return st;
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&t[i], e0, e1);
    if (e != hipSuccess) return hip_fail(e, "autotune timing");
  }
  std::sort(t, t + 3);
  *ms = t[1];
  return BIN_OK;
}

}  // namespace

int autotune(const bin_request* reqs, int count) {
  if (!reqs || count <= 0) return fail(BIN_ERR_INVALID_ARG, "autotune needs at least one request");
  for (int i = 0; i < count; ++i) {
    const bin_request& r = reqs[i];
    int st = validate(&r.coords, &r.attrs, r.n, r.axes, r.bounds, r.nx, r.ny, r.ops, &r.out, false);
    if (st) return st;
  }
  DeviceInfo dev;
  int st = device_info(&dev);
  if (st) return st;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return hip_fail(e, "autotune setup");
  const int cus = dev.cus;
  for (int i = 0; i < count && st == BIN_OK; ++i) {
    const bin_request& r = reqs[i];
    Prepared p;
    st = prepare(r, dev, PlanHints{}, nullptr, &p);
    if (st) break;
    std::vector<PlanHints> cands;
    PlanHints base;
    cands.push_back(base);
    if (p.cfg.strategy == bk::STRAT_LDS) {
      for (int block : {256, 512, 1024})
        for (int g : {0, cus / 2, cus, 2 * cus, 4 * cus}) {
          PlanHints h;
          h.force_strategy = bk::STRAT_LDS;
          h.block = block;
          h.grid = g;
          cands.push_back(h);
        }
    } else if (p.cfg.strategy == bk::STRAT_PART) {
      const int smax = p.part.lay.tile_shift;
      for (int sh : {smax, smax - 1})
        for (int nt : {512, 1024})
          for (int ppt : {4, 8, 16})
            for (int wg : {cus, 2 * cus, 4 * cus}) {
              if (sh < 6) continue;
              PlanHints h;
              h.force_strategy = bk::STRAT_PART;
              h.tile_shift = sh;
              h.scatter_threads = nt;
              h.scatter_ppt = ppt;
              h.part_wg = wg;
              cands.push_back(h);
            }
    }
    float best = 1e30f;
    PlanHints best_h = base;
    for (const PlanHints& h : cands) {
      float ms = 0.f;
      const int cst = time_config(r, h, s, e0, e1, &ms);
      if (cst == BIN_ERR_UNSUPPORTED) continue;  // configuration does not fit
      if (cst) {
        st = cst;
        break;
      }
      if (ms < best) {
        best = ms;
        best_h = h;
      }
    }
    if (st == BIN_OK) {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      load_locked();
      g_tune[class_key(r)] = best_h;
    }
  }
  (void)hipStreamSynchronize(s);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  if (st == BIN_OK) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    save_locked();
  }
  return st;
}

}  // namespace binimpl

extern "C" int bin_autotune(const bin_request* reqs, int32_t count) {
  binimpl::clear_error();
  return binimpl::autotune(reqs, count);
}
