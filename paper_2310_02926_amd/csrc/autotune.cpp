// Autotuner: times candidate launch configurations - including the
// strategy itself (whole grid in LDS or tile partition) where both apply -
// for representative requests and remembers the
// fastest per (device, shape class).  The planner looks the class up
// whenever the caller set no explicit override.
//
// Shape class: log2 buckets of n and of the bin count, attribute count,
// coordinate and attribute types and the op mask (precision flags included).
// A batch (bin_particles_batched, graphs, the server) plans its requests
// under a policy that the autotuner also chooses, by timing the whole set
// of requests it was given as one batch: each request's tuned plan, the
// planner's rules, or the rules with one shared scatter shape.
//
// The tables live in memory and, when the environment variable
// BIN_TUNE_CACHE names a file, are loaded from and saved to that file as
// JSON:
//   {"version": 1, "entries": {"<device>|<class>": {"strategy": s, "block": b,
//    "grid": g, "part_wg": w, "scatter_ppt": p, "scatter_threads": t,
//    "tile_shift": h, "split_len": l, "quads": q}, ...},
//    "batch": {"<device>": {"strategy": policy, "scatter_ppt": p,
//    "scatter_threads": t, ...}}}
// where <device> is the device's architecture name and compute-unit count,
// so one file can hold the tunings of several kinds of GPU.
#include <algorithm>
#include <cctype>
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
// batch policy per device: force_strategy holds BatchPolicy::mode,
// scatter_threads and scatter_ppt its shared scatter shape
std::map<std::string, PlanHints> g_batch;
bool g_tune_loaded = false;
thread_local int t_lookup_off = 0;

int log2_bucket(int64_t v) {
  int b = 0;
  while (v > 1) {
    v >>= 1;
    ++b;
  }
  return b;
}

std::string device_key(const DeviceInfo& dev) { return dev.arch[0] ? dev.arch : "unknown"; }

std::string class_key(const bin_request& r, const DeviceInfo& dev) {
  const int k = r.attrs.cols ? r.attrs.ncols : 0;
  char buf[192];
  snprintf(buf, sizeof buf, "%s|n%d_b%d_k%d_c%d_a%d_o%u", dev.arch[0] ? dev.arch : "unknown", log2_bucket(r.n),
           log2_bucket((int64_t)r.nx * r.ny), k, r.coords.dtype, k ? r.attrs.dtype : 0, r.ops);
  return buf;
}

const char* cache_path() { return getenv("BIN_TUNE_CACHE"); }

// The fields of a tuning entry, in file order.
struct Field {
  const char* name;
  int64_t PlanHints::*i64;
  int PlanHints::*i32;
};
const Field kFields[] = {{"strategy", nullptr, &PlanHints::force_strategy},
                         {"block", nullptr, &PlanHints::block},
                         {"grid", nullptr, &PlanHints::grid},
                         {"part_wg", nullptr, &PlanHints::part_wg},
                         {"scatter_ppt", nullptr, &PlanHints::scatter_ppt},
                         {"scatter_threads", nullptr, &PlanHints::scatter_threads},
                         {"tile_shift", nullptr, &PlanHints::tile_shift},
                         {"split_len", &PlanHints::split_len, nullptr},
                         {"quads", nullptr, &PlanHints::quads}};

// A small reader for the cache's own JSON layout: string keys, objects and
// integers only.  Anything else makes the file count as empty.
struct JsonIn {
  const std::string& t;
  size_t i = 0;
  void ws() {
    while (i < t.size() && std::isspace((unsigned char)t[i])) ++i;
  }
  bool eat(char c) {
    ws();
    if (i < t.size() && t[i] == c) {
      ++i;
      return true;
    }
    return false;
  }
  bool str(std::string& out) {
    if (!eat('"')) return false;
    out.clear();
    while (i < t.size() && t[i] != '"') {
      if (t[i] == '\\') return false;  // the writer never escapes
      out += t[i++];
    }
    return i++ < t.size();
  }
  bool num(long long& v) {
    ws();
    const char* b = t.c_str() + i;
    char* e = nullptr;
    v = std::strtoll(b, &e, 10);
    if (e == b) return false;
    i += (size_t)(e - b);
    return true;
  }
  bool entry(PlanHints& h) {
    if (!eat('{')) return false;
    if (eat('}')) return true;
    do {
      std::string name;
      long long v = 0;
      if (!str(name) || !eat(':') || !num(v)) return false;
      for (const Field& f : kFields)
        if (name == f.name) {
          if (f.i64) h.*(f.i64) = v;
          else h.*(f.i32) = (int)v;
        }
    } while (eat(','));
    return eat('}');
  }
  bool table(std::map<std::string, PlanHints>& out) {
    if (!eat('{')) return false;
    if (eat('}')) return true;
    do {
      std::string key;
      PlanHints h;
      if (!str(key) || !eat(':') || !entry(h)) return false;
      out[key] = h;
    } while (eat(','));
    return eat('}');
  }
  bool file(std::map<std::string, PlanHints>& out, std::map<std::string, PlanHints>& batch) {
    if (!eat('{')) return false;
    do {
      std::string name;
      if (!str(name) || !eat(':')) return false;
      if (name == "entries") {
        if (!table(out)) return false;
      } else if (name == "batch") {
        if (!table(batch)) return false;
      } else {
        long long v;
        if (!num(v)) return false;
      }
    } while (eat(','));
    return eat('}');
  }
};

void load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* p = cache_path();
  if (!p) return;
  std::ifstream f(p);
  if (!f) return;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string text = ss.str();
  std::map<std::string, PlanHints> m, b;
  JsonIn in{text};
  if (in.file(m, b)) {
    for (auto& kv : m) g_tune[kv.first] = kv.second;
    for (auto& kv : b) g_batch[kv.first] = kv.second;
  }
}

void write_table(std::ofstream& f, const std::map<std::string, PlanHints>& t) {
  f << '{';
  bool first = true;
  for (auto& kv : t) {
    f << (first ? "\n  " : ",\n  ") << '"' << kv.first << "\": {";
    first = false;
    const PlanHints& h = kv.second;
    for (size_t j = 0; j < sizeof kFields / sizeof kFields[0]; ++j) {
      const Field& fd = kFields[j];
      f << (j ? ", " : "") << '"' << fd.name << "\": " << (fd.i64 ? (long long)(h.*(fd.i64)) : (long long)(h.*(fd.i32)));
    }
    f << '}';
  }
  f << "\n}";
}

void save_locked() {
  const char* p = cache_path();
  if (!p) return;
  std::ofstream f(p, std::ios::trunc);
  f << "{\"version\": 1, \"entries\": ";
  write_table(f, g_tune);
  f << ", \"batch\": ";
  write_table(f, g_batch);
  f << "}\n";
}

bool is_default(const PlanHints& h) {
  return h.force_strategy < 0 && !h.block && !h.grid && !h.part_wg && !h.scatter_ppt && !h.scatter_threads &&
         !h.tile_shift && !h.split_len && !h.quads && h.share <= 1;
}

}  // namespace

bool hints_are_default(const PlanHints& h) { return is_default(h); }

TunedLookupOff::TunedLookupOff() { ++t_lookup_off; }
TunedLookupOff::~TunedLookupOff() { --t_lookup_off; }

BatchPolicy batch_policy(const DeviceInfo& dev) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_locked();
  BatchPolicy p;
  auto it = g_batch.find(device_key(dev));
  if (it != g_batch.end()) {
    p.mode = it->second.force_strategy;
    p.nt = it->second.scatter_threads;
    p.ppt = it->second.scatter_ppt;
  }
  return p;
}

// Hints for a request: the caller's explicit override if any, else the
// tuned entry of its shape class, else defaults.
PlanHints effective_hints(const bin_request& r, const DeviceInfo& dev, const PlanHints& explicit_hints) {
  if (!is_default(explicit_hints) || t_lookup_off) return explicit_hints;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  load_locked();
  if (g_tune.empty()) return explicit_hints;
  auto it = g_tune.find(class_key(r, dev));
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
    // The strategy is a candidate like any other setting: a grid that fits
    // LDS whole is also timed as a tile partition (the reverse is not
    // possible).  The global-atomic strategy is left to the planner's rule
    // (grids beyond the tile limit): batches and graphs take the other two.
    std::vector<PlanHints> cands;
    PlanHints base;
    cands.push_back(base);
    const int64_t nb = (int64_t)r.nx * r.ny;
    if (p.cfg.strategy == bk::STRAT_LDS) {
      for (int block : {256, 512, 1024})
        for (int g : {0, cus / 2, cus, 2 * cus, 4 * cus}) {
          PlanHints h;
          h.force_strategy = bk::STRAT_LDS;
          h.block = block;
          h.grid = g;
          cands.push_back(h);
        }
    }
    // tile sizes up to the largest that fits LDS (the plan's own choice for
    // a partition request, else the smallest power of two holding the grid)
    int smax = 6;
    if (p.cfg.strategy == bk::STRAT_PART) smax = p.part.lay.tile_shift;
    else
      while (smax < 15 && ((int64_t)1 << smax) < nb) ++smax;
    for (int sh : {smax, smax - 1, smax - 2})
      for (int nt : {512, 1024})
        for (int ppt : {4, 8, 16})
          for (int wg : {cus, 2 * cus, 4 * cus})
            for (int q : {0, 1, 2}) {
              if (sh < 6 || (int64_t)1 << sh > 2 * nb) continue;
              if (q && (ppt != 16 || nt != 1024 || wg != 2 * cus)) continue;  // quads: one shape
              PlanHints h;
              h.force_strategy = bk::STRAT_PART;
              h.tile_shift = sh;
              h.scatter_threads = nt;
              h.scatter_ppt = ppt;
              h.part_wg = wg;
              h.quads = q;
              cands.push_back(h);
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
      g_tune[class_key(r, dev)] = best_h;
    }
  }
  // The batch policy: the whole set as one batch (bin_particles_batched,
  // graphs and the server plan this way) under each policy; per-request
  // plans tuned alone can split a batch into more, smaller launch groups.
  if (st == BIN_OK && count >= 2) {
    std::vector<PlanHints> pols;
    for (int mode : {1, 0}) {
      PlanHints h;
      h.force_strategy = mode;
      pols.push_back(h);
    }
    for (auto shape : {std::make_pair(1024, 8), std::make_pair(1024, 4), std::make_pair(512, 8)}) {
      PlanHints h;
      h.force_strategy = 2;
      h.scatter_threads = shape.first;
      h.scatter_ppt = shape.second;
      pols.push_back(h);
    }
    const std::string dk = device_key(dev);
    float best = 1e30f;
    PlanHints best_p = pols[0];
    for (const PlanHints& pol : pols) {
      {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_batch[dk] = pol;
      }
      float t[3];
      int bst = run_batch(reqs, count, s, PlanHints{});  // warm-up
      for (int i = 0; i < 3 && bst == BIN_OK; ++i) {
        hipError_t e = hipEventRecord(e0, s);
        if (e == hipSuccess) bst = run_batch(reqs, count, s, PlanHints{});
        if (bst) break;
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&t[i], e0, e1);
        if (e != hipSuccess) bst = hip_fail(e, "autotune batch timing");
      }
      if (bst == BIN_ERR_UNSUPPORTED) continue;
      if (bst) {
        st = bst;
        break;
      }
      std::sort(t, t + 3);
      if (t[1] < best) {
        best = t[1];
        best_p = pol;
      }
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_batch[dk] = best_p;
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
