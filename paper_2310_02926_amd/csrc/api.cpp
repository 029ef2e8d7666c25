// C ABI of libbinning.so: argument validation, planning, scratch pools and
// the launch sequence init -> bin -> finalize for one request.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/binning.h"
#include "internal.h"
#include "kernels.h"

namespace binimpl {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

int fail(int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? BIN_ERR_OOM : BIN_ERR_DEVICE, "%s: %s", what,
              hipGetErrorString(e));
}

void clear_error() { g_last_error.clear(); }
const char* last_error() { return g_last_error.c_str(); }

// ---------------------------------------------------------------------------
// Validation: pure host logic, no HIP call.
// ---------------------------------------------------------------------------
static bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

static int check_axis(const char* name, double lo, double hi, int32_t n) {
  if (!std::isfinite(lo) || !std::isfinite(hi))
    return fail(BIN_ERR_INVALID_ARG, "%s bounds must be finite (got %g, %g)", name, lo, hi);
  if (!(lo < hi)) return fail(BIN_ERR_INVALID_ARG, "%s bounds need lo < hi (got %g, %g)", name, lo, hi);
  const double w = hi - lo;
  if (!std::isfinite(w)) return fail(BIN_ERR_INVALID_ARG, "%s extent hi - lo overflows", name);
  const double s = (double)n / w;
  if (!std::isfinite(s) || !(s > 0.0))
    return fail(BIN_ERR_INVALID_ARG, "%s scale n / (hi - lo) is not a finite positive number", name);
  return BIN_OK;
}

int validate(const bin_columns* coords, const bin_columns* attrs, int64_t n, const int32_t axes[2],
             const double bounds[4], int32_t nx, int32_t ny, uint32_t ops, const bin_output* out,
             bool allow_null_bounds) {
  if (!coords || !coords->cols) return fail(BIN_ERR_INVALID_ARG, "coords table is NULL");
  if (coords->ncols < 1 || coords->ncols > BIN_MAX_COLUMNS)
    return fail(BIN_ERR_INVALID_ARG, "coords->ncols = %d outside [1, %d]", coords->ncols, BIN_MAX_COLUMNS);
  if (coords->dtype != BIN_F32 && coords->dtype != BIN_F64)
    return fail(BIN_ERR_INVALID_ARG, "coords->dtype = %d is not BIN_F32/BIN_F64", coords->dtype);
  if (!axes) return fail(BIN_ERR_INVALID_ARG, "axes is NULL");
  for (int i = 0; i < 2; ++i)
    if (axes[i] < 0 || axes[i] >= coords->ncols)
      return fail(BIN_ERR_INVALID_ARG, "axes[%d] = %d outside [0, %d)", i, axes[i], coords->ncols);
  const int k = attrs ? attrs->ncols : 0;
  if (attrs) {
    if (k < 0 || k > BIN_MAX_ATTRS)
      return fail(BIN_ERR_INVALID_ARG, "attrs->ncols = %d outside [0, %d]", k, BIN_MAX_ATTRS);
    if (k > 0 && !attrs->cols) return fail(BIN_ERR_INVALID_ARG, "attrs->cols is NULL");
    if (attrs->dtype != BIN_F32 && attrs->dtype != BIN_F64)
      return fail(BIN_ERR_INVALID_ARG, "attrs->dtype = %d is not BIN_F32/BIN_F64", attrs->dtype);
  }
  if (n < 0 || (uint64_t)n > 0xFFFFFFFFull)
    return fail(BIN_ERR_INVALID_ARG, "n = %lld outside [0, UINT32_MAX]", (long long)n);
  if (nx < 1 || ny < 1) return fail(BIN_ERR_INVALID_ARG, "nx, ny must be >= 1 (got %d, %d)", nx, ny);
  if ((int64_t)nx * (int64_t)ny > 0x7FFFFFFFll)
    return fail(BIN_ERR_INVALID_ARG, "nx * ny = %lld exceeds 2^31 - 1", (long long)nx * ny);
  const uint32_t opbits = ops & BIN_OPS_ALL;
  if (ops & ~(BIN_OPS_ALL | BIN_PREC_PLAIN | BIN_PREC_F64 | BIN_PREC_COMP))
    return fail(BIN_ERR_INVALID_ARG, "ops = 0x%x has unknown bits", ops);
  if (!opbits) return fail(BIN_ERR_INVALID_ARG, "ops requests no reduction");
  const uint32_t pf = ops & (BIN_PREC_PLAIN | BIN_PREC_F64 | BIN_PREC_COMP);
  if (pf & (pf - 1)) return fail(BIN_ERR_INVALID_ARG, "the BIN_PREC_* flags are mutually exclusive");
  if ((opbits & (BIN_SUM | BIN_MIN | BIN_MAX | BIN_AVG)) && k == 0)
    return fail(BIN_ERR_INVALID_ARG, "sum/min/max/avg requested with no attribute columns");
  if (bounds) {
    int s = check_axis("x", bounds[0], bounds[1], nx);
    if (s) return s;
    s = check_axis("y", bounds[2], bounds[3], ny);
    if (s) return s;
  } else if (!allow_null_bounds) {
    return fail(BIN_ERR_INVALID_ARG, "bounds is NULL");
  }
  const size_t csz = coords->dtype == BIN_F64 ? 8 : 4;
  if (n > 0) {
    for (int i = 0; i < 2; ++i) {
      const void* p = coords->cols[axes[i]];
      if (!p) return fail(BIN_ERR_INVALID_ARG, "coordinate column %d is NULL", axes[i]);
      if (!aligned(p, csz)) return fail(BIN_ERR_INVALID_ARG, "coordinate column %d is misaligned", axes[i]);
    }
    const size_t asz = (attrs && attrs->dtype == BIN_F64) ? 8 : 4;
    for (int j = 0; j < k; ++j) {
      if (!attrs->cols[j]) return fail(BIN_ERR_INVALID_ARG, "attribute column %d is NULL", j);
      if (!aligned(attrs->cols[j], asz)) return fail(BIN_ERR_INVALID_ARG, "attribute column %d is misaligned", j);
    }
  }
  if (!out) return fail(BIN_ERR_INVALID_ARG, "out is NULL");
  if ((opbits & BIN_COUNT) && !out->count) return fail(BIN_ERR_INVALID_ARG, "out->count is NULL but BIN_COUNT is set");
  if (out->count && !aligned(out->count, 4)) return fail(BIN_ERR_INVALID_ARG, "out->count is misaligned");
  const bool af64 = attrs && attrs->dtype == BIN_F64;
  const size_t mm_sz = af64 ? 8 : 4;
  const size_t sum_sz = (!af64 && (ops & BIN_PREC_PLAIN)) ? 4 : 8;
  struct {
    uint32_t bit;
    void* const* arr;
    const char* name;
    size_t sz;
  } req[4] = {{BIN_SUM, out->sum, "sum", sum_sz},
              {BIN_MIN, out->min, "min", mm_sz},
              {BIN_MAX, out->max, "max", mm_sz},
              {BIN_AVG, out->avg, "avg", sum_sz}};
  for (auto& r : req) {
    if (!(opbits & r.bit)) continue;
    if (!r.arr) return fail(BIN_ERR_INVALID_ARG, "out->%s is NULL but the op is requested", r.name);
    for (int j = 0; j < k; ++j) {
      if (!r.arr[j]) return fail(BIN_ERR_INVALID_ARG, "out->%s[%d] is NULL", r.name, j);
      if (!aligned(r.arr[j], r.sz)) return fail(BIN_ERR_INVALID_ARG, "out->%s[%d] is misaligned", r.name, j);
    }
  }
  return BIN_OK;
}

// Meshes of one to three axes: the checks of the two-axis request the call
// maps to, then those of the axes that mapping does not show.
int validate_nd(const bin_columns* coords, const bin_columns* attrs, int64_t n, int32_t ndim,
                const int32_t* axes, const double* bounds, const int32_t* dims, uint32_t ops,
                const bin_output* out) {
  if (ndim < 1 || ndim > 3) return fail(BIN_ERR_INVALID_ARG, "ndim = %d outside [1, 3]", ndim);
  if (!axes) return fail(BIN_ERR_INVALID_ARG, "axes is NULL");
  if (!dims) return fail(BIN_ERR_INVALID_ARG, "dims is NULL");
  int64_t nb = 1;
  for (int d = 0; d < ndim; ++d) {
    if (dims[d] < 1) return fail(BIN_ERR_INVALID_ARG, "dims[%d] = %d must be >= 1", d, dims[d]);
    nb *= dims[d];
    if (nb > 0x7FFFFFFFll) return fail(BIN_ERR_INVALID_ARG, "the product of dims exceeds 2^31 - 1");
  }
  const int32_t a2[2] = {axes[0], ndim > 1 ? axes[1] : axes[0]};
  const int32_t nx = dims[0], ny = ndim == 1 ? 1 : (ndim == 2 ? dims[1] : dims[1] * dims[2]);
  int st = validate(coords, attrs, n, a2, nullptr, nx, ny, ops, out, true);
  if (st) return st;
  if (ndim == 3) {
    if (axes[2] < 0 || axes[2] >= coords->ncols)
      return fail(BIN_ERR_INVALID_ARG, "axes[2] = %d outside [0, %d)", axes[2], coords->ncols);
    const size_t csz = coords->dtype == BIN_F64 ? 8 : 4;
    if (n > 0) {
      const void* p = coords->cols[axes[2]];
      if (!p) return fail(BIN_ERR_INVALID_ARG, "coordinate column %d is NULL", axes[2]);
      if (!aligned(p, csz)) return fail(BIN_ERR_INVALID_ARG, "coordinate column %d is misaligned", axes[2]);
    }
    if (coords->dtype == BIN_F32 && (int64_t)dims[1] * dims[2] > (1ll << 24))
      return fail(BIN_ERR_INVALID_ARG, "f32 coordinates need dims[1] * dims[2] <= 2^24 (got %lld)",
                  (long long)dims[1] * dims[2]);
  }
  if (bounds) {
    static const char* const names[3] = {"axis 0", "axis 1", "axis 2"};
    for (int d = 0; d < ndim; ++d) {
      st = check_axis(names[d], bounds[2 * d], bounds[2 * d + 1], dims[d]);
      if (st) return st;
    }
  }
  return BIN_OK;
}

// ---------------------------------------------------------------------------
// Device facts, queried once per device.
// ---------------------------------------------------------------------------
static std::mutex g_dev_mu;
static std::unordered_map<int, DeviceInfo> g_devs;

int device_info(DeviceInfo* info) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_dev_mu);
  auto it = g_devs.find(dev);
  if (it != g_devs.end()) {
    *info = it->second;
    return BIN_OK;
  }
  hipDeviceProp_t p;
  e = hipGetDeviceProperties(&p, dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  DeviceInfo d;
  d.device = dev;
  d.cus = p.multiProcessorCount;
  d.lds_per_block = p.sharedMemPerBlock;
  d.lds_per_cu = p.maxSharedMemoryPerMultiProcessor ? p.maxSharedMemoryPerMultiProcessor : p.sharedMemPerBlock;
  {
    std::string arch = p.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);  // drop feature flags
    snprintf(d.arch, sizeof d.arch, "%s:%d", arch.c_str(), d.cus);
  }
  // Dynamic LDS beyond the default needs an explicit opt-in per kernel.
  e = bk::set_lds_limit(d.lds_per_block);
  if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute(max dynamic LDS)");
  g_devs[dev] = d;
  *info = d;
  return BIN_OK;
}

// ---------------------------------------------------------------------------
// Scratch pool: one growing device buffer per (device, stream), reused by
// stream order.  Grown with stream-ordered allocation so that earlier work on
// the stream can still use the old buffer while it is released.
// ---------------------------------------------------------------------------
struct Pool {
  void* ptr = nullptr;
  size_t bytes = 0;
};
static std::mutex g_pool_mu;
static std::unordered_map<std::string, Pool> g_pools;

static std::string pool_key(int dev, hipStream_t s) {
  char b[64];
  snprintf(b, sizeof b, "%d:%p", dev, (void*)s);
  return b;
}

int scratch_get(int dev, hipStream_t s, size_t bytes, void** out) {
  *out = nullptr;
  if (bytes == 0) return BIN_OK;
  bytes = (bytes + 255) & ~size_t(255);
  std::lock_guard<std::mutex> lk(g_pool_mu);
  Pool& p = g_pools[pool_key(dev, s)];
  if (p.bytes < bytes) {
    if (p.ptr) {
      hipError_t e = hipFreeAsync(p.ptr, s);
      if (e != hipSuccess) return hip_fail(e, "hipFreeAsync(scratch)");
      p.ptr = nullptr;
      p.bytes = 0;
    }
    size_t want = std::max(bytes, size_t(1) << 20);
    if (fault_injection_hit()) return fail(BIN_ERR_OOM, "injected scratch allocation failure");
    hipError_t e = hipMallocAsync(&p.ptr, want, s);
    if (e != hipSuccess) {
      p.ptr = nullptr;
      return hip_fail(e, "hipMallocAsync(scratch)");
    }
    p.bytes = want;
  }
  *out = p.ptr;
  return BIN_OK;
}

int scratch_release(int dev, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_pool_mu);
  auto it = g_pools.find(pool_key(dev, s));
  if (it == g_pools.end() || !it->second.ptr) return BIN_OK;
  const hipError_t e = hipFreeAsync(it->second.ptr, s);  // after the stream's work that used it
  g_pools.erase(it);
  return e == hipSuccess ? BIN_OK : hip_fail(e, "hipFreeAsync(scratch)");
}

int release_all_scratch() {
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  std::lock_guard<std::mutex> lk(g_pool_mu);
  for (auto& kv : g_pools)
    if (kv.second.ptr) (void)hipFree(kv.second.ptr);
  g_pools.clear();
  return BIN_OK;
}

// Test hook: BIN_FAIL_ALLOC_AT=N makes the N-th scratch allocation of the
// process fail with BIN_ERR_OOM (N counted from 1).
bool fault_injection_hit() {
  static std::atomic<long> counter{0};
  static long target = [] {
    const char* s = getenv("BIN_FAIL_ALLOC_AT");
    return s ? atol(s) : 0L;
  }();
  if (target <= 0) return false;
  return ++counter == target;
}

// ---------------------------------------------------------------------------
// Kernel timing (bin_timing_*).
// ---------------------------------------------------------------------------
// While enabled, every launch of the library is bracketed by an event pair
// on its stream; the pairs are resolved into per-kernel totals on read.
struct Pending {
  std::string name;
  hipEvent_t a, b;
};
static std::mutex g_tm_mu;
static bool g_tm_on = false;
static std::vector<Pending> g_tm_pending;
static std::map<std::string, std::pair<int64_t, double>> g_tm_totals;

namespace {
class EventTimer : public bk::KTimer {
 public:
  void begin(hipStream_t s) override {
    a_ = b_ = nullptr;
    if (hipEventCreate(&a_) != hipSuccess || hipEventCreate(&b_) != hipSuccess || hipEventRecord(a_, s) != hipSuccess)
      a_ = nullptr;
  }
  void end(const char* name, hipStream_t s) override {
    if (!a_ || hipEventRecord(b_, s) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_tm_mu);
    g_tm_pending.push_back(Pending{name, a_, b_});
    a_ = b_ = nullptr;
  }

 private:
  hipEvent_t a_ = nullptr, b_ = nullptr;
};
thread_local EventTimer t_timer;

// Resolve pending event pairs (waits for them) into the totals.
int resolve_pending() {
  std::vector<Pending> ev;
  {
    std::lock_guard<std::mutex> lk(g_tm_mu);
    ev.swap(g_tm_pending);
  }
  int status = BIN_OK;
  for (auto& p : ev) {
    hipError_t e = hipEventSynchronize(p.b);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.a, p.b);
    if (e != hipSuccess && status == BIN_OK) status = hip_fail(e, "hipEventElapsedTime");
    {
      std::lock_guard<std::mutex> lk(g_tm_mu);
      auto& t = g_tm_totals[p.name];
      t.first += 1;
      t.second += ms;
    }
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  return status;
}
}  // namespace

bk::KTimer* timing_timer() {
  std::lock_guard<std::mutex> lk(g_tm_mu);
  return g_tm_on ? &t_timer : nullptr;
}

int timing_enable(int on) {
  if (on) {
    int st = resolve_pending();
    std::lock_guard<std::mutex> lk(g_tm_mu);
    g_tm_totals.clear();
    g_tm_on = true;
    return st;
  }
  std::lock_guard<std::mutex> lk(g_tm_mu);
  g_tm_on = false;
  return BIN_OK;
}

int timing_read(int64_t* launches, double* total_ms) {
  int st = resolve_pending();
  std::lock_guard<std::mutex> lk(g_tm_mu);
  int64_t n = 0;
  double best = -1.0;
  for (auto& kv : g_tm_totals)
    if (kv.second.second > best) {
      best = kv.second.second;
      n = kv.second.first;
    }
  if (launches) *launches = n;
  if (total_ms) *total_ms = best < 0 ? 0.0 : best;
  return st;
}

int timing_report(char* buf, size_t buflen) {
  int st = resolve_pending();
  std::string out = "{";
  {
    std::lock_guard<std::mutex> lk(g_tm_mu);
    bool first = true;
    for (auto& kv : g_tm_totals) {
      char item[256];
      snprintf(item, sizeof item, "%s\"%s\": [%lld, %.6f]", first ? "" : ", ", kv.first.c_str(),
               (long long)kv.second.first, kv.second.second);
      out += item;
      first = false;
    }
  }
  out += "}";
  if (buf && buflen) {
    std::strncpy(buf, out.c_str(), buflen - 1);
    buf[buflen - 1] = 0;
    if (out.size() >= buflen) return fail(BIN_ERR_INVALID_ARG, "timing report needs %zu bytes", out.size() + 1);
  }
  return st;
}

}  // namespace binimpl
