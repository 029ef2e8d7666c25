// extern "C" entry points of libbinning.so (declared in include/binning.h).
#include <cstring>

#include "internal.h"

using namespace binimpl;

namespace binimpl {

bin_request make_request(const bin_columns* coords, const bin_columns* attrs, int64_t n,
                         const int32_t axes[2], const double bounds[4], int32_t nx, int32_t ny,
                         uint32_t ops, const bin_output* out) {
  bin_request r;
  std::memset(&r, 0, sizeof r);
  r.coords = *coords;
  if (attrs) r.attrs = *attrs;
  r.n = n;
  r.axes[0] = axes[0];
  r.axes[1] = axes[1];
  if (bounds) std::memcpy(r.bounds, bounds, sizeof r.bounds);
  r.nx = nx;
  r.ny = ny;
  r.ops = ops;
  r.out = *out;
  return r;
}

}  // namespace binimpl

namespace {

// A stream that already holds a fault makes every later call on it fail.
int precheck_stream(hipStream_t s) {
  hipError_t e = hipStreamQuery(s);
  if (e == hipSuccess || e == hipErrorNotReady) return BIN_OK;
  return hip_fail(e, "stream holds an earlier device error");
}

}  // namespace

namespace binimpl {
static thread_local PlanHints t_hints;
const PlanHints& thread_hints() { return t_hints; }
PlanHints& thread_hints_mut() { return t_hints; }

// Scratch of 'bytes' for a request on stream s: from the caller's fixed
// block (no allocation; a request that needs more is refused), else from
// the library's pool for (device, stream).
static int take_scratch(int device, hipStream_t s, size_t bytes, const FixedScratch* fixed, void** out) {
  if (!fixed) return scratch_get(device, s, bytes, out);
  if (bytes > fixed->cap)
    return fail(BIN_ERR_INVALID_ARG,
                "the request needs %zu bytes of scratch on this device, more than the %zu bytes the "
                "allocation-free entry point holds; use bin_particles",
                bytes, fixed->cap);
  *out = bytes ? fixed->ptr : nullptr;
  return BIN_OK;
}

int run_request_in(const bin_request& r, hipStream_t s, const PlanHints& hints, const FixedScratch* fixed,
                   bk::KTimer* tm) {
  DeviceInfo dev;
  int st = device_info(&dev);
  if (st) return st;
  st = precheck_stream(s);
  if (st) return st;
  Prepared p;
  st = prepare(r, dev, hints, nullptr, &p);  // sizing pass
  if (st) return st;
  void* scratch = nullptr;
  if (p.scratch_bytes) {
    st = take_scratch(dev.device, s, p.scratch_bytes, fixed, &scratch);
    if (st) return st;
    st = prepare(r, dev, hints, scratch, &p);
    if (st) return st;
  }
  return enqueue(p, s, tm);
}

// Single request on a stream (also used by the autotuner).
int run_request(const bin_request& r, hipStream_t s, const PlanHints& hints) {
  return run_request_in(r, s, hints, nullptr, timing_timer());
}

// Bounds from the data (bounds == NULL): a min/max pass over the two axis
// columns writes four keys at the start of the scratch block; the binning
// kernels read them instead of host bounds.  The plan itself does not
// depend on the bounds, so it is made with a placeholder.
int run_auto_bounds_in(const bin_request& r0, hipStream_t s, const FixedScratch* fixed, bk::KTimer* tm) {
  bin_request r = r0;
  r.bounds[0] = 0.0;
  r.bounds[1] = 1.0;
  r.bounds[2] = 0.0;
  r.bounds[3] = 1.0;
  DeviceInfo dev;
  int st = device_info(&dev);
  if (st) return st;
  st = precheck_stream(s);
  if (st) return st;
  const PlanHints& hints = thread_hints();
  Prepared p;
  st = prepare(r, dev, hints, nullptr, &p);
  if (st) return st;
  void* scratch = nullptr;
  st = take_scratch(dev.device, s, p.scratch_bytes + 256, fixed, &scratch);
  if (st) return st;
  st = prepare(r, dev, hints, static_cast<unsigned char*>(scratch) + 256, &p);
  if (st) return st;
  long long* keys = static_cast<long long*>(scratch);
  p.bin.dyn = keys;
  p.lds.dyn = keys;
  p.part.dyn = keys;
  hipError_t e = bk::launch_bounds(r.coords.cols[r.axes[0]], r.coords.cols[r.axes[1]], p.coord_f64, r.n, keys,
                                   dev.cus, s, tm);
  if (e != hipSuccess) return hip_fail(e, "launch bounds kernels");
  return enqueue(p, s, tm);
}

int run_auto_bounds(const bin_request& r, hipStream_t s) { return run_auto_bounds_in(r, s, nullptr, timing_timer()); }

// Three axes: fold axes 1 and 2 into a composite column in scratch (one
// pass), then bin (axis 0, composite) on a dims[0] x dims[1] * dims[2] mesh
// whose second axis is [0, dims[1] * dims[2]].  Scratch: 256 bytes of
// bounds keys (0-5: the three axes from the data, 8-11: the folded mesh),
// the composite column, then the plan's own scratch.
int run_fold3(const bin_columns* coords, const bin_columns* attrs, int64_t n, const int32_t* axes,
              const double* bounds, const int32_t* dims, uint32_t ops, const bin_output* out, hipStream_t s) {
  const bool f64 = coords->dtype == BIN_F64;
  const size_t csz = f64 ? 8 : 4;
  const int32_t nyz = dims[1] * dims[2];
  const void* cols2[2] = {coords->cols[axes[0]], nullptr};
  const bin_columns c2{cols2, 2, coords->dtype};
  const int32_t ax2[2] = {0, 1};
  const double b4[4] = {bounds ? bounds[0] : 0.0, bounds ? bounds[1] : 1.0, 0.0, (double)nyz};
  bin_request r = make_request(&c2, attrs, n, ax2, b4, dims[0], nyz, ops, out);
  DeviceInfo dev;
  int st = device_info(&dev);
  if (st) return st;
  st = precheck_stream(s);
  if (st) return st;
  const PlanHints& hints = thread_hints();
  Prepared p;
  st = prepare(r, dev, hints, nullptr, &p);
  if (st) return st;
  const size_t comp_bytes = ((size_t)n * csz + 255) & ~size_t(255);
  void* scratch = nullptr;
  st = scratch_get(dev.device, s, 256 + comp_bytes + p.scratch_bytes, &scratch);
  if (st) return st;
  unsigned char* base = static_cast<unsigned char*>(scratch);
  long long* keys = reinterpret_cast<long long*>(base);
  cols2[1] = base + 256;  // r.coords.cols points at cols2
  st = prepare(r, dev, hints, base + 256 + comp_bytes, &p);
  if (st) return st;
  bk::FoldArgs fa;
  std::memset(&fa, 0, sizeof fa);
  fa.y = coords->cols[axes[1]];
  fa.z = coords->cols[axes[2]];
  fa.out = base + 256;
  fa.n = n;
  fa.vec = (reinterpret_cast<uintptr_t>(fa.y) % 16 == 0 && reinterpret_cast<uintptr_t>(fa.z) % 16 == 0) ? 1 : 0;
  if (bounds) {
    fa.ay = bk::Axis{bounds[2], bounds[3], (double)dims[1] / (bounds[3] - bounds[2]), dims[1], 0};
    fa.az = bk::Axis{bounds[4], bounds[5], (double)dims[2] / (bounds[5] - bounds[4]), dims[2], 0};
  } else {
    fa.ay = bk::Axis{0.0, 1.0, 0.0, dims[1], 0};
    fa.az = bk::Axis{0.0, 1.0, 0.0, dims[2], 0};
  }
  bk::KTimer* tm = timing_timer();
  if (!bounds) {
    hipError_t e = bk::launch_bounds(coords->cols[axes[0]], coords->cols[axes[1]], f64, n, keys, dev.cus, s, tm);
    if (e == hipSuccess)
      e = bk::launch_bounds(coords->cols[axes[2]], coords->cols[axes[2]], f64, n, keys + 4, dev.cus, s, tm);
    if (e != hipSuccess) return hip_fail(e, "launch bounds kernels");
    fa.dyn_in = keys;
    fa.dyn_out = keys + 8;
    p.bin.dyn = keys + 8;
    p.lds.dyn = keys + 8;
    p.part.dyn = keys + 8;
  }
  const hipError_t e = bk::launch_fold(fa, f64, dev.cus, s, tm);
  if (e != hipSuccess) return hip_fail(e, "launch fold kernel");
  return enqueue(p, s, tm);
}
}  // namespace binimpl

extern "C" {

int bin_validate(const bin_columns* coords, const bin_columns* attrs, int64_t n, const int32_t axes[2],
                 const double bounds[4], int32_t nx, int32_t ny, uint32_t ops, const bin_output* out) {
  clear_error();
  return validate(coords, attrs, n, axes, bounds, nx, ny, ops, out, true);
}

int bin_particles(const bin_columns* coords, const bin_columns* attrs, int64_t n, const int32_t axes[2],
                  const double bounds[4], int32_t nx, int32_t ny, uint32_t ops, const bin_output* out,
                  void* stream) {
  clear_error();
  int st = validate(coords, attrs, n, axes, bounds, nx, ny, ops, out, true);
  if (st) return st;
  bin_request r = make_request(coords, attrs, n, axes, bounds, nx, ny, ops, out);
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (!bounds) return run_auto_bounds(r, s);
  return run_request(r, s, thread_hints());
}

int bin_particles_async(const bin_columns* coords, const bin_columns* attrs, int64_t n, const int32_t axes[2],
                        const double bounds[4], int32_t nx, int32_t ny, uint32_t ops, const bin_output* out,
                        void* src_stream, void* bin_stream) {
  clear_error();
  int st = validate(coords, attrs, n, axes, bounds, nx, ny, ops, out, true);
  if (st) return st;
  hipStream_t ss = static_cast<hipStream_t>(src_stream);
  hipStream_t bs = static_cast<hipStream_t>(bin_stream);
  st = precheck_stream(ss);
  if (st) return st;
  st = precheck_stream(bs);
  if (st) return st;
  const int k = attrs ? attrs->ncols : 0;
  const size_t csz = coords->dtype == BIN_F64 ? 8 : 4;
  const size_t asz = (k && attrs->dtype == BIN_F64) ? 8 : 4;
  const size_t ccol = (size_t)n * csz, acol = (size_t)n * asz;
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t bytes = 2 * al(ccol) + (size_t)k * al(acol);
  if (bytes == 0) {  // nothing to copy: order the binning after src's work
    bin_request r = make_request(coords, attrs, n, axes, bounds, nx, ny, ops, out);
    hipEvent_t ev = nullptr;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, ss);
    if (e == hipSuccess) e = hipStreamWaitEvent(bs, ev, 0);
    if (ev) (void)hipEventDestroy(ev);
    if (e != hipSuccess) return hip_fail(e, "order binning after source stream");
    return bounds ? run_request(r, bs, thread_hints()) : run_auto_bounds(r, bs);
  }
  DeviceInfo dev;
  st = device_info(&dev);
  if (st) return st;
  const void* ccols[2];
  const void* acols[BIN_MAX_ATTRS];
  auto copy = [&](void* stage) -> int {
    unsigned char* p = static_cast<unsigned char*>(stage);
    size_t o = 0;
    for (int c = 0; c < 2; ++c, o += al(ccol)) {
      ccols[c] = p + o;
      const hipError_t e = hipMemcpyAsync(p + o, coords->cols[axes[c]], ccol, hipMemcpyDeviceToDevice, ss);
      if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(staging)");
    }
    for (int j = 0; j < k; ++j, o += al(acol)) {
      acols[j] = p + o;
      const hipError_t e = hipMemcpyAsync(p + o, attrs->cols[j], acol, hipMemcpyDeviceToDevice, ss);
      if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(staging)");
    }
    return BIN_OK;
  };
  auto bin = [&](void*) -> int {
    bin_columns sc{reinterpret_cast<const void* const*>(ccols), 2, coords->dtype};
    bin_columns sa{reinterpret_cast<const void* const*>(acols), k, k ? attrs->dtype : BIN_F32};
    const int32_t sax[2] = {0, 1};
    bin_request r = make_request(&sc, k ? &sa : nullptr, n, sax, bounds, nx, ny, ops, out);
    return bounds ? run_request(r, bs, thread_hints()) : run_auto_bounds(r, bs);
  };
  return stage_run(dev.device, ss, bs, bytes, copy, bin);
}

int bin_validate_nd(const bin_columns* coords, const bin_columns* attrs, int64_t n, int32_t ndim,
                    const int32_t* axes, const double* bounds, const int32_t* dims, uint32_t ops,
                    const bin_output* out) {
  clear_error();
  return validate_nd(coords, attrs, n, ndim, axes, bounds, dims, ops, out);
}

int bin_particles_nd(const bin_columns* coords, const bin_columns* attrs, int64_t n, int32_t ndim,
                     const int32_t* axes, const double* bounds, const int32_t* dims, uint32_t ops,
                     const bin_output* out, void* stream) {
  clear_error();
  int st = validate_nd(coords, attrs, n, ndim, axes, bounds, dims, ops, out);
  if (st) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (ndim == 3) return run_fold3(coords, attrs, n, axes, bounds, dims, ops, out, s);
  // One axis: the two-axis mesh dims[0] x 1 whose second axis is the first
  // one again; its inside test repeats the first one's and its index is 0.
  const int32_t a2[2] = {axes[0], ndim == 2 ? axes[1] : axes[0]};
  double b4[4];
  if (bounds) {
    b4[0] = bounds[0];
    b4[1] = bounds[1];
    b4[2] = ndim == 2 ? bounds[2] : bounds[0];
    b4[3] = ndim == 2 ? bounds[3] : bounds[1];
  }
  bin_request r = make_request(coords, attrs, n, a2, bounds ? b4 : nullptr, dims[0], ndim == 2 ? dims[1] : 1,
                               ops, out);
  return bounds ? run_request(r, s, thread_hints()) : run_auto_bounds(r, s);
}

int bin_set_plan_override(int32_t strategy, int32_t block, int32_t grid) {
  clear_error();
  if (strategy < -1 || strategy > 2) return fail(BIN_ERR_INVALID_ARG, "strategy must be -1, 0, 1 or 2");
  if (block != 0 && (block < 64 || block > 1024 || block % 64))
    return fail(BIN_ERR_INVALID_ARG, "block must be 0 or a multiple of 64 in [64, 1024]");
  if (grid < 0) return fail(BIN_ERR_INVALID_ARG, "grid must be >= 0");
  t_hints.force_strategy = strategy;
  t_hints.block = block;
  t_hints.grid = grid;
  return BIN_OK;
}

int bin_set_tuning(int32_t param, int64_t value) {
  clear_error();
  if (value < 0) return fail(BIN_ERR_INVALID_ARG, "tuning value must be >= 0");
  switch (param) {
    case BIN_TUNE_PART_WG:
      if (value > 65535) return fail(BIN_ERR_INVALID_ARG, "BIN_TUNE_PART_WG must be <= 65535");
      t_hints.part_wg = (int)value;
      return BIN_OK;
    case BIN_TUNE_SCATTER_PPT:
      if (value && value != 4 && value != 8 && value != 12 && value != 16 && value != 32)
        return fail(BIN_ERR_INVALID_ARG, "BIN_TUNE_SCATTER_PPT must be 4, 8, 12, 16 or 32");
      t_hints.scatter_ppt = (int)value;
      return BIN_OK;
    case BIN_TUNE_SCATTER_THREADS:
      if (value && value != 256 && value != 512 && value != 1024)
        return fail(BIN_ERR_INVALID_ARG, "BIN_TUNE_SCATTER_THREADS must be 256, 512 or 1024");
      t_hints.scatter_threads = (int)value;
      return BIN_OK;
    case BIN_TUNE_TILE_SHIFT:
      if (value && (value < 6 || value > 15)) return fail(BIN_ERR_INVALID_ARG, "BIN_TUNE_TILE_SHIFT must be in 6..15");
      t_hints.tile_shift = (int)value;
      return BIN_OK;
    case BIN_TUNE_SPLIT_LEN:
      if (value && (value < 1024 || value > 0x7FFFFFFF))
        return fail(BIN_ERR_INVALID_ARG, "BIN_TUNE_SPLIT_LEN must be in [1024, 2^31)");
      t_hints.split_len = value;
      return BIN_OK;
    case BIN_TUNE_QUADS:
      if (value > 2) return fail(BIN_ERR_INVALID_ARG, "BIN_TUNE_QUADS must be 0, 1 or 2");
      t_hints.quads = (int)value;
      return BIN_OK;
    default:
      return fail(BIN_ERR_INVALID_ARG, "unknown tuning parameter %d", param);
  }
}

const char* bin_status_string(int status) {
  switch (status) {
    case BIN_OK: return "BIN_OK";
    case BIN_ERR_INVALID_ARG: return "BIN_ERR_INVALID_ARG";
    case BIN_ERR_UNSUPPORTED: return "BIN_ERR_UNSUPPORTED";
    case BIN_ERR_OOM: return "BIN_ERR_OOM";
    case BIN_ERR_DEVICE: return "BIN_ERR_DEVICE";
    case BIN_ERR_ADMISSION: return "BIN_ERR_ADMISSION";
    case BIN_ERR_TIMEOUT: return "BIN_ERR_TIMEOUT";
    case BIN_ERR_NOT_FOUND: return "BIN_ERR_NOT_FOUND";
    default: return "BIN_ERR_UNKNOWN";
  }
}

const char* bin_last_error_message(void) { return last_error(); }

int bin_stream_status(void* stream) {
  clear_error();
  return precheck_stream(static_cast<hipStream_t>(stream));
}

int bin_release_workspace(void) {
  clear_error();
  int st = release_all_scratch();  // synchronises the device first
  const int st2 = release_all_staging();
  return st ? st : st2;
}

const char* bin_version(void) { return "0.1.0"; }

int bin_copy_to_host(void* host_dst, const void* device_src, size_t bytes) {
  clear_error();
  if (bytes == 0) return BIN_OK;
  if (!host_dst || !device_src) return fail(BIN_ERR_INVALID_ARG, "NULL copy pointer");
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(host_dst, device_src, bytes, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy(device to host)");
  return BIN_OK;
}

int bin_timing_enable(int on) { return timing_enable(on); }

int bin_timing_read(int64_t* launches, double* total_ms) {
  clear_error();
  return timing_read(launches, total_ms);
}

int bin_timing_report(char* buf, size_t buflen) {
  clear_error();
  return timing_report(buf, buflen);
}

int bin_describe_plan(const bin_request* req, char* buf, size_t buflen) {
  clear_error();
  if (!req || !buf || buflen == 0) return fail(BIN_ERR_INVALID_ARG, "NULL request or buffer");
  int st = validate(&req->coords, &req->attrs, req->n, req->axes, req->bounds, req->nx, req->ny, req->ops,
                    &req->out, false);
  if (st) return st;
  DeviceInfo dev;
  st = device_info(&dev);
  if (st) return st;
  Prepared p;
  st = prepare(*req, dev, thread_hints(), nullptr, &p);
  if (st) return st;
  std::string d = describe(p);
  std::strncpy(buf, d.c_str(), buflen - 1);
  buf[buflen - 1] = 0;
  return BIN_OK;
}

int bin_describe_plan_on(const bin_request* req, int32_t cus, int64_t lds_per_block, int64_t lds_per_cu, char* buf,
                         size_t buflen) {
  clear_error();
  if (!req || !buf || buflen == 0) return fail(BIN_ERR_INVALID_ARG, "NULL request or buffer");
  if (cus < 1 || lds_per_block < 1024 || lds_per_cu < lds_per_block)
    return fail(BIN_ERR_INVALID_ARG, "need cus >= 1 and 1024 <= lds_per_block <= lds_per_cu");
  int st = validate(&req->coords, &req->attrs, req->n, req->axes, req->bounds, req->nx, req->ny, req->ops,
                    &req->out, false);
  if (st) return st;
  DeviceInfo dev;
  dev.device = -1;
  dev.cus = cus;
  dev.lds_per_block = (size_t)lds_per_block;
  dev.lds_per_cu = (size_t)lds_per_cu;
  Prepared p;
  st = prepare(*req, dev, thread_hints(), nullptr, &p);
  if (st) return st;
  std::string d = describe(p);
  std::strncpy(buf, d.c_str(), buflen - 1);
  buf[buflen - 1] = 0;
  return BIN_OK;
}

}  // extern "C"
