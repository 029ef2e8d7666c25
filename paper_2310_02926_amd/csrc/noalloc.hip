// bin_particles_noalloc: bin_particles for callers that cannot allocate
// device memory (code under stream capture, tight serving loops, harnesses
// that forbid hipMalloc).  The request's scratch - partition records, run
// tables, per-slice counts, work items, partial slots, bounds keys - lives
// in one fixed device array of this library instead of the per-(device,
// stream) pool.
//
// Each GPU holds its own copy of the array, at its own address, from the
// first call on that device until the process ends.  In host code the
// array's name is only a stand-in for the device symbol: its device address
// is looked up once per device with hipGetSymbolAddress (with that device
// current) and only that address is handed to kernels.
//
// Every call on one device shares that device's array and leaves the last
// call's contents in it; the kernels initialise everything they read before
// reading it (as they do with the pooled scratch, which is reused across
// calls), so nothing is cleared here.  Calls whose work overlaps on one
// device - on different streams, or from several threads - race on the
// array: the caller orders them, e.g. by using one stream per device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

using namespace binimpl;

static __device__ __align__(256) unsigned char scratch[BIN_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of 'scratch' per device, once looked up

// Device address of this device's copy of the array (looked up on the first
// call made on the device, with it current).
int device_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices)
    return fail(BIN_ERR_UNSUPPORTED, "device %d: the allocation-free entry point serves devices 0..%d", dev,
                kMaxDevices - 1);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(BIN_ERR_DEVICE, "hipGetSymbolAddress(scratch) gave a null address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return BIN_OK;
}

}  // namespace

extern "C" int bin_particles_noalloc(const bin_columns* coords, const bin_columns* attrs, int64_t n,
                                     const int32_t axes[2], const double bounds[4], int32_t nx, int32_t ny,
                                     uint32_t ops, const bin_output* out, void* stream) {
  clear_error();
  int st = validate(coords, attrs, n, axes, bounds, nx, ny, ops, out, true);
  if (st) return st;
  void* base = nullptr;
  st = device_scratch(&base);
  if (st) return st;
  const FixedScratch fixed{base, (size_t)BIN_NOALLOC_SCRATCH_BYTES};
  const bin_request r = make_request(coords, attrs, n, axes, bounds, nx, ny, ops, out);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // Untimed: the kernel timer creates events, which this entry point avoids.
  if (!bounds) return run_auto_bounds_in(r, s, &fixed, nullptr);
  return run_request_in(r, s, thread_hints(), &fixed, nullptr);
}
