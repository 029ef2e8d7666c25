// Declarations shared by the host-side translation units of libbinning.so.
#ifndef BINNING_INTERNAL_H
#define BINNING_INTERNAL_H

#include <hip/hip_runtime.h>
#include <stdarg.h>

#include <atomic>
#include <functional>
#include <string>

#include "../../include/binning.h"
#include "kernels.h"

namespace binimpl {

// Tuning overrides for the planner (autotuner, tests); zero fields = default.
struct PlanHints {
  int force_strategy = -1;  // -1 auto, else bk::Strategy
  int block = 0;
  int grid = 0;
  // partition tuning (bin_set_tuning)
  int part_wg = 0;
  int scatter_ppt = 0;
  int scatter_threads = 0;
  int tile_shift = 0;
  int64_t split_len = 0;
  int quads = 0;  // 0 planner's choice, 1 off, 2 on
  int share = 1;  // grids binned together in one call: their tiles fill the device together
};
PlanHints& thread_hints_mut();

// errors (thread-local message)
int fail(int status, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);
void clear_error();
const char* last_error();

// argument checks (no HIP calls)
int validate(const bin_columns* coords, const bin_columns* attrs, int64_t n, const int32_t axes[2],
             const double bounds[4], int32_t nx, int32_t ny, uint32_t ops, const bin_output* out,
             bool allow_null_bounds);
int validate_nd(const bin_columns* coords, const bin_columns* attrs, int64_t n, int32_t ndim,
                const int32_t* axes, const double* bounds, const int32_t* dims, uint32_t ops,
                const bin_output* out);

struct DeviceInfo {
  int device = 0;
  int cus = 256;
  size_t lds_per_block = 65536;
  size_t lds_per_cu = 65536;
  char arch[48] = "";  // "<architecture>:<compute units>", empty for a device described by sizes only
};
int device_info(DeviceInfo* info);

// scratch pools
int scratch_get(int dev, hipStream_t s, size_t bytes, void** out);
// Give the pool of (dev, s) back, in s's order.
int scratch_release(int dev, hipStream_t s);
int release_all_scratch();
// Asynchronous mode: copy(stage) enqueues the deep copy on src into a
// staging buffer of at least 'bytes'; bin(stage) enqueues the binning on bs,
// which is ordered after the copy.  Buffers are reused once their binning
// has completed.
int stage_run(int device, hipStream_t src, hipStream_t bs, size_t bytes,
              const std::function<int(void* stage)>& copy, const std::function<int(void* stage)>& bin);
int release_all_staging();
bool fault_injection_hit();

// kernel timing (bin_timing_*): a timer for one call, or null when off
bk::KTimer* timing_timer();
int timing_enable(int on);
int timing_read(int64_t* launches, double* total_ms);
int timing_report(char* buf, size_t buflen);

// One request turned into kernel arguments.
struct Prepared {
  bk::BinArgs bin;
  bk::InitArgs init;
  bk::FinArgs fin;
  bk::LdsArgs lds;
  bk::PartArgs part;
  bk::PartCfg pcfg;
  bk::LaunchCfg cfg;
  bool coord_f64 = false, attr_f64 = false;
  int prec = bk::PREC_F64;
  bool need_finalize = false;
  size_t scratch_bytes = 0;
  int init_grid = 1, fin_grid = 1;
};

const PlanHints& thread_hints();
int resolve_precision(uint32_t ops, bool attr_f64);
// The caller's explicit hints, else the autotuned entry for the request's
// shape class, else defaults.
PlanHints effective_hints(const bin_request& r, const DeviceInfo& dev, const PlanHints& explicit_hints);
bool hints_are_default(const PlanHints& h);
// How a batch plans its requests, chosen by bin_autotune by timing the
// whole set: 0 the planner's rules, 1 each request's tuned plan (also the
// choice without tuning data), 2 the planner's rules with one scatter shape
// (nt threads of ppt particles) for every tile-partition request.
struct BatchPolicy {
  int mode = 1;
  int nt = 0, ppt = 0;
};
BatchPolicy batch_policy(const DeviceInfo& dev);
// While alive, effective_hints on this thread ignores the tuning table.
struct TunedLookupOff {
  TunedLookupOff();
  ~TunedLookupOff();
};
int autotune(const bin_request* reqs, int count);

// Plan a validated request and lay out its scratch at 'scratch' (may be null
// when only sizing: then pointers into scratch are left null and
// scratch_bytes is filled in).
int prepare(const bin_request& r, const DeviceInfo& dev, const PlanHints& hints, void* scratch, Prepared* p);
// Sub-chunk sizes and the blk_off rows per slice of a partition request
// whose scatter runs with these threads and particles per thread.
void set_part_blocks(bk::PartArgs& a, int scatter_threads, int ppt);
// Place the scatter's LDS stage of run-table rows at stage_base (rounded up)
// with as many rows (a power of two, at most 16 and no more than a slice's
// sub-chunks need) as fit lds_limit; returns the scatter's LDS bytes.
size_t set_off_stage(bk::PartArgs& a, size_t stage_base, size_t lds_limit);
// Padding record slots per sub-chunk (runs padded to whole quads) and the
// record slots a partition request needs.
bool use_quads(int nk, bool attr_f64, int64_t ntiles, int64_t sub);
int32_t part_pad_row(int64_t ntiles, int64_t sub);
size_t part_records(const bk::PartArgs& a);
// Work-item and partial-slot bounds (max_items, max_slots, merge_blocks) of
// a partition request whose blocks and padding are set.
void set_part_items(bk::PartArgs& a, int cus);
// Workgroups of the split-tile merge launch (a.max_slots and a.lay set).
int32_t merge_blocks(const bk::PartArgs& a, int cus);
// Enqueue the kernels of a prepared request.
int enqueue(const Prepared& p, hipStream_t s, bk::KTimer* tm);
// Human-readable plan.
std::string describe(const Prepared& p);

// Whole requests.
bin_request make_request(const bin_columns* coords, const bin_columns* attrs, int64_t n, const int32_t axes[2],
                         const double bounds[4], int32_t nx, int32_t ny, uint32_t ops, const bin_output* out);
int run_request(const bin_request& r, hipStream_t s, const PlanHints& hints);
int run_auto_bounds(const bin_request& r, hipStream_t s);
// The same with the scratch taken from a fixed device block of cap bytes
// (nothing is allocated; a request needing more fails with
// BIN_ERR_INVALID_ARG), or from the pool when fixed is null; tm times the
// launches (null: untimed).
struct FixedScratch {
  void* ptr;
  size_t cap;
};
int run_request_in(const bin_request& r, hipStream_t s, const PlanHints& hints, const FixedScratch* fixed,
                   bk::KTimer* tm);
int run_auto_bounds_in(const bin_request& r, hipStream_t s, const FixedScratch* fixed, bk::KTimer* tm);
int run_batch(const bin_request* reqs, int nreq, hipStream_t s, const PlanHints& hints);
// Device scratch a batch needs (0 and *status set on a bad batch).
size_t batch_scratch_bytes(const bin_request* reqs, int nreq, int* status);

}  // namespace binimpl

#endif
