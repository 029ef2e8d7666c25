/*
 * binning.h - C ABI of libbinning.so: in situ particle data binning on
 * AMD Instinct MI355X (gfx950).
 *
 * The operation (paper, Section 4.2): particle data is a table whose columns
 * are variables and whose rows are particles.  Two of the variables are the
 * axes of a uniform 2D Cartesian mesh with given bounds; the two coordinate
 * values of a particle select the mesh cell ("bin") it falls in.  Per bin the
 * library counts particles (a histogram) and reduces each other requested
 * variable by sum, minimum, maximum and average.
 *
 * Readings of points the paper leaves open (shared by every entry point):
 *  - Inside test: a particle is binned iff lo <= x <= hi on both axes (the
 *    upper edge is closed and belongs to the last bin).  NaN/Inf coordinates
 *    are never inside.  Particles outside take part in no reduction.
 *  - Bin index, in IEEE binary64 with no fused multiply-add:
 *      s = (double)nbins / (hi - lo);  i = trunc(((double)x - lo) * s);
 *      if (i > nbins - 1) i = nbins - 1;
 *    flat bin b = iy * nx + ix; every output grid is row-major [ny][nx].
 *  - min/max follow IEEE totalOrder on non-NaN values (-0 < +0).  NaN
 *    attribute values are outside the contract.
 *  - Empty bins: count 0, sum 0, min +Inf, max -Inf, avg NaN.
 *  - avg = sum / count formed in binary64 from the merged sum.
 *
 * Data placement (paper, Section 2, zero-copy transfer): the caller hands over
 * raw device pointers together with a stream; the library reads and writes
 * them in place and never copies or frees them.  With raw pointers the caller
 * manages their lifetime: inputs and outputs must stay valid and unmodified
 * until the work enqueued on the stream has completed.
 *
 * Stream semantics (paper, Section 2, asynchronous stream mode): every
 * compute entry point only enqueues work on the given stream and returns; the
 * results are valid once the stream has been synchronised.  No entry point
 * synchronises the stream unless its comment says so.  A stream argument is a
 * hipStream_t passed as void*; NULL means the default stream.
 *
 * Errors: every entry point returns BIN_OK (0) or a negative bin_status.  All
 * argument checks run before the first HIP call, so they hold without a GPU.
 * bin_last_error_message() gives a thread-local explanation of the last
 * failure.  A fault of already-enqueued device work surfaces as
 * BIN_ERR_DEVICE from a later call, or from bin_stream_status().
 *
 * Thread safety: calls on different streams may run concurrently.  Calls on
 * the same stream from several threads are serialised by the stream.
 */
#ifndef BINNING_H
#define BINNING_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
typedef enum bin_status {
  BIN_OK = 0,
  BIN_ERR_INVALID_ARG = -1, /* an argument breaks the contract below        */
  BIN_ERR_UNSUPPORTED = -2, /* valid request the library does not implement */
  BIN_ERR_OOM = -3,         /* device scratch allocation failed             */
  BIN_ERR_DEVICE = -4,      /* a HIP call or enqueued kernel failed         */
  BIN_ERR_ADMISSION = -5,   /* server: request can never fit the budget     */
  BIN_ERR_TIMEOUT = -6,     /* server: wait timed out                       */
  BIN_ERR_NOT_FOUND = -7    /* server: unknown or already released ticket   */
} bin_status;

/* ---- element types ----------------------------------------------------- */
typedef enum bin_dtype { BIN_F32 = 0, BIN_F64 = 1 } bin_dtype;

/* ---- op bits and precision flags (the 'ops' argument) ------------------- */
#define BIN_COUNT 1u  /* per-bin particle count (the histogram)             */
#define BIN_SUM 2u    /* per-bin sum of each attribute                       */
#define BIN_MIN 4u    /* per-bin minimum of each attribute                   */
#define BIN_MAX 8u    /* per-bin maximum of each attribute                   */
#define BIN_AVG 16u   /* per-bin average of each attribute                   */
#define BIN_OPS_ALL 31u
/* Precision of sums of f32 attributes (f64 attributes always accumulate in
 * binary64).  At most one flag:
 *  BIN_PREC_COMP   FP32 accumulation with compensation: per bin an FP32 sum
 *                  word S and an FP32 error word C, updated by the error-free
 *                  TwoSum transformation; S + C merged and finalised in
 *                  binary64.  sum/avg outputs are double.
 *  BIN_PREC_PLAIN  uncompensated FP32 sums; sum/avg outputs are float.
 *  BIN_PREC_F64    binary64 accumulation; sum/avg outputs are double.
 *  (none)          default: at least the accuracy of BIN_PREC_COMP with
 *                  double outputs; on gfx950 this is binary64 accumulation,
 *                  which is also the fastest of the three there. */
#define BIN_PREC_PLAIN 0x100u
#define BIN_PREC_F64 0x200u
#define BIN_PREC_COMP 0x400u

#define BIN_MAX_COLUMNS 64   /* max coordinate columns in one table         */
#define BIN_MAX_ATTRS 16     /* max attributes reduced by one request       */

/* A table of n-row device columns (structure of arrays).  cols[i] is a
 * device pointer to n elements of 'dtype', aligned to the element size. */
typedef struct bin_columns {
  const void* const* cols; /* host array of ncols device pointers           */
  int32_t ncols;
  int32_t dtype; /* bin_dtype */
} bin_columns;

/* Caller-allocated device output grids, each of nx*ny elements, row-major
 * [ny][nx].  They are overwritten, not accumulated into.
 *   count: uint32_t*, required iff BIN_COUNT is requested.
 *   sum/min/max/avg: host arrays of k device pointers (k = attrs->ncols),
 *   required iff the op is requested, NULL otherwise.
 *   Element types: min/max = attribute dtype; sum/avg = double, except float
 *   for f32 attributes under BIN_PREC_PLAIN.
 * No output may alias an input or another output. */
typedef struct bin_output {
  uint32_t* count;
  void* const* sum;
  void* const* min;
  void* const* max;
  void* const* avg;
} bin_output;

/* One binning request (the arguments of bin_particles as a record); used by
 * the batched, graph and server entry points. */
typedef struct bin_request {
  bin_columns coords;
  bin_columns attrs;
  int64_t n;
  int32_t axes[2];
  double bounds[4];
  int32_t nx, ny;
  uint32_t ops;
  bin_output out;
} bin_request;

/* ---- plain entry point -------------------------------------------------- */
/* Bin n particles (paper, Section 4.2) and reduce the attributes per bin.
 *  coords  table of candidate coordinate columns (e.g. x, y, z); axes[0] and
 *          axes[1] pick the columns used as the mesh x and y axes, so the x-y
 *          and x-z planes of one table are two calls on the same columns.
 *  attrs   columns to reduce (k = attrs->ncols, 0..BIN_MAX_ATTRS; attrs may
 *          be NULL for k = 0).  Both tables are f32 or f64; they may differ.
 *  n       rows, 0 <= n <= UINT32_MAX; n == 0 writes empty-bin values.
 *  bounds  {xlo, xhi, ylo, yhi}, finite, lo < hi, (hi - lo) and
 *          nbins / (hi - lo) finite.  NULL asks for bounds computed on the
 *          fly from the minimum and maximum of each axis column (Section
 *          4.2): the library derives them on the device before binning.
 *  nx, ny  mesh cells per axis, >= 1, nx * ny <= 2^31 - 1.
 *  ops     nonzero OR of BIN_COUNT..BIN_AVG, optionally one BIN_PREC_* flag;
 *          SUM/MIN/MAX/AVG need k >= 1.
 *  out     output grids (see bin_output).
 *  stream  hipStream_t (as void*), NULL = default stream.
 * Library scratch (when needed) comes from a pool owned by the library per
 * (device, stream) and is reused across calls; bin_release_workspace frees
 * it.  Returns BIN_OK once the work is enqueued. */
int bin_particles(const bin_columns* coords, const bin_columns* attrs, int64_t n,
                  const int32_t axes[2], const double bounds[4], int32_t nx, int32_t ny,
                  uint32_t ops, const bin_output* out, void* stream);

/* Validate the arguments of bin_particles without touching the GPU.
 * Returns BIN_OK or the status bin_particles would return before any HIP
 * call. */
int bin_validate(const bin_columns* coords, const bin_columns* attrs, int64_t n,
                 const int32_t axes[2], const double bounds[4], int32_t nx, int32_t ny,
                 uint32_t ops, const bin_output* out);

/* ---- allocation-free variant ---------------------------------------------- */
/* For callers that cannot allocate device memory: code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same arguments,
 * outputs, readings and stream semantics as bin_particles, and the same
 * kernels; the library's scratch for the call comes from one fixed device
 * array of BIN_NOALLOC_SCRATCH_BYTES per GPU (part of the library's device
 * code, held from the first call on that GPU until the process ends), so
 * the call allocates nothing: no hipMalloc/hipFree, no allocating library
 * routine, no events.  The caller still owns inputs and outputs.
 * Limit: a request whose plan needs more scratch than the array holds is
 * refused with BIN_ERR_INVALID_ARG before anything is enqueued (roughly, a
 * partition-strategy request takes 6 bytes per particle plus 4 per extra
 * attribute, a whole-grid LDS request one partial grid per workgroup; a
 * request with no scratch - one workgroup - always fits).
 * Concurrency: every call on one GPU uses that GPU's one array, and the
 * array keeps the last call's contents (the kernels set up what they read).
 * Calls whose work overlaps on one GPU - on different streams or from
 * several threads - race on the array; order them, e.g. one stream per GPU. */
#define BIN_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int bin_particles_noalloc(const bin_columns* coords, const bin_columns* attrs, int64_t n,
                          const int32_t axes[2], const double bounds[4], int32_t nx, int32_t ny,
                          uint32_t ops, const bin_output* out, void* stream);

/* ---- meshes of one, two or three axes ----------------------------------- */
/* The mesh axes are any chosen subset of the particle variables (paper,
 * Section 4.2); this entry point takes one, two or three of them.
 *  ndim     1, 2 or 3.
 *  axes     host array of ndim coordinate column indices (repeats allowed).
 *  bounds   host array of 2*ndim doubles {lo0, hi0, lo1, hi1, ...}, finite,
 *           lo < hi; or NULL for bounds from the data (as bin_particles).
 *  dims     host array of ndim bin counts, each >= 1, product <= 2^31 - 1.
 *           With f32 coordinates and ndim = 3, dims[1] * dims[2] <= 2^24.
 * Every axis follows the readings above (closed upper edge, binary64 index);
 * a particle is inside iff it is inside on every axis.  Axis 0 varies
 * fastest: the flat bin is (i2 * dims[1] + i1) * dims[0] + i0 and every
 * output grid is row-major [dims[2]][dims[1]][dims[0]], prod(dims) elements.
 * Other arguments, outputs, errors and stream semantics as bin_particles.
 * ndim = 2 is bin_particles.  With ndim = 3 the library first folds axes 1
 * and 2 into one composite coordinate column in its scratch (one extra pass
 * over those two columns), then bins the two-axis mesh dims[0] by
 * dims[1] * dims[2], which gives the same bins exactly. */
int bin_particles_nd(const bin_columns* coords, const bin_columns* attrs, int64_t n, int32_t ndim,
                     const int32_t* axes, const double* bounds, const int32_t* dims, uint32_t ops,
                     const bin_output* out, void* stream);

/* Argument checks of bin_particles_nd, without touching the GPU. */
int bin_validate_nd(const bin_columns* coords, const bin_columns* attrs, int64_t n, int32_t ndim,
                    const int32_t* axes, const double* bounds, const int32_t* dims, uint32_t ops,
                    const bin_output* out);

/* ---- batched entry point ------------------------------------------------ */
/* Run nreq independent requests (uneven n and grid sizes allowed) on
 * 'stream'.  Requests are planned one by one and grouped by strategy, element
 * types, precision, scatter shape and gather form; each group runs one
 * table-driven launch per stage (scatter, work items, tile binning, merge;
 * or whole-grid LDS binning and merge) for all its requests, a block map
 * listing each block's request and index.  The tile binning and the
 * whole-grid binning split into up to four and three launches by the LDS
 * each request's tile or grid takes, so that small tiles run several
 * workgroups per compute unit next to requests with large ones.  Each result equals
 * what bin_particles gives for the same request, within the sum tolerance;
 * counts, min and max are identical.  Requests must not share output
 * buffers.  The request array is read during the call only.  Enqueues and
 * returns; the descriptor tables go up through a ring of 4 pinned buffers
 * per stream, so the host waits only when 4 earlier batched calls on the
 * same stream have not yet reached the device. */
int bin_particles_batched(const bin_request* reqs, int32_t nreq, void* stream);

/* ---- asynchronous in situ binning ------------------------------------------ */
/* The asynchronous mode of the paper (Section 2, used in the runs of Section
 * 4.3): the simulation hands its data over and carries on at once while the
 * analysis works on a deep copy.  Arguments as bin_particles, plus:
 *  src_stream  the simulation's stream.  The columns the request reads (the
 *              two axis columns and the attributes) are copied device to
 *              device on it, into staging memory that the library allocates
 *              in that stream's order.  Work the caller enqueues on
 *              src_stream after this call runs after the copy, so it may
 *              overwrite the columns at once.
 *  bin_stream  the analysis stream.  It waits for the copy (an event), bins
 *              from the staged copy and frees it in its own order.  The
 *              outputs are valid once bin_stream has completed the call.
 * The two streams may be the same.  Returns BIN_OK once everything is
 * enqueued; errors as bin_particles, plus BIN_ERR_OOM when staging memory
 * cannot be allocated.  Never synchronises. */
int bin_particles_async(const bin_columns* coords, const bin_columns* attrs, int64_t n,
                        const int32_t axes[2], const double bounds[4], int32_t nx, int32_t ny,
                        uint32_t ops, const bin_output* out, void* src_stream, void* bin_stream);

/* ---- several grids over one particle table --------------------------------- */
/* One binning of the table per grid spec.  The in situ load of the paper's
 * experiments (Section 4.3) bins the same variables over several coordinate
 * systems at every step, each system as its own operator instance run in
 * sequence; here all of them are one enqueue.  When the specs qualify (f32
 * columns, 2 to 32 specs on the tile partition, at most 40 distinct columns)
 * the table is read from device memory once: one fused scatter stages each
 * block of particles' columns on chip and writes every grid's tile-ordered
 * records, then one tile-binning launch serves all grids.  Other spec sets
 * run as one batch (bin_particles_batched).  Each spec picks its own axes
 * (two columns of coords), bounds ({xlo, xhi, ylo, yhi}, explicit), mesh,
 * ops and outputs, with the rules of bin_particles; all specs share coords,
 * attrs and n.  Attributes binned on the same axes belong in one spec (k
 * attributes of one spec share every per-particle step).  Results equal
 * those of one bin_particles call per spec.  Invalid specs are reported as
 * "request g: ..." before anything is enqueued.  Outputs of different specs
 * must not overlap.  Enqueues and returns. */
typedef struct bin_grid_spec {
  int32_t axes[2];
  double bounds[4];
  int32_t nx, ny;
  uint32_t ops;
  bin_output out;
} bin_grid_spec;
int bin_particles_multi(const bin_columns* coords, const bin_columns* attrs, int64_t n,
                        const bin_grid_spec* grids, int32_t ngrids, void* stream);

/* ---- graphs ---------------------------------------------------------------- */
/* Capture the batched launch of nreq requests as a HIP graph.  The graph
 * owns its descriptor and scratch memory; the caller's buffers are borrowed
 * each time the graph is launched.  Replays re-read the input columns and
 * overwrite the outputs, so the caller may refill the inputs between
 * launches.  Creating a graph synchronises the device once. */
typedef struct bin_graph bin_graph;
int bin_graph_create(const bin_request* reqs, int32_t nreq, bin_graph** graph);
/* The same for what bin_particles_multi(coords, attrs, n, grids, ngrids)
 * enqueues (the fused pass over the table when the specs qualify, else
 * their batch): the per-step in situ load of the paper's experiments
 * (Section 4.3), replayed every step.  The columns and outputs named here are
 * borrowed by every launch; refill them between launches.  Arguments are
 * checked as by bin_particles_multi, before any HIP call. */
int bin_graph_create_multi(const bin_columns* coords, const bin_columns* attrs, int64_t n,
                           const bin_grid_spec* grids, int32_t ngrids, bin_graph** graph);
int bin_graph_launch(bin_graph* graph, void* stream);
int bin_graph_destroy(bin_graph* graph);

/* ---- autotuning ------------------------------------------------------------ */
/* Time the candidate kernel configurations for requests shaped like
 * reqs[0..count) and remember the fastest per (device, shape class).  The
 * candidates include the strategy itself where both apply (whole grid in
 * LDS, tile partition), the tile size, the scatter shape and the gather
 * form.  With two or more requests it then times the whole set as one batch
 * under each batch policy - every request's tuned plan, the planner's rules,
 * or the rules with one shared scatter shape - and keeps the fastest for the
 * device: batched calls, graphs and the server plan under it (plans tuned
 * one request at a time can split a batch into more, smaller launch groups).
 * The tables are kept in memory and, if the environment variable
 * BIN_TUNE_CACHE names a file, read from and written back to it as JSON:
 *   {"version": 1, "entries": {"gfx950:256|n20_b16_k1_c0_a0_o31":
 *     {"strategy": 2, "block": 0, "grid": 0, "part_wg": 512,
 *      "scatter_ppt": 16, "scatter_threads": 1024, "tile_shift": 13,
 *      "split_len": 0, "quads": 2}, ...},
 *    "batch": {"gfx950:256": {"strategy": 0, ...}}}
 * (entry key: device architecture and compute units, then log2 of n and of
 * the bin count, attributes, coordinate and attribute dtypes, ops; batch
 * "strategy": 0 rules, 1 tuned plans, 2 rules with the entry's
 * scatter_threads and scatter_ppt).  Runs kernels on a private stream and
 * synchronises it; it overwrites the requests' output buffers.  Without
 * tuning data the built-in rules apply. */
int bin_autotune(const bin_request* reqs, int32_t count);

/* ---- diagnostics -------------------------------------------------------- */
const char* bin_status_string(int status);
/* Thread-local description of the last failure on this thread ("" if none). */
const char* bin_last_error_message(void);
/* Non-blocking: BIN_ERR_DEVICE if work on 'stream' has faulted, else BIN_OK. */
int bin_stream_status(void* stream);
/* Free every scratch pool of the library (all devices and streams).
 * Synchronises the device first, so no enqueued work can still use them. */
int bin_release_workspace(void);
/* Library version as "major.minor.patch". */
const char* bin_version(void);
/* Copy 'bytes' from device memory to host memory, synchronously (waits for
 * all work on the device).  A convenience for callers without a HIP runtime
 * of their own, e.g. to read a server's resident result grids. */
int bin_copy_to_host(void* host_dst, const void* device_src, size_t bytes);

/* Kernel timing, for measurement only: while enabled, every kernel launch of
 * the library is bracketed by a HIP event pair on its stream.  Enabling
 * clears earlier totals.  bin_timing_read waits for the recorded events and
 * returns the launches and summed milliseconds of the kernel with the
 * largest total (the dominant kernel); bin_timing_report writes all kernels
 * as JSON {"name": [launches, total_ms], ...} into buf. */
int bin_timing_enable(int on);
int bin_timing_read(int64_t* launches, double* total_ms);
int bin_timing_report(char* buf, size_t buflen);

/* Override the planner for later calls made by this thread (tests and the
 * autotuner): strategy -1 = automatic, 0 = global atomics, 1 = whole grid
 * in LDS, 2 = partition by tile (1 and 2 are ignored when they do not fit);
 * block/grid 0 = automatic (grid = workgroups of the binning or partition
 * pass). */
int bin_set_plan_override(int32_t strategy, int32_t block, int32_t grid);

/* Tuning parameters of the partition strategy for later calls made by this
 * thread (autotuner, tests); value 0 restores the planner's choice.
 *  BIN_TUNE_PART_WG          workgroups of the count and scatter passes
 *  BIN_TUNE_SCATTER_PPT      particles per thread per scatter sub-chunk (4, 8, 12, 16 or
 *                            32; 12 with 1024 threads only, else taken as 8)
 *  BIN_TUNE_SCATTER_THREADS  threads per scatter workgroup (256, 512 or 1024)
 *  BIN_TUNE_TILE_SHIFT       log2 of the largest tile (6..15)
 *  BIN_TUNE_SPLIT_LEN        max records per binning work item (>= 1024)
 *  BIN_TUNE_QUADS            1 = gather record by record, 2 = pad each tile's run
 *                            to whole quads of 4 records and gather a quad per lane
 *                            (default: quads for at most one f32 attribute and
 *                            sub-chunks of 16 or more records per tile)
 * Returns BIN_ERR_INVALID_ARG for an unknown parameter or value. */
#define BIN_TUNE_PART_WG 1
#define BIN_TUNE_SCATTER_PPT 2
#define BIN_TUNE_SCATTER_THREADS 3
#define BIN_TUNE_TILE_SHIFT 4
#define BIN_TUNE_SPLIT_LEN 5
#define BIN_TUNE_QUADS 6
int bin_set_tuning(int32_t param, int64_t value);

/* Describe the strategy the planner picks for a request (no GPU work):
 * writes a short NUL-terminated text such as "lds wg=256 ppt=8" into buf. */
int bin_describe_plan(const bin_request* req, char* buf, size_t buflen);

/* The plan bin_describe_plan gives for a device with 'cus' compute units and
 * the given LDS bytes per workgroup and per CU, without any HIP call (for
 * capacity planning and for tests on machines without a GPU).  MI355X:
 * 256, 163840, 163840.  Same errors as bin_describe_plan, plus
 * BIN_ERR_INVALID_ARG for cus < 1 or LDS sizes outside
 * 1024 <= lds_per_block <= lds_per_cu. */
int bin_describe_plan_on(const bin_request* req, int32_t cus, int64_t lds_per_block, int64_t lds_per_cu, char* buf,
                         size_t buflen);

/* ---- serving --------------------------------------------------------------- */
/* A request server with continuous batching: binsrv_submit may be called
 * from any thread while earlier requests run.  Waiting requests are admitted
 * in arrival order as soon as a stream slot and enough device memory (the
 * budget: result grids plus the library scratch of the batch as it will run)
 * are free - by binsrv_submit itself when a slot is free, else when a batch
 * finishes or grids are released - and each admitted group runs as one
 * batched launch on its slot's stream (a lone request runs the
 * single-request kernels).  Each slot has a waiter thread blocked on the
 * slot's completion event, which stamps the requests done.  Result grids
 * stay resident on the device until binsrv_release.  Device memory is
 * allocated outside the server's lock. */
typedef struct binsrv binsrv;
typedef struct binsrv_config {
  uint64_t budget_bytes;   /* device memory for result grids and scratch    */
  int32_t n_slots;         /* concurrent batches in flight (streams), >= 1  */
  int32_t max_batch;       /* max requests per batched launch, >= 1         */
  int32_t device;          /* HIP device ordinal                            */
  int32_t reserved;
} binsrv_config;

/* A server request: like bin_request but without outputs; the server
 * allocates the result grids (all five op kinds as requested, with the
 * default precision rules) from its budget.  producer_stream: the stream
 * (hipStream_t as void*) whose work writes the input columns, or NULL when
 * they are complete on the device before binsrv_submit.  The server records
 * an event on it at submit time and its kernels read the columns only after
 * that event, so a simulation may enqueue its writes and submit at once. */
typedef struct binsrv_request {
  bin_columns coords;
  bin_columns attrs;
  int64_t n;
  int32_t axes[2];
  double bounds[4];
  int32_t nx, ny;
  uint32_t ops;
  void* producer_stream;
} binsrv_request;

/* Where a finished request's resident grids are (device pointers owned by
 * the server until binsrv_release), plus its timing. */
typedef struct bin_result {
  int32_t status;          /* BIN_OK or the request's error                 */
  int32_t k;
  uint32_t* count;
  void* sum[BIN_MAX_ATTRS];
  void* min[BIN_MAX_ATTRS];
  void* max[BIN_MAX_ATTRS];
  void* avg[BIN_MAX_ATTRS];
  double submit_to_done_ms; /* arrival (submit) to completion observed      */
  double queue_ms;          /* arrival to dispatch                          */
} bin_result;

typedef struct binsrv_stats {
  uint64_t submitted, completed, failed, released;
  uint64_t batches, in_flight, queued;
  uint64_t bytes_in_use, peak_bytes;
} binsrv_stats;

int binsrv_create(const binsrv_config* cfg, binsrv** srv);
/* Queue a request (and launch it at once when a slot and memory are free).
 * Inputs are borrowed until the request completes; they must be complete on
 * the device before submit, or written on req->producer_stream.  Returns
 * BIN_ERR_ADMISSION if it can never fit the budget.  A request whose result
 * grids cannot be allocated fails alone (BIN_ERR_OOM from binsrv_wait). */
int binsrv_submit(binsrv* srv, const binsrv_request* req, uint64_t* ticket);
/* Wait up to timeout_ns (negative = forever) for a ticket's completion;
 * fills *result and returns the request's status.  BIN_ERR_TIMEOUT if it is
 * not done in time.  Safe to call while another thread destroys the server:
 * the call then either fails with BIN_ERR_INVALID_ARG or completes before
 * the server is freed. */
int binsrv_wait(binsrv* srv, uint64_t ticket, int64_t timeout_ns, bin_result* result);
/* Return a finished request's grids to the server's pool. */
int binsrv_release(binsrv* srv, uint64_t ticket);
int binsrv_get_stats(binsrv* srv, binsrv_stats* stats);
/* Drain waiting and in-flight work, free every grid and stop the slot
 * waiters.  Calls made concurrently on the same server either fail with
 * BIN_ERR_INVALID_ARG or finish before it is freed. */
int binsrv_destroy(binsrv* srv);

#ifdef __cplusplus
}
#endif
#endif /* BINNING_H */
