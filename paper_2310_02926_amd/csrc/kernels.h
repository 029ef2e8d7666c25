// Argument records shared by the binning kernels and their host launchers.
// Plain C++ structs passed by value as kernel arguments; device pointers only.
#ifndef BINNING_KERNELS_H
#define BINNING_KERNELS_H

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bk {

constexpr int kMaxAttrs = 16;  // matches BIN_MAX_ATTRS

// Sum accumulation: FP32 with TwoSum compensation, plain FP32, binary64.
enum Prec { PREC_COMP = 0, PREC_PLAIN = 1, PREC_F64 = 2 };
// STRAT_GLOBAL: device-scope atomics into the result grids.
// STRAT_LDS: each workgroup holds the whole grid in LDS.
// STRAT_PART: particles partitioned by tile, one LDS tile per work item.
enum Strategy { STRAT_GLOBAL = 0, STRAT_LDS = 1, STRAT_PART = 2 };
enum SrcKind { SRC_F64 = 0, SRC_F32 = 1, SRC_F32_COMP = 2 };

// One mesh axis: bounds, precomputed binary64 scale n / (hi - lo), cells.
struct Axis {
  double lo, hi, scale;
  int32_t n;
  int32_t pad;
};

// Result grids (null = not requested).  sum/avg are double, or float under
// PREC_PLAIN; min/max have the attribute's type.
struct Outs {
  uint32_t* cnt;
  void* sum[kMaxAttrs];
  void* mn[kMaxAttrs];
  void* mx[kMaxAttrs];
  void* avg[kMaxAttrs];
};

// Accumulators of one tile of TB bins in LDS, and the same accumulators as
// a partial slot in device memory (byte offsets; count array at offset 0 in
// both).  Sum words: f64, or f32 S and C (compensated), or f32 (plain) in
// LDS; f64 (or f32 plain) in slots.  min/max as order-preserving keys.
struct TileLayout {
  int32_t lds_sum_off[kMaxAttrs];
  int32_t lds_min_off[kMaxAttrs];
  int32_t lds_max_off[kMaxAttrs];
  int32_t slot_sum_off[kMaxAttrs];
  int32_t slot_min_off[kMaxAttrs];
  int32_t slot_max_off[kMaxAttrs];
  int64_t slot_bytes;
  int32_t tile_shift;  // TB = 1 << tile_shift (partition); LDS strategy: TB = nbins
  int32_t tb;          // bins held in LDS per tile
  int32_t want_sum;    // accumulate sums (SUM or AVG requested)
  int32_t want_min, want_max;
  int32_t mm_pair;     // min and max both kept: interleaved in LDS (min of local bin b at
                       // element 2b of the min array, max at 2b + 1 = the max array's 2b)
};

// ---- global-atomic strategy ---------------------------------------------
// Global accumulators of one attribute.  sum: double* or float* (see
// sum_is_f64); comp: float* error words (compensated mode only); mn/mx:
// result arrays of the attribute's type, or null when not requested.
struct AccPtrs {
  void* sum;
  float* comp;
  void* mn;
  void* mx;
  int32_t sum_is_f64;
  int32_t minmax_f64;
};

struct BinArgs {
  const void* x;
  const void* y;
  const void* attr[kMaxAttrs];
  uint32_t* cnt;  // global count accumulator, or null
  AccPtrs acc[kMaxAttrs];
  Axis ax, ay;
  const long long* dyn;  // bounds computed on the device (4 keys), or null
  int64_t n;
  int32_t nx, nbins, k, pad;
};

struct InitArgs {
  uint32_t* cnt;
  AccPtrs acc[kMaxAttrs];
  int64_t nbins;
  int32_t k, pad;
};

struct FinAttr {
  const void* src;    // merged sum words (kind below)
  const float* comp;  // error words for SRC_F32_COMP
  void* sum_out;      // double sum output written here (SRC_F32_COMP only)
  void* avg_out;      // avg output or null
  int32_t src_kind;
  int32_t avg_f64;
};

struct FinArgs {
  const uint32_t* cnt;
  FinAttr attr[kMaxAttrs];
  int64_t nbins;
  int32_t k, pad;
};

// ---- LDS strategy (whole grid per workgroup) -----------------------------
struct LdsArgs {
  const void* x;
  const void* y;
  const void* attr[kMaxAttrs];
  Axis ax, ay;
  const long long* dyn;  // bounds computed on the device (4 keys), or null
  int64_t n;
  int64_t chunk;   // particles per workgroup
  int32_t nx, nbins, k, nslots;
  int32_t vec;     // every column 16-byte aligned and chunk % 4 == 0: wide loads
  int32_t pad;
  Outs out;
  TileLayout lay;
  void* partial;   // nslots partial slots (nslots > 1)
};

// A batch of LDS-strategy requests (records in a device table).
struct LdsBatch {
  const LdsArgs* descs;
  const uint32_t* map_slot;   // binning blocks (index = workgroup slice)
  const uint32_t* map_merge;  // merge blocks (index = 64-bin chunk)
  int32_t nreq, n_slot_blocks, n_merge_blocks, pad;
  // The binning blocks run as up to three launches, one per class of grid
  // LDS: class c is map_slot[cls_first[c], cls_first[c + 1]) with
  // cls_block[c] threads and cls_lds[c] bytes of LDS per workgroup.
  int32_t cls_first[4];
  int32_t cls_block[3];
  int32_t cls_lds[3];
};

// ---- partition strategy --------------------------------------------------
struct PartArgs {
  const void* x;
  const void* y;
  const void* attr[kMaxAttrs];
  Axis ax, ay;
  const long long* dyn;  // bounds computed on the device (4 keys), or null
  int64_t n;
  int64_t chunk;       // particles per scatter workgroup slice (a multiple of 64)
  int32_t nx, nbins, k, ntiles, nwg, max_items;
  uint32_t split_len;  // max records per work item (whole slices are never split)
  int32_t stage_val_off;  // byte offset of staged values in the scatter LDS
  int32_t sub;         // particles per whole sub-chunk (scatter threads x particles per thread)
  int32_t sub_tail;    // particles per remainder sub-chunk (scatter threads x 4)
  int32_t nbpw;        // rows of the run table reserved per slice (upper bound on its sub-chunks)
  int32_t vec;         // every column 16-byte aligned: whole sub-chunks use wide loads
  int32_t nfull_a, nblocks_a;  // whole / all sub-chunks of every slice but the last
  int32_t nfull_z, nblocks_z;  // the same for the last slice
  int32_t off_shift;   // the scatter stages 2^off_shift rows of the run table in LDS
  int32_t off_stage;   // byte offset of that stage in the scatter LDS
  int32_t quads;       // runs padded to whole quads of 4 records, gathered a quad per lane
  int32_t pad_row;     // record slots per sub-chunk beyond its particles (a multiple of 4;
                       // 0 without quads)
  uint32_t* counts;    // [ntiles][nwg] records of each tile in each slice
  uint16_t* blk_off;   // [ntiles + 1][nwg * nbpw] start of each tile's run within its sub-chunk
                       // (row w * nbpw + j = sub-chunk j of slice w; entry ntiles = records)
  uint16_t* rec_bin;   // records: sub-chunk j of slice w, starting at particle i, writes
  void* rec_val[kMaxAttrs];  //   its records, grouped by tile (with quads each tile's run
                       //   padded to a multiple of 4, pad bin 0xFFFF), from
                       //   i + (w * nbpw + j) * pad_row
  uint32_t* ilist;     // [ntiles][nwg] first slice of each of a tile's items
  uint32_t* items;     // [max_items][3]: tile, first slice, end slice
  uint32_t* n_items;   // [1]
  uint32_t* tile_items;  // [ntiles][3]: first item, item count, first partial slot
  uint32_t* split_list;  // [ntiles + 1]: tiles binned by several items; count at [ntiles]
  int32_t merge_blocks;  // workgroups of the merge launch
  void* partial;       // max_slots partial slots (items of split tiles)
  int32_t max_slots, pad;
  Outs out;
  TileLayout lay;
};

// A batch of partition requests: records in a device table; each launch
// lists its blocks in a map (request << 16 | index within the request).
struct PartBatch {
  const PartArgs* descs;
  const uint32_t* map_wg;    // scatter blocks (index = workgroup slice)
  const uint32_t* map_walk;  // item walk blocks (index = group of 16 tiles)
  const uint32_t* map_item;  // binning blocks (index = work item)
  const uint32_t* map_tile;  // merge blocks (index = merge workgroup of the request)
  int32_t nreq, n_wg_blocks, n_walk_blocks, n_item_blocks, n_tile_blocks;
  // The binning blocks run as up to four launches, one per class of tile
  // LDS: class c is map_item[cls_first[c], cls_first[c + 1]) with
  // cls_block[c] threads and cls_lds[c] bytes of LDS per workgroup.
  int32_t cls_first[5];
  int32_t cls_block[4];
  int32_t cls_lds[4];
};

// ---- several grids over one table: the fused scatter -----------------------
// Every grid's requests share the table, n, the slices and the sub-chunk
// size; per sub-chunk the union of the columns the grids read (f32) is
// staged in LDS once and each grid then writes its records exactly as the
// single-grid scatter does.  Sub-chunks are all of kMultiSub particles (the
// slice shape of unaligned requests with 512 threads of 4 particles).
constexpr int kMultiGrids = 32;
constexpr int kMultiCols = 40;
constexpr int kMultiSub = 2048;      // particles per sub-chunk
constexpr int kMultiThreads = 1024;  // threads per workgroup (2 particles each)
constexpr int kMultiGroup = 4;       // grids ranked and staged together
constexpr int kMultiPrefetch = 12;   // columns whose next sub-chunk is read ahead in registers
struct MultiScatterArgs {
  const PartArgs* grids;            // device descriptors of the grids
  const float* cols[kMultiCols];    // union of the columns read
  int32_t gx[kMultiGrids], gy[kMultiGrids];  // union index of each grid's x and y column
  int32_t attr_col[kMaxAttrs];      // union index of attribute j (shared by every grid)
  int32_t grid_lds[kMultiGrids];    // byte offset of grid g's counters (cnt[2][T], off[T], tot[T])
  int32_t grid_ost[kMultiGrids];    // byte offset of grid g's staged run-table rows
  int32_t ngrids, ncols, k;
  int32_t cols_lds;                 // byte offset of the staged columns ([ncols][sub] floats)
  int32_t stage;                    // byte offset of the record stages, one per grid of a group:
                                    //   bins u16[kMultiSub], then source particles u16[kMultiSub]
  int32_t group;                    // grids ranked and staged together (1..kMultiGroup)
  int32_t vec;                      // every column 16-byte aligned: staged with wide loads
};

struct PartCfg {
  size_t scatter_lds, bin_lds;
  int ppt;              // particles per thread per scatter sub-chunk
  int scatter_threads;  // threads per scatter workgroup
  int bin_block;
  int quads;            // batches: the group's requests gather a quad per lane
};

// Three-axis meshes: axes 1 and 2 folded into one composite coordinate
// column (out, same type as the coordinates, n entries).
struct FoldArgs {
  const void* y;
  const void* z;
  void* out;
  Axis ay, az;
  const long long* dyn_in;  // six keys (axes 0, 1, 2) or null for given bounds
  long long* dyn_out;       // four keys for the folded two-axis mesh, or null
  int64_t n;
  int32_t vec;              // y, z and out 16-byte aligned
  int32_t pad;
};

// Optional per-kernel timing: begin() records an event before a launch,
// end(name) one after it; both on the launch stream.
struct KTimer {
  virtual void begin(hipStream_t s) = 0;
  virtual void end(const char* name, hipStream_t s) = 0;
  virtual ~KTimer() {}
};

struct LaunchCfg {
  int strategy;
  int grid, block;
  size_t lds_bytes;
};

hipError_t launch_bin_global(const BinArgs& a, bool coord_f64, bool attr_f64, int prec, const LaunchCfg& c,
                             hipStream_t s, KTimer* tm);
hipError_t launch_bin_lds(const LdsArgs& a, bool coord_f64, bool attr_f64, int prec, const LaunchCfg& c,
                          hipStream_t s, KTimer* tm);
hipError_t launch_lds_batch(const LdsBatch& b, bool coord_f64, bool attr_f64, int prec, hipStream_t s, KTimer* tm);
hipError_t launch_init(const InitArgs& a, int grid, hipStream_t s, KTimer* tm);
hipError_t launch_finalize(const FinArgs& a, int grid, hipStream_t s, KTimer* tm);
hipError_t launch_partition(const PartArgs& a, bool coord_f64, bool attr_f64, int prec, const PartCfg& c,
                            hipStream_t s, KTimer* tm);
hipError_t launch_partition_batch(const PartBatch& b, bool coord_f64, bool attr_f64, int prec, const PartCfg& c,
                                  hipStream_t s, KTimer* tm);
hipError_t set_lds_limit(size_t bytes);
hipError_t set_dynamic_lds_limit(const void* fn, size_t total);
hipError_t launch_bounds(const void* x, const void* y, bool coord_f64, int64_t n, long long* keys, int cus,
                         hipStream_t s, KTimer* tm);
hipError_t set_partition_lds_limit(size_t bytes);
// Fused scatter of several grids over one table (args: device copy).
hipError_t launch_scatter_multi(const MultiScatterArgs* args, int nwg, size_t lds, hipStream_t s, KTimer* tm);
// The stages after the scatter of a batch of partition requests.
hipError_t launch_partition_batch_after_scatter(const PartBatch& b, bool coord_f64, bool attr_f64, int prec,
                                                const PartCfg& c, hipStream_t s, KTimer* tm);

hipError_t launch_fold(const FoldArgs& a, bool coord_f64, int cus, hipStream_t s, KTimer* tm);

}  // namespace bk

#endif
