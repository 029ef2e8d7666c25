// Planning of one binning request: strategy choice, launch shapes, scratch
// layout and kernel argument records; then the launch sequence.
//
// Strategy choice on gfx950 (LDS atomics ~100x the rate of device-scope
// atomics):
//   LDS        whole grid fits one workgroup's LDS: each workgroup bins a
//              slice, partials merged with plain loads/stores.
//   PARTITION  otherwise, if the grid splits into at most kMaxTiles
//              LDS-sized tiles: particles are partitioned by tile first.
//   GLOBAL     device-scope atomics; only for grids beyond kMaxTiles tiles.
#include <algorithm>
#include <cstdio>
#include <cstring>

#include "internal.h"

namespace binimpl {

namespace {

constexpr int kMaxTiles = 4096;         // tile ids are 16-bit in the scatter stage
constexpr size_t kScatterStatic = 256;  // static LDS of part_scatter_kernel (wave totals)

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }
size_t align16(size_t v) { return (v + 15) & ~size_t(15); }
int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Bump allocator over the scratch block (or a pure size count when base is
// null).
struct Carve {
  unsigned char* base;
  size_t used = 0;
  void* take(size_t bytes) {
    void* p = base ? base + used : nullptr;
    used += align256(bytes);
    return p;
  }
};

// Sub-chunks of partition slice w (mirrors the device-side slice shape):
// whole ones of 'sub' particles for aligned requests, then remainder ones of
// 'sub_tail'.
int64_t slice_blocks(const bk::PartArgs& a, int64_t w) {
  const int64_t lo = w * a.chunk;
  const int64_t hi = std::min<int64_t>(lo + a.chunk, a.n);
  const int64_t len = std::max<int64_t>(hi - lo, 0);
  const int64_t nfull = a.vec ? len / a.sub : 0;
  return nfull + ceil_div(len - nfull * a.sub, (int64_t)a.sub_tail);
}

}  // namespace

// Merge workgroups: enough for every (split tile, 1024-bin chunk) unit when
// all possible split tiles occur (each has two or more slots), at most two
// per CU.
int32_t merge_blocks(const bk::PartArgs& a, int cus) {
  const int64_t chunks = ceil_div((int64_t)1 << a.lay.tile_shift, 1024);
  const int64_t units = (int64_t)(a.max_slots / 2) * chunks;
  return (int32_t)std::min<int64_t>(std::max<int64_t>(units, 0), 2 * (int64_t)cus);
}

void set_part_blocks(bk::PartArgs& a, int scatter_threads, int ppt) {
  a.sub = scatter_threads * ppt;
  a.sub_tail = 4 * scatter_threads;
  // every slice but the last has the first one's length
  auto shape = [&](int64_t w, int32_t& nfull, int32_t& nblocks) {
    const int64_t lo = w * a.chunk;
    const int64_t len = std::max<int64_t>(std::min<int64_t>(lo + a.chunk, a.n) - lo, 0);
    nfull = (int32_t)(a.vec ? len / a.sub : 0);
    nblocks = (int32_t)slice_blocks(a, w);
  };
  shape(0, a.nfull_a, a.nblocks_a);
  shape(a.nwg - 1, a.nfull_z, a.nblocks_z);
  a.nbpw = std::max({a.nblocks_a, a.nblocks_z, 1});
}

void set_part_items(bk::PartArgs& a, int cus) {
  // Slice w of tile t opens item floor(excl(w) / L) of the tile, with excl(w)
  // the tile's records (padding included) in the slices before w and L the
  // split length.  The item numbers of a tile run from 0 to at most
  // m = floor(R_t / L) for a tile of R_t records, so it has at most m + 1
  // items; a split tile (two or more items) has m >= 1 and so at most 2 m.
  // Summed over tiles, with R = all record slots: items <= tiles + R / L,
  // and partial slots (items of split tiles) <= 2 R / L.
  const int64_t q = (int64_t)part_records(a) / (int64_t)a.split_len;
  a.max_items = (int32_t)((int64_t)a.ntiles + q);
  a.max_slots = (int32_t)std::min<int64_t>(a.max_items, 2 * q);
  a.merge_blocks = merge_blocks(a, cus);
}

bool use_quads(int nk, bool attr_f64, int64_t ntiles, int64_t sub) {
  // Whole quads per lane pay off where runs are long (a sub-chunk averages
  // 16 or more records per tile) and a quad carries at most one f32
  // attribute: there the padding is small and the gather's per-record work
  // drops.  With more attributes, or short runs, the padding costs more.
  return nk <= 1 && !attr_f64 && sub >= 16 * ntiles;
}

int32_t part_pad_row(int64_t ntiles, int64_t sub) {
  // each tile's run in a sub-chunk gains at most 3 padding records, and only
  // a tile with a record has a run
  return (int32_t)((3 * std::min<int64_t>(ntiles, sub) + 3) & ~int64_t(3));
}

size_t part_records(const bk::PartArgs& a) {
  return (size_t)std::max<int64_t>(a.n, 0) + (size_t)a.nwg * a.nbpw * (size_t)a.pad_row + 4;
}

size_t set_off_stage(bk::PartArgs& a, size_t stage_base, size_t lds_limit) {
  a.off_stage = (int32_t)align16(stage_base);
  const size_t cols = (size_t)a.ntiles + 1;
  int shift = 0;
  while (shift < 4 && (1 << shift) < a.nbpw &&
         a.off_stage + align16(cols * 2 << (shift + 1)) <= lds_limit)
    ++shift;
  a.off_shift = shift;
  return a.off_stage + align16(cols * 2 << shift);
}

namespace {

// LDS and slot layout of a tile of tb bins.  Returns the LDS bytes.
size_t tile_layout(int tb, int k, bool sum, bool mn, bool mx, int prec, size_t asz, bk::TileLayout* L) {
  std::memset(L, 0, sizeof *L);
  L->tb = tb;
  L->want_sum = sum;
  L->want_min = mn;
  L->want_max = mx;
  const size_t lds_sum = (prec == bk::PREC_PLAIN) ? 4 : 8;
  const size_t slot_sum = (prec == bk::PREC_PLAIN) ? 4 : 8;
  size_t lo = align16(4 * (size_t)tb), so = align16(4 * (size_t)tb);
  for (int j = 0; j < k; ++j) {
    L->lds_sum_off[j] = (int32_t)std::min<size_t>(lo, INT32_MAX);
    L->slot_sum_off[j] = (int32_t)std::min<size_t>(so, INT32_MAX);
    if (sum) {
      lo = align16(lo + lds_sum * tb);
      so = align16(so + slot_sum * tb);
    }
    // With both min and max kept, the LDS holds them interleaved (one
    // 8-byte read per record for both filters); slots keep two arrays.
    L->mm_pair = mn && mx;
    L->lds_min_off[j] = (int32_t)std::min<size_t>(lo, INT32_MAX);
    L->slot_min_off[j] = (int32_t)std::min<size_t>(so, INT32_MAX);
    if (L->mm_pair) {
      L->lds_max_off[j] = (int32_t)std::min<size_t>(lo + asz, INT32_MAX);
      lo = align16(lo + 2 * asz * tb);
      so = align16(so + asz * tb);
    } else if (mn) {
      lo = align16(lo + asz * tb);
      so = align16(so + asz * tb);
    }
    if (!L->mm_pair) L->lds_max_off[j] = (int32_t)std::min<size_t>(lo, INT32_MAX);
    L->slot_max_off[j] = (int32_t)std::min<size_t>(so, INT32_MAX);
    if (mx) {
      if (!L->mm_pair) lo = align16(lo + asz * tb);
      so = align16(so + asz * tb);
    }
  }
  L->slot_bytes = (int64_t)align256(so);
  return lo;
}

void fill_outs(const bin_request& r, int k, bk::Outs* o) {
  std::memset(o, 0, sizeof *o);
  o->cnt = (r.ops & BIN_COUNT) ? r.out.count : nullptr;
  for (int j = 0; j < k; ++j) {
    o->sum[j] = (r.ops & BIN_SUM) ? r.out.sum[j] : nullptr;
    o->mn[j] = (r.ops & BIN_MIN) ? r.out.min[j] : nullptr;
    o->mx[j] = (r.ops & BIN_MAX) ? r.out.max[j] : nullptr;
    o->avg[j] = (r.ops & BIN_AVG) ? r.out.avg[j] : nullptr;
  }
}

}  // namespace

int resolve_precision(uint32_t ops, bool attr_f64) {
  if (attr_f64) return bk::PREC_F64;
  if (ops & BIN_PREC_PLAIN) return bk::PREC_PLAIN;
  if (ops & BIN_PREC_COMP) return bk::PREC_COMP;
  // Default: binary64 accumulation.  On gfx950 an LDS binary64 atomic add is
  // several times faster than the FP32 one, and a global binary64 add is one
  // atomic where TwoSum needs two; the result is at least as accurate as the
  // compensated FP32 sum.
  return bk::PREC_F64;
}

int prepare(const bin_request& r, const DeviceInfo& dev, const PlanHints& hints_in, void* scratch, Prepared* p) {
  const PlanHints hints = effective_hints(r, dev, hints_in);
  std::memset(&p->bin, 0, sizeof p->bin);
  std::memset(&p->init, 0, sizeof p->init);
  std::memset(&p->fin, 0, sizeof p->fin);
  std::memset(&p->lds, 0, sizeof p->lds);
  std::memset(&p->part, 0, sizeof p->part);
  std::memset(&p->pcfg, 0, sizeof p->pcfg);
  std::memset(&p->cfg, 0, sizeof p->cfg);
  const uint32_t ops = r.ops;
  const int k = r.attrs.cols ? r.attrs.ncols : 0;
  const int64_t nb = (int64_t)r.nx * r.ny;
  p->coord_f64 = r.coords.dtype == BIN_F64;
  p->attr_f64 = k > 0 && r.attrs.dtype == BIN_F64;
  p->prec = resolve_precision(ops, p->attr_f64);
  const bool want_cnt = ops & (BIN_COUNT | BIN_AVG);
  const bool want_sum = ops & (BIN_SUM | BIN_AVG);
  const bool want_min = ops & BIN_MIN;
  const bool want_max = ops & BIN_MAX;
  const bool want_avg = ops & BIN_AVG;
  const size_t asz = p->attr_f64 ? 8 : 4;
  const int nk = (want_sum || want_min || want_max) ? k : 0;
  const size_t lds_budget = dev.lds_per_block;
  const int cus = std::max(dev.cus, 1);
  const int64_t n = r.n;
  const bk::Axis ax{r.bounds[0], r.bounds[1], (double)r.nx / (r.bounds[1] - r.bounds[0]), r.nx, 0};
  const bk::Axis ay{r.bounds[2], r.bounds[3], (double)r.ny / (r.bounds[3] - r.bounds[2]), r.ny, 0};

  // --- strategy
  bk::TileLayout whole;
  const size_t whole_lds = nb <= (int64_t)lds_budget
                               ? tile_layout((int)nb, nk, want_sum, want_min, want_max, p->prec, asz, &whole)
                               : SIZE_MAX;
  // Largest power-of-two tile whose accumulators fit LDS.
  int shift = hints.tile_shift ? hints.tile_shift : 15;
  bk::TileLayout tl;
  size_t tile_lds = 0;
  for (; shift >= 6; --shift) {
    tile_lds = tile_layout(1 << shift, nk, want_sum, want_min, want_max, p->prec, asz, &tl);
    if (tile_lds <= lds_budget) break;
  }
  // Smaller tiles while the grid would give fewer than two tiles per CU:
  // the tile binning then runs one item per tile on every CU, each with a
  // smaller LDS footprint, instead of splitting a few tiles into many
  // partial slots that have to be merged.  Grids binned together in one
  // call (hints.share of them) count together.  Not below 256 bins:
  // smaller tiles were measured slower on clustered data (a heavy tile is
  // split into several items anyway, while tiny tiles make short runs and
  // put most records of a window into the same few bins).
  if (!hints.tile_shift)
    while (shift > 8 && ceil_div(nb, (int64_t)1 << shift) * std::max(hints.share, 1) < 2 * (int64_t)cus) --shift;
  tile_lds = tile_layout(1 << std::max(shift, 6), nk, want_sum, want_min, want_max, p->prec, asz, &tl);
  tl.tile_shift = shift;
  const int64_t ntiles = ceil_div(nb, (int64_t)1 << shift);
  int strat;
  if (whole_lds <= lds_budget) strat = bk::STRAT_LDS;
  else if (shift >= 6 && ntiles <= kMaxTiles) strat = bk::STRAT_PART;
  else strat = bk::STRAT_GLOBAL;
  if (hints.force_strategy == bk::STRAT_GLOBAL) strat = bk::STRAT_GLOBAL;
  if (hints.force_strategy == bk::STRAT_LDS && whole_lds <= lds_budget) strat = bk::STRAT_LDS;
  if (hints.force_strategy == bk::STRAT_PART && shift >= 6 && ntiles <= kMaxTiles) strat = bk::STRAT_PART;
  p->cfg.strategy = strat;
  Carve cv{static_cast<unsigned char*>(scratch)};

  if (strat == bk::STRAT_LDS) {
    bk::LdsArgs& a = p->lds;
    a.x = r.coords.cols[r.axes[0]];
    a.y = r.coords.cols[r.axes[1]];
    for (int j = 0; j < nk; ++j) a.attr[j] = r.attrs.cols[j];
    a.ax = ax;
    a.ay = ay;
    a.n = n;
    a.nx = r.nx;
    a.nbins = (int32_t)nb;
    a.k = nk;
    fill_outs(r, nk, &a.out);
    a.lay = whole;
    bk::LaunchCfg& c = p->cfg;
    c.lds_bytes = whole_lds;
    c.block = hints.block ? hints.block : (whole_lds > 40 * 1024 ? 1024 : 512);
    // At most 1024 threads per CU: every workgroup writes a slot of the
    // whole grid that the merge reads back, and on 32²-64² grids with 16M
    // particles fewer, fuller workgroups were measured 21-29% faster overall
    // than two or four per CU.
    const int per_cu = (int)std::max<size_t>(
        1, std::min<size_t>(dev.lds_per_cu / std::max<size_t>(whole_lds, 1), 1024 / c.block));
    // Enough particles per workgroup to amortise writing and merging a slot.
    const int64_t min_chunk = std::max<int64_t>(2 * nb, 16384);
    int64_t grid = std::min<int64_t>(ceil_div(std::max<int64_t>(n, 1), min_chunk), (int64_t)cus * per_cu);
    if (hints.grid) grid = hints.grid;
    grid = std::max<int64_t>(grid, 1);
    a.chunk = ceil_div(ceil_div(std::max<int64_t>(n, 1), grid), 64) * 64;
    c.grid = (int)ceil_div(std::max<int64_t>(n, 1), a.chunk);
    bool aligned = ((uintptr_t)a.x % 16 == 0) && ((uintptr_t)a.y % 16 == 0);
    for (int j = 0; j < nk; ++j) aligned = aligned && ((uintptr_t)a.attr[j] % 16 == 0);
    a.vec = aligned ? 1 : 0;
    a.nslots = c.grid;
    if (a.nslots > 1) a.partial = cv.take((size_t)a.lay.slot_bytes * a.nslots);
    p->scratch_bytes = cv.used;
    return BIN_OK;
  }

  if (strat == bk::STRAT_PART) {
    bk::PartArgs& a = p->part;
    bk::PartCfg& c = p->pcfg;
    a.x = r.coords.cols[r.axes[0]];
    a.y = r.coords.cols[r.axes[1]];
    for (int j = 0; j < nk; ++j) a.attr[j] = r.attrs.cols[j];
    a.ax = ax;
    a.ay = ay;
    a.n = n;
    a.nx = r.nx;
    a.nbins = (int32_t)nb;
    a.k = nk;
    a.ntiles = (int32_t)ntiles;
    fill_outs(r, nk, &a.out);
    a.lay = tl;
    const int T = (int)ntiles;
    int64_t nwg = std::min<int64_t>(ceil_div(std::max<int64_t>(n, 1), 32768), 2 * (int64_t)cus);
    if (hints.grid) nwg = std::min<int64_t>(hints.grid, 65535);
    if (hints.part_wg) nwg = hints.part_wg;
    nwg = std::max<int64_t>(nwg, 1);
    // Slices start at multiples of 64 particles so that aligned columns are
    // read with 16-byte loads.
    a.chunk = ceil_div(ceil_div(std::max<int64_t>(n, 1), nwg), 64) * 64;
    a.nwg = (int32_t)ceil_div(std::max<int64_t>(n, 1), a.chunk);
    bool aligned = ((uintptr_t)a.x % 16 == 0) && ((uintptr_t)a.y % 16 == 0);
    for (int j = 0; j < nk; ++j) aligned = aligned && ((uintptr_t)a.attr[j] % 16 == 0);
    a.vec = aligned ? 1 : 0;
    // Split length.  With at least one tile per CU the tiles alone fill the
    // device: only tiles above twice the average are split.  With fewer
    // tiles, items of about n / (2 CUs) records keep every CU busy.
    int64_t L = ntiles >= cus ? std::max<int64_t>(ceil_div(2 * n, ntiles), ceil_div(n, 2 * (int64_t)cus))
                              : ceil_div(n, 2 * (int64_t)cus);
    L = std::max<int64_t>(L, 16384);
    if (hints.split_len) L = hints.split_len;
    a.split_len = (uint32_t)std::min<int64_t>(L, 0x7FFFFFFF);
    // scatter LDS: 4 T counters, S tile/bin words, S values (one attribute
    // at a time)
    // 1024-thread scatter workgroups measured fastest on MI355X for both the
    // 1- and 4-attribute workloads (one workgroup per CU, LDS-bound).
    // Largest scatter stage that fits LDS: 1024 threads first (fastest on
    // MI355X), fewer particles per thread, then fewer threads (many
    // attributes).  Register budget (no spills): a 1024-thread workgroup
    // allows 128 VGPRs per lane, enough for 16 particles per thread with f32
    // columns, 8 with f64 ones; smaller workgroups take 32 (f32
    // coordinates) or 16 (f64).
    int nt = 0, ppt = 0;
    size_t sc = 0;
    const bool wide = p->coord_f64 || p->attr_f64;
    for (int tnt = hints.scatter_threads ? hints.scatter_threads : 1024; tnt >= 256 && !ppt; tnt /= 2) {
      int cap = tnt >= 1024 ? (wide ? 8 : 16) : (p->coord_f64 ? 16 : 32);
      if (nk >= 2) cap = std::min(cap, 8192 / tnt);  // multi-attribute sub-chunks hold <= 8192
      int tp0 = std::min(hints.scatter_ppt ? hints.scatter_ppt : 16, cap);
      if (tp0 == 12 && tnt != 1024) tp0 = 8;  // 12 per thread exists for 1024 threads only
      for (int tp = tp0; tp >= 4; tp = tp == 12 ? 8 : tp / 2) {
        const size_t S = (size_t)tnt * tp;
        const bool quads = hints.quads ? hints.quads == 2 : use_quads(nk, p->attr_f64, T, (int64_t)S);
        const size_t SP = S + (quads ? part_pad_row(T, (int64_t)S) : 0);  // staged records incl. padding
        const int32_t svo = (int32_t)align16(16 * (size_t)T + 2 * SP);
        // values, then at least one staged row of the run table
        const size_t need = svo + (nk ? SP * asz : 0);
        if (align16(need) + align16(2 * ((size_t)T + 1)) + kScatterStatic <= lds_budget) {
          nt = tnt;
          ppt = tp;
          a.stage_val_off = svo;
          sc = need;
          break;
        }
      }
      if (hints.scatter_threads) break;
    }
    if (!ppt) return fail(BIN_ERR_UNSUPPORTED, "partition scatter stage does not fit LDS");
    c.ppt = ppt;
    c.scatter_threads = nt;
    c.bin_lds = tile_lds;
    // Half-size workgroups when two tiles fit a CU's LDS: two items per CU.
    c.bin_block = 2 * tile_lds <= dev.lds_per_cu ? 512 : 1024;
    set_part_blocks(a, nt, ppt);
    a.quads = (hints.quads ? hints.quads == 2 : use_quads(nk, p->attr_f64, T, (int64_t)nt * ppt)) ? 1 : 0;
    // Each tile's record total, padding included, is counted in 32 bits;
    // with up to 3 padding records per sub-chunk, quads only while n plus
    // that padding stays below 2^32 (without padding the total is <= n).
    if (a.quads && (uint64_t)a.n + 3ull * (uint64_t)a.nwg * (uint64_t)a.nbpw > 0xFFFFFFFFull) a.quads = 0;
    a.pad_row = a.quads ? part_pad_row(T, (int64_t)nt * ppt) : 0;
    c.scatter_lds = set_off_stage(a, sc, lds_budget - kScatterStatic);
    set_part_items(a, cus);
    // scratch
    a.counts = static_cast<uint32_t*>(cv.take(4 * (size_t)ntiles * a.nwg));
    a.blk_off = static_cast<uint16_t*>(cv.take(2 * (size_t)a.nwg * a.nbpw * (size_t)(ntiles + 1)));
    a.ilist = static_cast<uint32_t*>(cv.take(4 * (size_t)ntiles * a.nwg));
    a.items = static_cast<uint32_t*>(cv.take(12 * (size_t)a.max_items));
    a.n_items = static_cast<uint32_t*>(cv.take(4));
    a.tile_items = static_cast<uint32_t*>(cv.take(12 * (size_t)T));
    a.split_list = static_cast<uint32_t*>(cv.take(4 * ((size_t)T + 1)));
    a.rec_bin = static_cast<uint16_t*>(cv.take(2 * part_records(a)));
    for (int j = 0; j < nk; ++j) a.rec_val[j] = cv.take(asz * part_records(a));
    a.partial = a.max_slots > 0 ? cv.take((size_t)a.lay.slot_bytes * a.max_slots) : nullptr;
    p->scratch_bytes = cv.used;
    p->cfg.grid = a.max_items;
    p->cfg.block = c.bin_block;
    return BIN_OK;
  }

  // --- global-atomic strategy
  uint32_t* cnt = nullptr;
  if (want_cnt) cnt = (ops & BIN_COUNT) ? r.out.count : static_cast<uint32_t*>(cv.take(4 * nb));
  const bool comp_global = p->prec == bk::PREC_COMP;
  bk::BinArgs& a = p->bin;
  a.x = r.coords.cols[r.axes[0]];
  a.y = r.coords.cols[r.axes[1]];
  a.cnt = cnt;
  a.n = n;
  a.nx = r.nx;
  a.nbins = (int32_t)nb;
  a.k = nk;
  a.ax = ax;
  a.ay = ay;
  bk::FinArgs& f = p->fin;
  f.cnt = cnt;
  f.nbins = nb;
  f.k = want_avg || comp_global ? nk : 0;
  p->need_finalize = false;
  for (int j = 0; j < nk; ++j) {
    a.attr[j] = r.attrs.cols[j];
    bk::AccPtrs& acc = a.acc[j];
    acc.minmax_f64 = p->attr_f64;
    acc.mn = want_min ? r.out.min[j] : nullptr;
    acc.mx = want_max ? r.out.max[j] : nullptr;
    bk::FinAttr& fa = f.attr[j];
    fa.avg_out = want_avg ? r.out.avg[j] : nullptr;
    fa.avg_f64 = p->prec != bk::PREC_PLAIN;
    if (want_sum) {
      if (comp_global) {
        acc.sum = cv.take(4 * nb);
        acc.comp = static_cast<float*>(cv.take(4 * nb));
        acc.sum_is_f64 = 0;
        fa.src = acc.sum;
        fa.comp = acc.comp;
        fa.src_kind = bk::SRC_F32_COMP;
        fa.sum_out = (ops & BIN_SUM) ? r.out.sum[j] : nullptr;
        p->need_finalize = true;
      } else {
        const bool f64 = p->prec != bk::PREC_PLAIN;
        acc.sum = (ops & BIN_SUM) ? r.out.sum[j] : cv.take((f64 ? 8 : 4) * nb);
        acc.sum_is_f64 = f64;
        fa.src = acc.sum;
        fa.src_kind = f64 ? bk::SRC_F64 : bk::SRC_F32;
      }
    }
    if (want_avg) p->need_finalize = true;
  }
  p->scratch_bytes = cv.used;
  bk::InitArgs& in = p->init;
  in.cnt = cnt;
  in.nbins = nb;
  in.k = nk;
  for (int j = 0; j < nk; ++j) in.acc[j] = a.acc[j];
  p->init_grid = (int)std::max<int64_t>(1, std::min<int64_t>(ceil_div(nb, 256), (int64_t)cus * 8));
  p->fin_grid = p->init_grid;
  bk::LaunchCfg& c = p->cfg;
  c.block = hints.block ? hints.block : 256;
  int64_t grid = std::min<int64_t>(ceil_div(std::max<int64_t>(n, 1), (int64_t)c.block * 4), (int64_t)cus * 16);
  if (hints.grid) grid = hints.grid;
  c.grid = (int)std::max<int64_t>(grid, 1);
  return BIN_OK;
}

int enqueue(const Prepared& p, hipStream_t s, bk::KTimer* tm) {
  hipError_t e = hipSuccess;
  switch (p.cfg.strategy) {
    case bk::STRAT_LDS:
      e = bk::launch_bin_lds(p.lds, p.coord_f64, p.attr_f64, p.prec, p.cfg, s, tm);
      if (e != hipSuccess) return hip_fail(e, "launch LDS binning kernels");
      return BIN_OK;
    case bk::STRAT_PART:
      e = bk::launch_partition(p.part, p.coord_f64, p.attr_f64, p.prec, p.pcfg, s, tm);
      if (e != hipSuccess) return hip_fail(e, "launch partition binning kernels");
      return BIN_OK;
    default:
      break;
  }
  e = bk::launch_init(p.init, p.init_grid, s, tm);
  if (e != hipSuccess) return hip_fail(e, "launch bin_init_kernel");
  if (p.bin.n > 0) {
    e = bk::launch_bin_global(p.bin, p.coord_f64, p.attr_f64, p.prec, p.cfg, s, tm);
    if (e != hipSuccess) return hip_fail(e, "launch bin_global_kernel");
  }
  if (p.need_finalize) {
    e = bk::launch_finalize(p.fin, p.fin_grid, s, tm);
    if (e != hipSuccess) return hip_fail(e, "launch bin_finalize_kernel");
  }
  return BIN_OK;
}

std::string describe(const Prepared& p) {
  char buf[320];
  const char* prec = p.prec == bk::PREC_PLAIN ? "fp32" : p.prec == bk::PREC_F64 ? "fp64" : "fp32-comp";
  switch (p.cfg.strategy) {
    case bk::STRAT_LDS:
      snprintf(buf, sizeof buf, "lds grid=%d block=%d lds=%zu chunk=%lld vec=%d prec=%s", p.cfg.grid,
               p.cfg.block, p.cfg.lds_bytes, (long long)p.lds.chunk, p.lds.vec, prec);
      break;
    case bk::STRAT_PART:
      snprintf(buf, sizeof buf,
               "partition tiles=%d tile_bins=%d wg=%d chunk=%lld threads=%d ppt=%d sub=%d blocks=%d staged_rows=%d quads=%d split=%u "
               "max_items=%d "
               "scatter_lds=%zu bin_lds=%zu vec=%d prec=%s",
               p.part.ntiles, 1 << p.part.lay.tile_shift, p.part.nwg, (long long)p.part.chunk, p.pcfg.scatter_threads,
               p.pcfg.ppt, p.part.sub, p.part.nbpw, 1 << p.part.off_shift, p.part.quads,
               p.part.split_len, p.part.max_items, p.pcfg.scatter_lds, p.pcfg.bin_lds, p.part.vec, prec);
      break;
    default:
      snprintf(buf, sizeof buf, "global grid=%d block=%d prec=%s", p.cfg.grid, p.cfg.block, prec);
  }
  return buf;
}

}  // namespace binimpl
