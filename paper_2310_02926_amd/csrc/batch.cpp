// Batched binning: many independent requests of uneven size run as a few
// launches instead of a launch sequence per request.  Also the HIP-graph
// capture of a batch, and the fused multi-grid path (several grids over
// one table).
//
// Requests are planned one by one - under the batch policy bin_autotune
// chose: each request's tuned plan, the planner's rules, or the rules with
// one shared scatter shape - then grouped by (strategy, coordinate type,
// attribute type, precision) and, for tile partitions, by the scatter shape
// and gather form their plans chose.  Every request keeps its own
// scratch (records, run table, counts, items, partial slots); the groups
// share device tables of descriptors and block maps, uploaded once, and
// each group runs one table-driven launch per stage for all its requests
// (the binning stage as up to four launches, by the LDS of each request's
// tile or grid).  Requests that need the global-atomic strategy run one by
// one.
#include <algorithm>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <optional>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "batch_classes.h"
#include "internal.h"

namespace binimpl {

namespace {

size_t al256(size_t v) { return (v + 255) & ~size_t(255); }
size_t al16(size_t v) { return (v + 15) & ~size_t(15); }
int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

struct PartGroup {
  bool cf64 = false, af64 = false;
  int prec = 0;
  int nt = 1024, ppt = 8;  // scatter shape shared by the group
  bool quads = false;      // runs padded to quads, gathered a quad per lane
  std::vector<int> idx;              // request indices
  std::vector<bk::PartArgs> args;    // patched records
  bk::PartCfg cfg{};
  bk::PartBatch b{};
  size_t desc_off = 0, map_wg_off = 0, map_walk_off = 0, map_item_off = 0, map_tile_off = 0;
  std::vector<uint32_t> map_wg, map_walk, map_item, map_tile;
};

struct LdsGroup {
  bool cf64 = false, af64 = false;
  int prec = 0;
  std::vector<int> idx;
  std::vector<bk::LdsArgs> args;
  bk::LdsBatch b{};
  size_t desc_off = 0, map_slot_off = 0, map_merge_off = 0;
  std::vector<uint32_t> map_slot, map_merge;
};

}  // namespace

struct BatchPlan {
  std::vector<Prepared> preps;
  std::vector<PartGroup> part;
  std::vector<LdsGroup> lds;
  std::vector<int> global_reqs;
  size_t scratch_bytes = 0;  // device scratch, tables included
  size_t tables_off = 0, tables_bytes = 0;
  std::vector<unsigned char> tables;  // host image of the device tables
};

namespace {

// Pass 1 (base == nullptr) sizes everything; pass 2 lays out pointers.
int plan_batch(const bin_request* reqs, int nreq, const DeviceInfo& dev, const PlanHints& hints,
               unsigned char* base, BatchPlan* bp) {
  bp->preps.assign(nreq, Prepared{});
  bp->part.clear();
  bp->lds.clear();
  bp->global_reqs.clear();
  // Groups: strategy and types, and for tile partitions the scatter shape
  // and gather form each request's own plan chose (one launch serves one
  // shape; requests of different shapes go to different groups rather than
  // all taking the smallest shape).
  std::map<std::tuple<int, int, int, int, int, int, int>, int> gmap;
  // Without an explicit override the batch policy chosen by bin_autotune
  // applies: each request's tuned plan, the planner's rules, or the rules
  // with one shared scatter shape.
  PlanHints bh = hints;
  std::optional<TunedLookupOff> rules_only;
  if (hints_are_default(hints)) {
    const BatchPolicy pol = batch_policy(dev);
    if (pol.mode != 1) rules_only.emplace();
    if (pol.mode == 2) {
      bh.scatter_threads = pol.nt;
      bh.scatter_ppt = pol.ppt;
    }
  }
  for (int i = 0; i < nreq; ++i) {
    Prepared& p = bp->preps[i];
    int st = prepare(reqs[i], dev, bh, nullptr, &p);
    if (st == BIN_ERR_UNSUPPORTED && !hints_are_default(bh) && hints_are_default(hints)) {
      clear_error();
      st = prepare(reqs[i], dev, hints, nullptr, &p);  // the shared shape does not fit this request
    }
    if (st) return st;
    const int strat = p.cfg.strategy;
    if (strat == bk::STRAT_GLOBAL) {
      bp->global_reqs.push_back(i);
      continue;
    }
    int nt = 0, ppt = 0, quads = 0;
    if (strat == bk::STRAT_PART) {
      nt = p.pcfg.scatter_threads;
      ppt = p.pcfg.ppt;
      // The table-driven scatter needs a few more registers than the single
      // one: at most 8 particles per thread at 1024 threads.
      if (nt >= 1024) ppt = std::min(ppt, 8);
      bk::PartArgs a = p.part;
      set_part_blocks(a, nt, ppt);
      quads = (p.part.quads && use_quads(a.k, p.attr_f64, a.ntiles, (int64_t)nt * ppt) &&
               (uint64_t)a.n + 3ull * (uint64_t)a.nwg * (uint64_t)a.nbpw <= 0xFFFFFFFFull)
                  ? 1
                  : 0;
    }
    auto key = std::make_tuple(strat, (int)p.coord_f64, (int)p.attr_f64, p.prec, nt, ppt, quads);
    auto it = gmap.find(key);
    if (it == gmap.end()) {
      if (strat == bk::STRAT_PART) {
        PartGroup g;
        g.cf64 = p.coord_f64;
        g.af64 = p.attr_f64;
        g.prec = p.prec;
        g.nt = nt;
        g.ppt = ppt;
        g.quads = quads != 0;
        bp->part.push_back(g);
        it = gmap.emplace(key, (int)bp->part.size() - 1).first;
      } else {
        LdsGroup g;
        g.cf64 = p.coord_f64;
        g.af64 = p.attr_f64;
        g.prec = p.prec;
        bp->lds.push_back(g);
        it = gmap.emplace(key, (int)bp->lds.size() - 1).first;
      }
    }
    if (strat == bk::STRAT_PART) bp->part[it->second].idx.push_back(i);
    else bp->lds[it->second].idx.push_back(i);
  }

  size_t off = 0;
  auto take = [&](size_t bytes) {
    unsigned char* p = base ? base + off : nullptr;
    off += al256(std::max<size_t>(bytes, 1));
    return p;
  };
  // --- partition groups
  for (auto& g : bp->part) {
    const int R = (int)g.idx.size();
    if (R > 65535) return fail(BIN_ERR_UNSUPPORTED, "a batch group holds at most 65535 requests");
    g.args.resize(R);
    // The group's scatter shape; staged values sized for the largest request.
    const int ppt = g.ppt, nt = g.nt;
    size_t asz = g.af64 ? 8 : 4;
    const size_t S = (size_t)nt * ppt;
    // Per request: tile counters, record stage (with quad padding) and
    // values, then its staged rows of the run table; the launch takes the
    // largest.
    size_t scatter_lds = 16;
    for (int r = 0; r < R; ++r) {
      bk::PartArgs a = bp->preps[g.idx[r]].part;
      set_part_blocks(a, nt, ppt);
      const size_t SP = S + (g.quads ? part_pad_row(a.ntiles, (int64_t)S) : 0);
      const size_t sv = al16(16 * (size_t)a.ntiles + 2 * SP);
      scatter_lds = std::max(scatter_lds, set_off_stage(a, sv + (a.k ? SP * asz : 0), dev.lds_per_block - 256));
    }
    g.cfg.ppt = ppt;
    g.cfg.scatter_threads = nt;
    g.cfg.quads = g.quads ? 1 : 0;
    g.cfg.scatter_lds = scatter_lds;
    if (scatter_lds + 256 > dev.lds_per_block)
      return fail(BIN_ERR_UNSUPPORTED, "batched scatter stage does not fit LDS");
    // Per-request scratch: tile totals, sub-chunk run tables, records,
    // items and partial slots.
    uint32_t* n_items = reinterpret_cast<uint32_t*>(take(4 * (size_t)R));
    for (int r = 0; r < R; ++r) {
      bk::PartArgs a = bp->preps[g.idx[r]].part;
      set_part_blocks(a, nt, ppt);
      a.quads = g.quads ? 1 : 0;
      a.pad_row = g.quads ? part_pad_row(a.ntiles, (int64_t)S) : 0;
      const size_t SP = S + a.pad_row;
      const size_t nrec = part_records(a);
      a.stage_val_off = (int32_t)al16(16 * (size_t)a.ntiles + 2 * SP);
      set_off_stage(a, a.stage_val_off + (a.k ? SP * asz : 0), dev.lds_per_block - 256);
      set_part_items(a, dev.cus);
      a.counts = reinterpret_cast<uint32_t*>(take(4 * (size_t)a.ntiles * a.nwg));
      a.blk_off = reinterpret_cast<uint16_t*>(take(2 * (size_t)a.nwg * a.nbpw * (size_t)(a.ntiles + 1)));
      a.ilist = reinterpret_cast<uint32_t*>(take(4 * (size_t)a.ntiles * a.nwg));
      a.items = reinterpret_cast<uint32_t*>(take(12 * (size_t)a.max_items));
      a.n_items = n_items ? n_items + r : nullptr;
      a.tile_items = reinterpret_cast<uint32_t*>(take(12 * (size_t)a.ntiles));
      a.split_list = reinterpret_cast<uint32_t*>(take(4 * ((size_t)a.ntiles + 1)));
      a.rec_bin = reinterpret_cast<uint16_t*>(take(2 * nrec));
      for (int j = 0; j < a.k; ++j) a.rec_val[j] = take(asz * nrec);
      a.partial = a.max_slots > 0 ? take((size_t)a.lay.slot_bytes * a.max_slots) : nullptr;
      // The requests share the merge launch: at most 16 workgroups each, or
      // two per CU over the group when it has few requests (the grids of a
      // multi-grid call: nine 256-square planes merge in 0.24 ms instead of
      // 0.52 ms with 16 each).
      a.merge_blocks = std::min(a.merge_blocks, std::max(16, 2 * dev.cus / R));
      g.args[r] = a;
    }
    g.b.nreq = R;
    g.map_wg.clear();
    g.map_walk.clear();
    g.map_item.clear();
    g.map_tile.clear();
    // Tile-binning classes by the LDS of each request's tile: an eighth of
    // a CU's LDS or less runs in 128-thread workgroups (eight per CU), a
    // quarter or less in 256-thread ones (four per CU), half or less in
    // 512-thread ones (two per CU), larger tiles in 1024-thread ones.  Every
    // CU then holds 16 waves either way, but small tiles have several work
    // items in flight per CU, so one item's chain of dependent loads (its
    // item record, its run table, its first records) and its result stores
    // overlap another's binning: on batches of many small requests an
    // item's fixed cost is several times its per-record cost.
    std::vector<uint32_t> cls_items[4];
    size_t cls_lds[4] = {0, 0, 0, 0};
    for (int r = 0; r < R; ++r) {
      const bk::PartArgs& a = g.args[r];
      for (int w = 0; w < a.nwg; ++w) g.map_wg.push_back(((uint32_t)r << 16) | (uint32_t)w);
      for (int b = 0; b < (a.ntiles + 15) / 16; ++b) g.map_walk.push_back(((uint32_t)r << 16) | (uint32_t)b);
      const size_t tl = bp->preps[g.idx[r]].pcfg.bin_lds;
      static const int kTileShares[3] = {8, 4, 2};
      const int q = lds_class(tl, dev.lds_per_cu, kTileShares, 3);
      cls_lds[q] = std::max(cls_lds[q], tl);
      for (int i = 0; i < a.max_items; ++i) cls_items[q].push_back(((uint32_t)r << 16) | (uint32_t)i);
      for (int b = 0; b < a.merge_blocks; ++b) g.map_tile.push_back(((uint32_t)r << 16) | (uint32_t)b);
      if (a.nwg > 65536 || a.max_items > 65536 || a.ntiles > 65536)
        return fail(BIN_ERR_UNSUPPORTED, "request too large for a batch block map");
    }
    // Workgroups go to the 8 XCDs round-robin.  The tile-binning blocks are
    // reordered so that each XCD takes runs of C = 8 consecutive items (the
    // items of neighbouring tiles, whose runs share cache lines, read
    // through one L2), the runs dealt round-robin so that every XCD gets a
    // share of every request; 0xFFFFFFFF pads to a whole round.  (Runs of
    // 8 beat 1, 4 and 32 on the 256-request batch and the nine-plane
    // multi-grid call.)
    merge_small_classes(cls_items, cls_lds, 4, (size_t)dev.cus);
    for (int q = 0; q < 4; ++q) {
      const size_t C = 8, round = 8 * C;
      const std::vector<uint32_t>& it = cls_items[q];
      const size_t nat = it.size(), npad = (nat + round - 1) / round * round;
      g.b.cls_first[q] = (int32_t)g.map_item.size();
      g.b.cls_block[q] = 128 << q;
      g.b.cls_lds[q] = (int32_t)cls_lds[q];
      for (size_t b = 0; b < npad; ++b) {
        const size_t i = b / round * round + (b % 8) * C + (b / 8) % C;
        g.map_item.push_back(i < nat ? it[i] : 0xFFFFFFFFu);
      }
    }
    g.b.cls_first[4] = (int32_t)g.map_item.size();
    g.b.n_wg_blocks = (int32_t)g.map_wg.size();
    g.b.n_walk_blocks = (int32_t)g.map_walk.size();
    g.b.n_item_blocks = (int32_t)g.map_item.size();
    g.b.n_tile_blocks = (int32_t)g.map_tile.size();
  }
  // --- LDS groups
  for (auto& g : bp->lds) {
    const int R = (int)g.idx.size();
    if (R > 65535) return fail(BIN_ERR_UNSUPPORTED, "a batch group holds at most 65535 requests");
    g.args.resize(R);
    g.map_slot.clear();
    g.map_merge.clear();
    // Classes by the LDS of each request's grid, as for the tile binning: a
    // quarter of a CU's LDS or less in 512-thread workgroups (four per CU;
    // the kernel's registers allow 32 waves), half or less and larger ones
    // in 1024-thread workgroups (two or one per CU).  A large grid no
    // longer holds every small request of the batch to one workgroup per CU.
    std::vector<uint32_t> cls_slots[3];
    size_t cls_lds[3] = {0, 0, 0};
    // Slices twice as long as each request's own plan when the group's
    // slices would still fill the device twice over: those plans size them
    // to fill the device alone, while a large batch shares it.  Half the
    // partial slots to write and merge; on the 256-request batch the merge
    // went from 0.16 to 0.07 ms, and four times as long made the binning's
    // tail cost more than the merge saved.  A small batch (a few requests
    // the server gathered) keeps its requests' own slices and parallelism.
    int64_t group_slots = 0;
    for (int r = 0; r < R; ++r) group_slots += bp->preps[g.idx[r]].lds.nslots;
    const bool longer = group_slots >= 4 * (int64_t)dev.cus;
    for (int r = 0; r < R; ++r) {
      const Prepared& p = bp->preps[g.idx[r]];
      bk::LdsArgs a = p.lds;
      if (longer && a.nslots > 1) {
        a.chunk = (a.chunk * 2 + 63) / 64 * 64;
        a.nslots = (int32_t)cdiv(std::max<int64_t>(a.n, 1), a.chunk);
      }
      a.partial = a.nslots > 1 ? take((size_t)a.lay.slot_bytes * a.nslots) : nullptr;
      g.args[r] = a;
      const size_t gl = p.cfg.lds_bytes;
      static const int kGridShares[2] = {4, 2};
      const int q = lds_class(gl, dev.lds_per_cu, kGridShares, 2);
      cls_lds[q] = std::max(cls_lds[q], gl);
      for (int s = 0; s < a.nslots; ++s) cls_slots[q].push_back(((uint32_t)r << 16) | (uint32_t)s);
      if (a.nslots > 1)
        for (int64_t c = 0; c < cdiv(a.nbins, 64); ++c) g.map_merge.push_back(((uint32_t)r << 16) | (uint32_t)c);
    }
    merge_small_classes(cls_slots, cls_lds, 3, (size_t)dev.cus);
    for (int q = 0; q < 3; ++q) {
      g.b.cls_first[q] = (int32_t)g.map_slot.size();
      g.b.cls_block[q] = q == 0 ? 512 : 1024;
      g.b.cls_lds[q] = (int32_t)cls_lds[q];
      g.map_slot.insert(g.map_slot.end(), cls_slots[q].begin(), cls_slots[q].end());
    }
    g.b.cls_first[3] = (int32_t)g.map_slot.size();
    g.b.nreq = R;
    g.b.n_slot_blocks = (int32_t)g.map_slot.size();
    g.b.n_merge_blocks = (int32_t)g.map_merge.size();
  }
  // --- tables: descriptors and maps, one upload
  size_t t = 0;
  auto tab = [&](size_t bytes) {
    const size_t o = t;
    t += al256(std::max<size_t>(bytes, 1));
    return o;
  };
  for (auto& g : bp->part) {
    g.desc_off = tab(sizeof(bk::PartArgs) * g.args.size());
    g.map_wg_off = tab(4 * g.map_wg.size());
    g.map_walk_off = tab(4 * g.map_walk.size());
    g.map_item_off = tab(4 * g.map_item.size());
    g.map_tile_off = tab(4 * g.map_tile.size());
  }
  for (auto& g : bp->lds) {
    g.desc_off = tab(sizeof(bk::LdsArgs) * g.args.size());
    g.map_slot_off = tab(4 * g.map_slot.size());
    g.map_merge_off = tab(4 * g.map_merge.size());
  }
  bp->tables_bytes = t;
  bp->tables_off = off;
  unsigned char* tdev = take(t);
  bp->scratch_bytes = off;
  if (!base) return BIN_OK;
  bp->tables.assign(t, 0);
  unsigned char* h = bp->tables.data();
  for (auto& g : bp->part) {
    std::memcpy(h + g.desc_off, g.args.data(), sizeof(bk::PartArgs) * g.args.size());
    std::memcpy(h + g.map_wg_off, g.map_wg.data(), 4 * g.map_wg.size());
    std::memcpy(h + g.map_walk_off, g.map_walk.data(), 4 * g.map_walk.size());
    std::memcpy(h + g.map_item_off, g.map_item.data(), 4 * g.map_item.size());
    std::memcpy(h + g.map_tile_off, g.map_tile.data(), 4 * g.map_tile.size());
    g.b.descs = reinterpret_cast<const bk::PartArgs*>(tdev + g.desc_off);
    g.b.map_wg = reinterpret_cast<const uint32_t*>(tdev + g.map_wg_off);
    g.b.map_walk = reinterpret_cast<const uint32_t*>(tdev + g.map_walk_off);
    g.b.map_item = reinterpret_cast<const uint32_t*>(tdev + g.map_item_off);
    g.b.map_tile = reinterpret_cast<const uint32_t*>(tdev + g.map_tile_off);
  }
  for (auto& g : bp->lds) {
    std::memcpy(h + g.desc_off, g.args.data(), sizeof(bk::LdsArgs) * g.args.size());
    std::memcpy(h + g.map_slot_off, g.map_slot.data(), 4 * g.map_slot.size());
    std::memcpy(h + g.map_merge_off, g.map_merge.data(), 4 * g.map_merge.size());
    g.b.descs = reinterpret_cast<const bk::LdsArgs*>(tdev + g.desc_off);
    g.b.map_slot = reinterpret_cast<const uint32_t*>(tdev + g.map_slot_off);
    g.b.map_merge = reinterpret_cast<const uint32_t*>(tdev + g.map_merge_off);
  }
  return BIN_OK;
}

// Kernel launches of a laid-out batch (tables already on the device).
int launch_batch(const BatchPlan& bp, hipStream_t s, bk::KTimer* tm) {
  for (const auto& g : bp.part) {
    hipError_t e = bk::launch_partition_batch(g.b, g.cf64, g.af64, g.prec, g.cfg, s, tm);
    if (e != hipSuccess) return hip_fail(e, "launch batched partition kernels");
  }
  for (const auto& g : bp.lds) {
    hipError_t e = bk::launch_lds_batch(g.b, g.cf64, g.af64, g.prec, s, tm);
    if (e != hipSuccess) return hip_fail(e, "launch batched LDS kernels");
  }
  return BIN_OK;
}

int validate_requests(const bin_request* reqs, int nreq) {
  if (!reqs && nreq > 0) return fail(BIN_ERR_INVALID_ARG, "reqs is NULL");
  if (nreq < 0) return fail(BIN_ERR_INVALID_ARG, "nreq < 0");
  for (int i = 0; i < nreq; ++i) {
    const bin_request& r = reqs[i];
    int st = validate(&r.coords, &r.attrs, r.n, r.axes, r.bounds, r.nx, r.ny, r.ops, &r.out, false);
    if (st) {
      std::string msg = last_error();
      return fail(st, "request %d: %s", i, msg.c_str());
    }
  }
  return BIN_OK;
}

// Pinned staging for table uploads: per stream a small ring of buffers,
// each with an event that marks when its last upload has been consumed.  A
// call takes a buffer whose upload is done (adding one while the ring has
// fewer than kStageRing), so it does not wait for the stream; only with
// every buffer of a full ring still in flight does it wait for the oldest.
// The global lock only finds the stream's ring; each ring has its own lock,
// so calls on different streams do not wait for each other.
constexpr size_t kStageRing = 4;
struct StageBuf {
  void* host = nullptr;
  size_t bytes = 0;
  hipEvent_t done = nullptr;
};
struct StreamStage {
  std::mutex mu;
  std::vector<StageBuf> ring;
  size_t next = 0;  // the oldest upload when the ring is full
};
std::mutex g_stage_mu;
std::unordered_map<void*, std::unique_ptr<StreamStage>> g_stages;

int upload_tables(const BatchPlan& bp, unsigned char* scratch, hipStream_t s) {
  if (bp.tables_bytes == 0) return BIN_OK;
  StreamStage* ss;
  {
    std::lock_guard<std::mutex> lk(g_stage_mu);
    auto& p = g_stages[(void*)s];
    if (!p) p = std::make_unique<StreamStage>();
    ss = p.get();
  }
  std::lock_guard<std::mutex> lk(ss->mu);
  hipError_t e;
  size_t pick = ss->ring.size();
  for (size_t i = 0; i < ss->ring.size(); ++i)
    if (hipEventQuery(ss->ring[i].done) == hipSuccess) {
      pick = i;
      if (ss->ring[i].bytes >= bp.tables_bytes) break;
    }
  if (pick == ss->ring.size()) {
    if (ss->ring.size() < kStageRing) {
      StageBuf b;
      e = hipEventCreateWithFlags(&b.done, hipEventDisableTiming);
      if (e != hipSuccess) return hip_fail(e, "hipEventCreate(staging)");
      ss->ring.push_back(b);
    } else {
      pick = ss->next;
      ss->next = (ss->next + 1) % kStageRing;
      e = hipEventSynchronize(ss->ring[pick].done);  // every buffer still feeds an upload
      if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize(staging)");
    }
  }
  StageBuf& st = ss->ring[pick];
  if (st.bytes < bp.tables_bytes) {  // its last upload is done: safe to replace
    if (st.host) (void)hipHostFree(st.host);
    st.host = nullptr;
    st.bytes = 0;
    e = hipHostMalloc(&st.host, bp.tables_bytes, hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(e, "hipHostMalloc(staging)");
    st.bytes = bp.tables_bytes;
  }
  std::memcpy(st.host, bp.tables.data(), bp.tables_bytes);
  e = hipMemcpyAsync(scratch + bp.tables_off, st.host, bp.tables_bytes, hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(batch tables)");
  e = hipEventRecord(st.done, s);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord(staging)");
  return BIN_OK;
}

// Several grids over one table in one pass over the table: every grid is a
// tile-partition request with the same slices and sub-chunks of 2048
// particles (512 threads x 4); one fused scatter stages the union of the
// columns per sub-chunk in LDS and writes every grid's records, then the
// rest of the batch's stages run as usual.  The requests qualify with f32
// columns, 2..kMultiGrids grids, all on the partition strategy, at most
// kMultiCols distinct columns, and an LDS stage that fits.

// The fused path's plan: tile partition, 512 threads of 4 particles per
// scatter sub-chunk, record-by-record gather (one launch serves every grid),
// tiles sized for the ngrids grids together.
PlanHints multi_hints(int ngrids) {
  PlanHints h;
  h.force_strategy = bk::STRAT_PART;
  h.scatter_threads = 512;
  h.scatter_ppt = 4;
  h.quads = 1;
  h.share = ngrids;
  return h;
}

struct MultiPlan {
  BatchPlan bp;
  bk::MultiScatterArgs m;
  size_t lds = 0;    // dynamic LDS of the fused scatter
  size_t extra = 0;  // bytes of its arguments, after the batch's tables
  std::vector<int> shifts;  // staged run-table rows per grid (log2)
  size_t scratch_bytes() const { return bp.scratch_bytes + extra; }
};

// Sizing pass.  Returns false when the requests do not qualify (*status
// BIN_OK) or on an error (*status set).
bool multi_plan(const bin_request* reqs, int nreq, const DeviceInfo& dev, MultiPlan* mp, int* status) {
  *status = BIN_OK;
  if (nreq < 2 || nreq > bk::kMultiGrids) return false;
  const bin_request& r0 = reqs[0];
  const int k = r0.attrs.cols ? r0.attrs.ncols : 0;
  if (r0.coords.dtype != BIN_F32 || (k && r0.attrs.dtype != BIN_F32) || r0.n < 1) return false;
  // union of the columns: each grid's axes, then the shared attributes
  std::vector<const void*> cols;
  auto col_index = [&](const void* p) {
    for (size_t u = 0; u < cols.size(); ++u)
      if (cols[u] == p) return (int)u;
    cols.push_back(p);
    return (int)cols.size() - 1;
  };
  bk::MultiScatterArgs& m = mp->m;
  std::memset(&m, 0, sizeof m);
  for (int g = 0; g < nreq; ++g) {
    const bin_request& r = reqs[g];
    if (r.n != r0.n || r.coords.cols != r0.coords.cols || r.attrs.cols != r0.attrs.cols) return false;
    m.gx[g] = col_index(r.coords.cols[r.axes[0]]);
    m.gy[g] = col_index(r.coords.cols[r.axes[1]]);
  }
  for (int j = 0; j < k; ++j) m.attr_col[j] = col_index(r0.attrs.cols[j]);
  if ((int)cols.size() > bk::kMultiCols) return false;
  BatchPlan& bp = mp->bp;
  const int st = plan_batch(reqs, nreq, dev, multi_hints(nreq), nullptr, &bp);
  if (st || bp.part.size() != 1 || !bp.lds.empty() || !bp.global_reqs.empty() ||
      (int)bp.part[0].idx.size() != nreq || bp.part[0].nt != 512 || bp.part[0].ppt != 4 || bp.part[0].quads) {
    clear_error();
    return false;  // (the record stages hold kMultiSub records: no quad padding)
  }
  // LDS: staged columns, per grid its counters and staged run-table rows,
  // the record stages of a group of grids; the largest group, then the most
  // staged rows (a power of two <= 16), that fit.
  const int S = bk::kMultiSub;
  static_assert(bk::kMultiSub == 512 * 4, "the plan's sub-chunk is 512 threads of 4 particles");
  const PartGroup& g0 = bp.part[0];
  const size_t limit = dev.lds_per_block - 256;
  for (int G = bk::kMultiGroup; G >= 1; --G) {
    for (int F = 16; F >= 1; F /= 2) {
      std::vector<int> shifts;
      size_t o = al16((size_t)cols.size() * S * 4);
      for (int g = 0; g < nreq; ++g) {
        const bk::PartArgs& a = g0.args[g];
        m.grid_lds[g] = (int32_t)o;
        o = al16(o + 16 * (size_t)a.ntiles);
        m.grid_ost[g] = (int32_t)o;
        const int f = std::min(F, std::max(1, (int)a.nbpw));
        int sh = 0;
        while ((1 << (sh + 1)) <= f) ++sh;
        shifts.push_back(sh);
        o = al16(o + ((2 * ((size_t)a.ntiles + 1)) << sh));
      }
      m.stage = (int32_t)o;
      o = al16(o + (size_t)G * 4 * S);
      if (o > limit) continue;
      m.group = std::min(G, nreq);
      m.ncols = (int32_t)cols.size();
      m.ngrids = nreq;
      m.k = k;
      m.cols_lds = 0;
      bool vec = true;
      for (size_t u = 0; u < cols.size(); ++u) {
        m.cols[u] = static_cast<const float*>(cols[u]);
        vec = vec && reinterpret_cast<uintptr_t>(cols[u]) % 16 == 0;
      }
      m.vec = vec ? 1 : 0;
      mp->shifts = shifts;
      mp->lds = o;
      mp->extra = al256(sizeof m);
      return true;
    }
  }
  return false;
}

// Layout pass in 'scratch' (MultiPlan::scratch_bytes() bytes): the batch's
// pointers and its tables image, the fused scatter's arguments appended.
// *dm is their device address.
int multi_layout(const bin_request* reqs, int nreq, const DeviceInfo& dev, unsigned char* scratch, MultiPlan* mp,
                 const bk::MultiScatterArgs** dm) {
  BatchPlan& bp = mp->bp;
  const int st = plan_batch(reqs, nreq, dev, multi_hints(nreq), scratch, &bp);
  if (st) return st;
  PartGroup& g = bp.part[0];
  for (int i = 0; i < nreq; ++i) g.args[i].off_shift = mp->shifts[i];
  std::memcpy(bp.tables.data() + g.desc_off, g.args.data(), sizeof(bk::PartArgs) * g.args.size());
  mp->m.grids = g.b.descs;
  const size_t moff = bp.tables.size();
  bp.tables.resize(moff + mp->extra, 0);
  std::memcpy(bp.tables.data() + moff, &mp->m, sizeof mp->m);
  bp.tables_bytes = bp.tables.size();
  *dm = reinterpret_cast<const bk::MultiScatterArgs*>(scratch + bp.tables_off + moff);
  return BIN_OK;
}

int multi_launch(const MultiPlan& mp, const bk::MultiScatterArgs* dm, hipStream_t s, bk::KTimer* tm) {
  const PartGroup& g = mp.bp.part[0];
  hipError_t e = bk::launch_scatter_multi(dm, g.args[0].nwg, mp.lds, s, tm);
  if (e == hipSuccess) e = bk::launch_partition_batch_after_scatter(g.b, g.cf64, g.af64, g.prec, g.cfg, s, tm);
  if (e != hipSuccess) return hip_fail(e, "launch fused multi-grid kernels");
  return BIN_OK;
}

// Returns false (nothing done) when the requests do not qualify.
bool run_multi_fused(const bin_request* reqs, int nreq, hipStream_t s, int* status) {
  DeviceInfo dev;
  *status = device_info(&dev);
  if (*status) return true;
  MultiPlan mp;
  if (!multi_plan(reqs, nreq, dev, &mp, status)) return *status != BIN_OK;
  void* scratch = nullptr;
  *status = scratch_get(dev.device, s, mp.scratch_bytes(), &scratch);
  if (*status) return true;
  const bk::MultiScatterArgs* dm = nullptr;
  *status = multi_layout(reqs, nreq, dev, static_cast<unsigned char*>(scratch), &mp, &dm);
  if (*status == BIN_OK) *status = upload_tables(mp.bp, static_cast<unsigned char*>(scratch), s);
  if (*status == BIN_OK) *status = multi_launch(mp, dm, s, timing_timer());
  return true;
}

}  // namespace

int run_batch(const bin_request* reqs, int nreq, hipStream_t s, const PlanHints& hints) {
  int st = validate_requests(reqs, nreq);
  if (st) return st;
  if (nreq == 0) return BIN_OK;
  if (nreq == 1) return run_request(reqs[0], s, hints);  // the single-request kernels
  DeviceInfo dev;
  st = device_info(&dev);
  if (st) return st;
  BatchPlan bp;
  st = plan_batch(reqs, nreq, dev, hints, nullptr, &bp);
  if (st) return st;
  void* scratch = nullptr;
  st = scratch_get(dev.device, s, bp.scratch_bytes, &scratch);
  if (st) return st;
  st = plan_batch(reqs, nreq, dev, hints, static_cast<unsigned char*>(scratch), &bp);
  if (st) return st;
  st = upload_tables(bp, static_cast<unsigned char*>(scratch), s);
  if (st) return st;
  bk::KTimer* tm = timing_timer();
  st = launch_batch(bp, s, tm);
  if (st) return st;
  for (int i : bp.global_reqs) {
    st = run_request(reqs[i], s, hints);
    if (st) return st;
  }
  return BIN_OK;
}

size_t batch_scratch_bytes(const bin_request* reqs, int nreq, int* status) {
  *status = validate_requests(reqs, nreq);
  if (*status || nreq == 0) return 0;
  DeviceInfo dev;
  *status = device_info(&dev);
  if (*status) return 0;
  BatchPlan bp;
  *status = plan_batch(reqs, nreq, dev, thread_hints(), nullptr, &bp);
  if (*status) return 0;
  size_t extra = 0;  // requests on the global strategy use their own scratch
  for (int i : bp.global_reqs) extra += al256(bp.preps[i].scratch_bytes);
  return bp.scratch_bytes + extra;
}

}  // namespace binimpl

// ---------------------------------------------------------------------------
// Graphs.
// ---------------------------------------------------------------------------
struct bin_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* scratch = nullptr;
  int device = 0;
};

namespace binimpl {
namespace {

// The requests of a multi-grid call: one per grid spec, all over the same
// columns; checked as bin_particles checks its arguments.
int specs_to_requests(const bin_columns* coords, const bin_columns* attrs, int64_t n, const bin_grid_spec* grids,
                      int32_t ngrids, std::vector<bin_request>* out) {
  if (!coords) return fail(BIN_ERR_INVALID_ARG, "coords is NULL");
  if (ngrids < 0 || ngrids > 65535) return fail(BIN_ERR_INVALID_ARG, "ngrids must be in [0, 65535]");
  if (ngrids > 0 && !grids) return fail(BIN_ERR_INVALID_ARG, "grids is NULL");
  std::vector<bin_request>& reqs = *out;
  reqs.assign((size_t)ngrids, bin_request{});
  for (int g = 0; g < ngrids; ++g) {
    bin_request& r = reqs[(size_t)g];
    std::memset(&r, 0, sizeof r);
    r.coords = *coords;
    if (attrs) r.attrs = *attrs;
    r.n = n;
    r.axes[0] = grids[g].axes[0];
    r.axes[1] = grids[g].axes[1];
    std::memcpy(r.bounds, grids[g].bounds, sizeof r.bounds);
    r.nx = grids[g].nx;
    r.ny = grids[g].ny;
    r.ops = grids[g].ops;
    r.out = grids[g].out;
  }
  return validate_requests(reqs.data(), ngrids);
}

int copy_tables(const BatchPlan& bp, unsigned char* scratch) {
  if (!bp.tables_bytes) return BIN_OK;
  const hipError_t e = hipMemcpy(scratch + bp.tables_off, bp.tables.data(), bp.tables_bytes, hipMemcpyHostToDevice);
  return e == hipSuccess ? BIN_OK : hip_fail(e, "hipMemcpy(graph tables)");
}

// A graph that owns scratch_bytes of device memory: 'layout' fills it (and
// uploads the tables), then 'launch' is captured on a private stream.
int capture_graph(int device, size_t scratch_bytes, const std::function<int(unsigned char*)>& layout,
                  const std::function<int(hipStream_t)>& launch, bin_graph** out) {
  bin_graph* g = new bin_graph;
  g->device = device;
  hipError_t e = hipMalloc(&g->scratch, std::max<size_t>(scratch_bytes, 256));
  if (e != hipSuccess) {
    delete g;
    return hip_fail(e, "hipMalloc(graph scratch)");
  }
  int st = layout(static_cast<unsigned char*>(g->scratch));
  hipStream_t cs = nullptr;
  if (st == BIN_OK) {
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) st = hip_fail(e, "hipStreamCreate(capture)");
  }
  if (st == BIN_OK) {
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) st = hip_fail(e, "hipStreamBeginCapture");
  }
  if (st == BIN_OK) {
    const int lst = launch(cs);
    e = hipStreamEndCapture(cs, &g->graph);
    if (lst) st = lst;
    else if (e != hipSuccess) st = hip_fail(e, "hipStreamEndCapture");
  }
  if (st == BIN_OK) {
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) st = hip_fail(e, "hipGraphInstantiate");
  }
  if (cs) (void)hipStreamDestroy(cs);
  if (st) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    (void)hipFree(g->scratch);
    delete g;
    return st;
  }
  *out = g;
  return BIN_OK;
}

// The batched launch sequence of validated requests as a graph.
int batch_graph(const bin_request* reqs, int nreq, bin_graph** out) {
  DeviceInfo dev;
  int st = device_info(&dev);
  if (st) return st;
  BatchPlan bp;
  const PlanHints& hints = thread_hints();
  st = plan_batch(reqs, nreq, dev, hints, nullptr, &bp);
  if (st) return st;
  if (!bp.global_reqs.empty())
    return fail(BIN_ERR_UNSUPPORTED, "graphs do not take requests that need the global-atomic strategy");
  return capture_graph(
      dev.device, bp.scratch_bytes,
      [&](unsigned char* scratch) {
        const int lst = plan_batch(reqs, nreq, dev, hints, scratch, &bp);
        return lst ? lst : copy_tables(bp, scratch);
      },
      [&](hipStream_t cs) { return launch_batch(bp, cs, nullptr); }, out);
}

}  // namespace
}  // namespace binimpl

using namespace binimpl;

extern "C" {

int bin_particles_batched(const bin_request* reqs, int32_t nreq, void* stream) {
  clear_error();
  return run_batch(reqs, nreq, static_cast<hipStream_t>(stream), thread_hints());
}

int bin_particles_multi(const bin_columns* coords, const bin_columns* attrs, int64_t n,
                        const bin_grid_spec* grids, int32_t ngrids, void* stream) {
  clear_error();
  std::vector<bin_request> reqs;
  int st = specs_to_requests(coords, attrs, n, grids, ngrids, &reqs);
  if (st) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (run_multi_fused(reqs.data(), ngrids, s, &st)) return st;
  return run_batch(reqs.data(), ngrids, s, thread_hints());
}

int bin_graph_create(const bin_request* reqs, int32_t nreq, bin_graph** out) {
  clear_error();
  if (!out) return fail(BIN_ERR_INVALID_ARG, "graph is NULL");
  *out = nullptr;
  int st = validate_requests(reqs, nreq);
  if (st) return st;
  if (nreq == 0) return fail(BIN_ERR_INVALID_ARG, "a graph needs at least one request");
  return batch_graph(reqs, nreq, out);
}

int bin_graph_create_multi(const bin_columns* coords, const bin_columns* attrs, int64_t n,
                           const bin_grid_spec* grids, int32_t ngrids, bin_graph** out) {
  clear_error();
  if (!out) return fail(BIN_ERR_INVALID_ARG, "graph is NULL");
  *out = nullptr;
  std::vector<bin_request> reqs;
  int st = specs_to_requests(coords, attrs, n, grids, ngrids, &reqs);
  if (st) return st;
  if (ngrids == 0) return fail(BIN_ERR_INVALID_ARG, "a graph needs at least one grid");
  DeviceInfo dev;
  st = device_info(&dev);
  if (st) return st;
  MultiPlan mp;
  if (!multi_plan(reqs.data(), ngrids, dev, &mp, &st)) {
    if (st) return st;
    return batch_graph(reqs.data(), ngrids, out);  // the specs run as one batch
  }
  const bk::MultiScatterArgs* dm = nullptr;
  return capture_graph(
      dev.device, mp.scratch_bytes(),
      [&](unsigned char* scratch) {
        const int lst = multi_layout(reqs.data(), ngrids, dev, scratch, &mp, &dm);
        return lst ? lst : copy_tables(mp.bp, scratch);
      },
      [&](hipStream_t cs) { return multi_launch(mp, dm, cs, nullptr); }, out);
}

int bin_graph_launch(bin_graph* g, void* stream) {
  clear_error();
  if (!g || !g->exec) return fail(BIN_ERR_INVALID_ARG, "graph is NULL");
  hipError_t e = hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return BIN_OK;
}

int bin_graph_destroy(bin_graph* g) {
  clear_error();
  if (!g) return BIN_OK;
  hipError_t e = hipDeviceSynchronize();  // no replay may still use the scratch
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->scratch) (void)hipFree(g->scratch);
  delete g;
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  return BIN_OK;
}

}  // extern "C"
