// Partition strategy for grids too large for one LDS tile.
//
// Global atomics on gfx950 sustain only a few tens of G lane-ops/s across
// the whole device, while LDS atomics run two orders of magnitude faster, so
// large grids are binned without any per-particle global atomic.  A tile is
// TB = 2^s consecutive flat bins, TB chosen so that a tile's accumulators
// fill one workgroup's LDS.
//
//   part_scatter  per workgroup slice of particles, per sub-chunk: LDS sort
//                 of the sub-chunk's inside particles by tile, then the
//                 records (u16 local bin + attribute values) are written
//                 back in tile order over the sub-chunk's own index range,
//                 so every store is part of one contiguous stream.  The
//                 start of each tile's run in the sub-chunk goes to a small
//                 table, and each slice's per-tile record totals to
//                 counts[tile][slice].
//   part_items    one work item per tile; a heavy tile is split into items
//                 that each take a range of whole slices.
//   part_bin      one workgroup per item: gathers the tile's runs from every
//                 sub-chunk of its slices (a wave-wide load-balanced search
//                 maps lanes to records), accumulates them in LDS, then
//                 writes the finished outputs - count, sum, min, max, avg -
//                 or, for a split tile, a partial slot.
//   part_merge    combines the partials of split tiles into outputs.
//
// Scattered runs of a few records per tile were measured on MI355X to write
// at under 2 TB/s, while the same bytes written as one stream per sub-chunk
// go at full rate; the gather in part_bin reads the same runs with many
// workgroups moving through the sub-chunks together, so neighbouring runs
// are read at about the same time.
//
// Every kernel body takes its request record by reference, so one body
// serves a single request (record passed by value as the kernel argument)
// and a batch (records in a device table, one block per (request, index)
// pair listed in a block map: map = request << 16 | index).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"
#include "kernels.h"

namespace bk {

// ---------------------------------------------------------------------------
// Shape of workgroup slice w: whole sub-chunks of 'sub' particles (aligned
// requests only), then remainder sub-chunks of 'sub_tail' particles.
// ---------------------------------------------------------------------------
struct SliceShape {
  int64_t lo, hi;
  int32_t nfull, nblocks;
};

// Every slice but the last has the same length, so the two shapes come
// from the host and no lane divides.
__device__ __forceinline__ SliceShape slice_shape(const PartArgs& a, int w) {
  SliceShape s;
  s.lo = (int64_t)w * a.chunk;
  s.hi = s.lo + a.chunk < a.n ? s.lo + a.chunk : a.n;
  const bool last = w == a.nwg - 1;
  s.nfull = last ? a.nfull_z : a.nfull_a;
  s.nblocks = last ? a.nblocks_z : a.nblocks_a;
  return s;
}

__device__ __forceinline__ int64_t block_base(const SliceShape& s, const PartArgs& a, int j) {
  return j < s.nfull ? s.lo + (int64_t)j * a.sub
                     : s.lo + (int64_t)s.nfull * a.sub + (int64_t)(j - s.nfull) * a.sub_tail;
}

// Fixed block size NT, wave shuffles (three barriers); wave_tot: NT/64 words.
template <int NT>
__device__ __forceinline__ uint32_t block_scan_excl(uint32_t v, uint32_t* wave_tot, uint32_t& total) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) wave_tot[wid] = x;
  __syncthreads();
  if (wid == 0) {
    uint32_t w = lane < NW ? wave_tot[lane] : 0u;
#pragma unroll
    for (int o = 1; o < NW; o <<= 1) {
      const uint32_t y = __shfl_up(w, o);
      if (lane >= o) w += y;
    }
    if (lane < NW) wave_tot[lane] = w;
  }
  __syncthreads();
  const uint32_t base = wid ? wave_tot[wid - 1] : 0u;
  total = wave_tot[NW - 1];
  __syncthreads();
  return base + x - v;
}

// ---------------------------------------------------------------------------
// Scatter: per sub-chunk of S = NT * PPT particles, rank each inside
// particle within its tile (LDS atomic), scan the tile counts, place records
// in LDS in tile order, then copy them out over the sub-chunk's own index
// range.  Lane t takes the groups of 4 consecutive particles starting at
// base + 4 * (q * NT + t), q < PPT / 4.  Whole sub-chunks of an aligned
// request are read with 16-byte loads and no bounds tests, and the next
// one's coordinates are loaded while the current one is sorted and written;
// the remainder (and unaligned requests) take a bounds-tested path with 4
// particles per thread.  Three barriers per sub-chunk (two more per extra
// attribute): the tile counters are double-buffered, and one wave scans
// them, adds them to the slice totals and clears the other buffer.  With
// quads each tile's run is padded to a multiple of 4 records (bin 0xFFFF).
// LDS: cnt[2][T] | off[T] | tot[T] | local bin u16[S + pad_row] |
//      values[S + pad_row] | staged run-table rows u16[T + 1][2^off_shift]
// ---------------------------------------------------------------------------
struct ScatterShared {
  uint32_t nsub;
};

template <typename CT, typename AT, int PPT, int NT, bool FULL>
__device__ __forceinline__ void scatter_sub(const PartArgs& a, unsigned char* smem, ScatterShared& sh,
                                            const Axis& ax, const Axis& ay, int64_t base, int64_t hi,
                                            int64_t full_end, int64_t row0, int j, bool flush, int parity,
                                            CT* px, CT* py) {
  constexpr int S = NT * PPT;
  constexpr int Q = PPT / 4;
  const int T = a.ntiles;
  uint32_t* cnt = reinterpret_cast<uint32_t*>(smem) + parity * T;
  uint32_t* cprev = reinterpret_cast<uint32_t*>(smem) + (parity ^ 1) * T;
  uint32_t* off = reinterpret_cast<uint32_t*>(smem) + 2 * T;
  uint32_t* tot = off + T;
  uint16_t* stg_b = reinterpret_cast<uint16_t*>(tot + T);
  AT* stg_v = reinterpret_cast<AT*>(smem + a.stage_val_off);
  const int shift = a.lay.tile_shift;
  const uint32_t lmask = (1u << shift) - 1u;
  const int k = a.k;

  // Whole sub-chunks index from a workgroup-uniform base pointer with 32-bit
  // lane offsets (one address register per load instead of two).  The first
  // attribute's values are loaded before the bins are located, so their
  // latency hides behind locating, ranking and the scan.
  const uint32_t lane4 = 4u * threadIdx.x;
  // (Sub-chunks of 16 or more particles per thread have no registers to
  // spare for this: they load the values when they stage them.)
  constexpr bool kPre = PPT <= 12;
  AT v0[kPre ? PPT : 1];
  if (kPre && k > 0) {
    if constexpr (FULL) {
      const AT* ab = static_cast<const AT*>(a.attr[0]) + base;
#pragma unroll
      for (int q = 0; q < Q; ++q) ld4v<AT>(ab, lane4 + 4u * q * NT, v0 + 4 * q);
    } else {
#pragma unroll
      for (int q = 0; q < Q; ++q)
        ld4<AT>(a.attr[0], base + 4 * ((int64_t)q * NT + threadIdx.x), hi, false, v0 + 4 * q);
    }
  }
  uint32_t tb[PPT], pos[PPT];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t i = base + 4 * ((int64_t)q * NT + threadIdx.x);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int u = 4 * q + e;
      tb[u] = 0xFFFFFFFFu;
      int ix, iy;
      if ((FULL || i + e < hi) && locate((double)px[u], ax, ix) && locate((double)py[u], ay, iy)) {
        const uint32_t b = (uint32_t)(iy * a.nx + ix);
        tb[u] = ((b >> shift) << 16) | (b & lmask);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < PPT; ++u) pos[u] = tb[u] != 0xFFFFFFFFu ? atomicAdd(cnt + (tb[u] >> 16), 1u) : 0u;
  if constexpr (FULL) {  // prefetch the next whole sub-chunk's coordinates
    if (base + S < full_end) {
      const CT* xb = static_cast<const CT*>(a.x) + (base + S);
      const CT* yb = static_cast<const CT*>(a.y) + (base + S);
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        ld4v<CT>(xb, lane4 + 4u * q * NT, px + 4 * q);
        ld4v<CT>(yb, lane4 + 4u * q * NT, py + 4 * q);
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < 64) {  // one wave: lane l owns tiles [l * m, l * m + m)
    const int lane = threadIdx.x;
    const int m = (T + 63) >> 6;
    const int t0 = lane * m;
    const uint32_t padm = a.quads ? 3u : 0u;  // runs padded to whole quads
    uint32_t own = 0;
    for (int q = 0; q < m; ++q)
      if (t0 + q < T) own += (cnt[t0 + q] + padm) & ~padm;
    uint32_t x = own;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    uint32_t o0 = x - own;
    for (int q = 0; q < m; ++q) {
      const int t = t0 + q;
      if (t < T) {
        const uint32_t c = (cnt[t] + padm) & ~padm;
        tot[t] += c;
        cprev[t] = 0u;
        off[t] = o0;
        o0 += c;
      }
    }
    if (lane == 63) sh.nsub = x;
  }
  __syncthreads();
  const uint32_t nsub = sh.nsub;
  // The run table is kept per tile (column t lists the tile's run starts in
  // consecutive sub-chunks), so that part_bin reads it contiguously.  Rows
  // are staged in LDS as [tile][F] and written F at a time.
  const int F = 1 << a.off_shift;
  uint16_t* ost = reinterpret_cast<uint16_t*>(smem + a.off_stage);
  for (int t = threadIdx.x; t <= T; t += NT) {
    ost[(t << a.off_shift) + (j & (F - 1))] = (uint16_t)(t < T ? off[t] : nsub);
    if (a.quads && t < T) {  // pad the tile's run to a whole quad: bin 0xFFFF, value 0
      const uint32_t c = cnt[t];
      const uint32_t e = off[t] + ((c + 3u) & ~3u);
      for (uint32_t p = off[t] + c; p < e; ++p) {
        stg_b[p] = 0xFFFFu;
        if (k > 0) stg_v[p] = AT(0);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    if (tb[u] == 0xFFFFFFFFu) continue;
    pos[u] += off[tb[u] >> 16];
    stg_b[pos[u]] = (uint16_t)(tb[u] & 0xFFFFu);
  }
  if (k > 0) {
    if constexpr (kPre) {
#pragma unroll
      for (int u = 0; u < PPT; ++u)
        if (tb[u] != 0xFFFFFFFFu) stg_v[pos[u]] = v0[kPre ? u : 0];
    } else {
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        AT v[4];
        if constexpr (FULL)
          ld4v<AT>(static_cast<const AT*>(a.attr[0]) + base, lane4 + 4u * q * NT, v);
        else
          ld4<AT>(a.attr[0], base + 4 * ((int64_t)q * NT + threadIdx.x), hi, false, v);
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (tb[4 * q + e] != 0xFFFFFFFFu) stg_v[pos[4 * q + e]] = v[e];
      }
    }
  }
  __syncthreads();
  if (flush) {  // rows [j0, j] of the slice: column t gets f consecutive entries
    const int j0 = j & ~(F - 1);
    const int f = j - j0 + 1;
    const int64_t nrows = (int64_t)a.nwg * a.nbpw;
    const int64_t r0 = row0 + j0;
    for (int i = threadIdx.x; i < ((T + 1) << a.off_shift); i += NT) {
      const int t = i >> a.off_shift, jj = i & (F - 1);
      if (jj < f) a.blk_off[(int64_t)t * nrows + r0 + jj] = ost[i];
    }
  }
  // One contiguous stream of records over [rbase, rbase + nsub); with quads
  // (nsub and rbase multiples of 4) as 8-byte bin and 16-byte value stores.
  const int64_t rbase = base + (row0 + j) * (int64_t)a.pad_row;
  if (a.quads) {
    u32x2* rb = reinterpret_cast<u32x2*>(a.rec_bin + rbase);
    const u32x2* sb = reinterpret_cast<const u32x2*>(stg_b);
    for (uint32_t p = threadIdx.x; p < nsub / 4; p += NT) __builtin_nontemporal_store(sb[p], rb + p);
  } else {
    uint16_t* rb = a.rec_bin + rbase;
    for (uint32_t p = threadIdx.x; p < nsub; p += NT) __builtin_nontemporal_store(stg_b[p], rb + p);
  }
  auto copy_values = [&](int jx) {
    if (a.quads) {
      constexpr uint32_t kVq = sizeof(AT) / 4;  // 16-byte units per quad of values
      u32x4* rv = reinterpret_cast<u32x4*>(static_cast<AT*>(a.rec_val[jx]) + rbase);
      const u32x4* sv = reinterpret_cast<const u32x4*>(stg_v);
      for (uint32_t p = threadIdx.x; p < nsub / 4 * kVq; p += NT) __builtin_nontemporal_store(sv[p], rv + p);
    } else {
      AT* rv = static_cast<AT*>(a.rec_val[jx]) + rbase;
      for (uint32_t p = threadIdx.x; p < nsub; p += NT) __builtin_nontemporal_store(stg_v[p], rv + p);
    }
  };
  if (k > 0) copy_values(0);
  // Further attributes reuse the one value stage (the positions are the
  // same), so the stage is as large for k attributes as for one.  Keeping
  // the positions live costs registers: requests with two or more
  // attributes run sub-chunks of at most 8192 particles (the planner's
  // rule), and only those instances carry this loop.
  if constexpr (S <= 8192)
  for (int jx = 1; jx < k; ++jx) {
    __syncthreads();  // the previous attribute's copy-out has read the stage
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      AT v[4];
      if constexpr (FULL)
        ld4v<AT>(static_cast<const AT*>(a.attr[jx]) + base, lane4 + 4u * q * NT, v);
      else
        ld4<AT>(a.attr[jx], base + 4 * ((int64_t)q * NT + threadIdx.x), hi, false, v);
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (tb[4 * q + e] != 0xFFFFFFFFu) stg_v[pos[4 * q + e]] = v[e];
    }
    __syncthreads();
    copy_values(jx);
  }
}

template <typename CT, typename AT, int PPT, int NT>
__device__ __forceinline__ void part_scatter_body(const PartArgs& a, int wg) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ ScatterShared sh;
  constexpr int S = NT * PPT;
  constexpr int Q = PPT / 4;
  const int T = a.ntiles;
  uint32_t* cnt = reinterpret_cast<uint32_t*>(smem);
  uint32_t* tot = cnt + 3 * T;
  Axis ax = a.ax, ay = a.ay;
  resolve_axes(a.dyn, ax, ay);
  for (int t = threadIdx.x; t < T; t += NT) {
    cnt[t] = 0u;
    cnt[T + t] = 0u;
    tot[t] = 0u;
  }
  const SliceShape shp = slice_shape(a, wg);
  const int64_t lo = shp.lo, hi = shp.hi;
  const int64_t full_end = lo + (int64_t)shp.nfull * S;
  const int64_t row0 = (int64_t)wg * a.nbpw;
  CT px[PPT], py[PPT];
  if (lo < full_end) {
    const CT* xb = static_cast<const CT*>(a.x) + lo;
    const CT* yb = static_cast<const CT*>(a.y) + lo;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      ld4v<CT>(xb, 4u * (q * NT + threadIdx.x), px + 4 * q);
      ld4v<CT>(yb, 4u * (q * NT + threadIdx.x), py + 4 * q);
    }
  }
  __syncthreads();
  int parity = 0;
  int j = 0;
  const int F = 1 << a.off_shift;
  auto flush_at = [&](int jj) { return ((jj + 1) & (F - 1)) == 0 || jj + 1 == shp.nblocks; };
  for (int64_t base = lo; base < full_end; base += S, parity ^= 1, ++j)
    scatter_sub<CT, AT, PPT, NT, true>(a, smem, sh, ax, ay, base, hi, full_end, row0, j, flush_at(j), parity, px,
                                       py);
  // The remainder in sub-chunks of 4 particles per thread (fewer registers;
  // the staging area holds S >= 4 * NT entries).
  constexpr int S4 = 4 * NT;
  for (int64_t base = full_end; base < hi; base += S4, parity ^= 1, ++j) {
    CT tx[4], ty[4];
    const int64_t i = base + 4 * (int64_t)threadIdx.x;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      tx[e] = i + e < hi ? ld<CT>(a.x, i + e) : CT(0);
      ty[e] = i + e < hi ? ld<CT>(a.y, i + e) : CT(0);
    }
    scatter_sub<CT, AT, 4, NT, false>(a, smem, sh, ax, ay, base, hi, full_end, row0, j, flush_at(j), parity, tx,
                                      ty);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < T; t += NT) a.counts[(int64_t)t * a.nwg + wg] = tot[t];
}

template <typename CT, typename AT, int PPT, int NT>
__global__ __launch_bounds__(NT) void part_scatter_kernel(PartArgs a) {
  part_scatter_body<CT, AT, PPT, NT>(a, blockIdx.x);
}
template <typename CT, typename AT, int PPT, int NT>
__global__ __launch_bounds__(NT) void part_scatter_batched(const PartArgs* __restrict__ d,
                                                           const uint32_t* __restrict__ map) {
  const uint32_t m = map[blockIdx.x];
  part_scatter_body<CT, AT, PPT, NT>(d[m >> 16], (int)(m & 0xFFFFu));
}

// ---------------------------------------------------------------------------
// Work items.  For tile t, slice w starts at record excl(w) of the tile (an
// exclusive prefix over the tile's per-slice counts); its item is
// floor(excl(w) / split_len), so an item holds whole slices and at most
// split_len records plus one slice's.  A tile has at most
// ceil(records / split_len) items; an empty tile has one item with no
// slices, which writes its empty bins.
// items[3i] = tile, [3i+1] = first slice, [3i+2] = end slice.
// tile_items[3t] = first item, [3t+1] = items, [3t+2] = first partial slot
// (split tiles only).  One block (1024 threads, one wave per tile at a
// time per tile in the walk, one block in the placement) per request.
// ---------------------------------------------------------------------------
struct ItemScan {
  uint32_t n;       // items of the tile
  uint32_t total;   // records of the tile
};

// One wave walks tile t's counts; emit(w, index within the tile) is called
// (on the lane of slice w) for each slice that starts an item.
template <typename F>
__device__ __forceinline__ ItemScan tile_item_walk(const PartArgs& a, int t, F emit) {
  const int lane = threadIdx.x & 63;
  const uint32_t* row = a.counts + (int64_t)t * a.nwg;
  uint32_t carry = 0, nflag = 0, mprev = 0;
  for (int w0 = 0; w0 < a.nwg; w0 += 64) {
    const int w = w0 + lane;
    const uint32_t c = w < a.nwg ? row[w] : 0u;
    uint32_t incl = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o);
      if (lane >= o) incl += y;
    }
    const uint32_t m = (carry + incl - c) / a.split_len;
    uint32_t up = __shfl_up(m, 1);
    if (lane == 0) up = mprev;
    const bool flag = w < a.nwg && (w == 0 || m != up);
    const uint64_t bal = __ballot(flag);
    if (flag) emit(w, nflag + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull)));
    nflag += (uint32_t)__popcll(bal);
    const int last = (a.nwg - w0 < 64 ? a.nwg - w0 : 64) - 1;
    mprev = __shfl(m, last);
    carry += __shfl(incl, 63);
  }
  return ItemScan{nflag, carry};
}

// Walk: one wave per tile records where the tile's items start (ilist) and
// how many there are and how many records the tile has (tile_items[3t+1],
// [3t+2], completed by the placement below).
__device__ __forceinline__ void part_items_walk_body(const PartArgs& a, int blk) {
  const int t = blk * 16 + (int)(threadIdx.x >> 6);
  if (t >= a.ntiles) return;
  uint32_t* list = a.ilist + (int64_t)t * a.nwg;
  const ItemScan is = tile_item_walk(a, t, [&](int w, uint32_t idx) { list[idx] = (uint32_t)w; });
  if ((threadIdx.x & 63) == 0) {
    a.tile_items[3 * t + 1] = is.n;
    a.tile_items[3 * t + 2] = is.total;
  }
}

// Placement: one block numbers the items of all tiles (exclusive scans over
// tiles, 4 tiles per thread) and writes them out.
// LDS workspace: wave_tot[16] then fi[4096] (the first item of each tile;
// T <= 4096).
constexpr int kPlaceLds = 4 * (16 + 4096);
__device__ __forceinline__ void part_items_place_body(const PartArgs& a, uint32_t* lds) {
  uint32_t* wave_tot = lds;
  uint32_t* fi = lds + 16;
  const int T = a.ntiles;
  const int t0 = 4 * threadIdx.x;
  uint32_t ni[4], nrec[4];
  uint32_t own = 0, sown = 0, nsplit = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    ni[q] = 0;
    nrec[q] = 0;
    if (t0 + q < T) {
      nrec[q] = a.tile_items[3 * (t0 + q) + 2];
      ni[q] = nrec[q] ? a.tile_items[3 * (t0 + q) + 1] : 1u;
      own += ni[q];
      sown += ni[q] > 1 ? ni[q] : 0u;
      nsplit += ni[q] > 1 ? 1u : 0u;
    }
  }
  uint32_t tot, stot, ntot;
  uint32_t first = block_scan_excl<1024>(own, wave_tot, tot);
  uint32_t sfirst = block_scan_excl<1024>(sown, wave_tot, stot);
  uint32_t lfirst = block_scan_excl<1024>(nsplit, wave_tot, ntot);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int t = t0 + q;
    if (t >= T) continue;
    if (ni[q] > 1) a.split_list[lfirst++] = (uint32_t)t;
    a.tile_items[3 * t] = first;
    a.tile_items[3 * t + 1] = ni[q];
    a.tile_items[3 * t + 2] = sfirst;
    // an empty tile's item has no slices: its end slice is written as 0 below
    fi[t] = first | (nrec[q] ? 0u : 0x80000000u);
    first += ni[q];
    sfirst += ni[q] > 1 ? ni[q] : 0u;
  }
  if (threadIdx.x == 0) a.split_list[T] = ntot;
  __syncthreads();
  // Item i: its tile is the last one whose first item is <= i (every tile
  // has at least one item, so the firsts strictly increase).
  const uint32_t cap = (uint32_t)a.max_items;  // a proven upper bound; the guards keep stores in range
  const uint32_t nitems = tot < cap ? tot : cap;
  for (uint32_t i = threadIdx.x; i < nitems; i += blockDim.x) {
    int lo = 0, hi = T - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if ((fi[mid] & 0x7FFFFFFFu) <= i) lo = mid;
      else hi = mid - 1;
    }
    const int t = lo;
    const uint32_t f = fi[t] & 0x7FFFFFFFu;
    const bool empty = (fi[t] >> 31) != 0;
    const uint32_t idx = i - f;
    const uint32_t nxt = t + 1 < T ? (fi[t + 1] & 0x7FFFFFFFu) : tot;
    const uint32_t* list = a.ilist + (int64_t)t * a.nwg;
    a.items[3 * i] = (uint32_t)t;
    a.items[3 * i + 1] = empty ? 0u : list[idx];
    a.items[3 * i + 2] = empty ? 0u : (i + 1 < nxt ? list[idx + 1] : (uint32_t)a.nwg);
  }
  if (threadIdx.x == 0) *a.n_items = nitems;
}

__global__ __launch_bounds__(1024) void part_items_walk_kernel(PartArgs a) { part_items_walk_body(a, blockIdx.x); }
__global__ __launch_bounds__(1024) void part_items_walk_batched(const PartArgs* __restrict__ d,
                                                                const uint32_t* __restrict__ map) {
  const uint32_t m = map[blockIdx.x];
  part_items_walk_body(d[m >> 16], (int)(m & 0xFFFFu));
}
__global__ __launch_bounds__(1024) void part_items_kernel(PartArgs a) {
  __shared__ uint32_t lds[kPlaceLds / 4];
  part_items_place_body(a, lds);
}
__global__ __launch_bounds__(1024) void part_items_batched(const PartArgs* __restrict__ d) {
  __shared__ uint32_t lds[kPlaceLds / 4];
  part_items_place_body(d[blockIdx.x], lds);
}

// ---------------------------------------------------------------------------
// Per-item tile binning; fused finalize for tiles binned by one item.
// Each wave takes 64 sub-chunks of the item's slices at a time, one per
// lane: the lane reads where the tile's run starts and ends in its
// sub-chunk; an inclusive scan of the run lengths across the wave then maps
// the concatenated runs onto the lanes 64 records at a time (a binary
// search over the scan for the lane's run).
// ---------------------------------------------------------------------------
// The 4 values of quad q (16-byte loads; zeros for no quad).  Records are
// read with plain loads: the cache lines at the ends of a run are shared
// with the neighbouring tiles' runs, which other workgroups gather at about
// the same time, so the lines should stay in L2 rather than be streamed
// past it.
template <typename AT>
__device__ __forceinline__ void ld_quad(const void* p, uint32_t q, AT* out) {
  if (q == 0xFFFFFFFFu) {
#pragma unroll
    for (int e = 0; e < 4; ++e) out[e] = AT(0);
    return;
  }
  if constexpr (sizeof(AT) == 4) {
    const f32x4 v = reinterpret_cast<const f32x4*>(p)[q];
    out[0] = v.x;
    out[1] = v.y;
    out[2] = v.z;
    out[3] = v.w;
  } else {
    const f64x2* d = reinterpret_cast<const f64x2*>(p) + 2 * (int64_t)q;
    const f64x2 a = d[0], b = d[1];
    out[0] = a.x;
    out[1] = a.y;
    out[2] = b.x;
    out[3] = b.y;
  }
}

template <typename AT, int PREC, bool QUAD>
__device__ __forceinline__ void part_bin_body(const PartArgs& a, int item) {
  using TL = Tile<AT, PREC>;
  extern __shared__ __align__(16) unsigned char smem[];
  if (item >= (int)*a.n_items) return;
  const uint32_t t = a.items[3 * item];
  const uint32_t w0 = a.items[3 * item + 1];
  const uint32_t w1 = a.items[3 * item + 2];
  const int shift = a.lay.tile_shift;
  const int64_t b0 = (int64_t)t << shift;
  const int TB = 1 << shift;
  const int nbt = (int)((b0 + TB <= a.nbins) ? TB : a.nbins - b0);
  const int k = a.k;
  TL::init(smem, a.lay, k);
  __syncthreads();

  const int lane = threadIdx.x & 63;
  const uint32_t wid = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // wave-uniform
  const uint32_t nwaves = blockDim.x >> 6;
  const uint32_t nblk = (w1 - w0) * (uint32_t)a.nbpw;
  // Column t of the run table from the item's first row: consecutive lanes
  // read consecutive entries.
  const int64_t nrows = (int64_t)a.nwg * a.nbpw;
  const uint16_t* col = a.blk_off + (int64_t)t * nrows + (int64_t)w0 * a.nbpw;
  // The lane's run in sub-chunk c of the item (len 0 past the end or for a
  // sub-chunk a short slice does not have).
  if constexpr (QUAD) {
    // The lane's run in sub-chunk c of the item, in quads of 4 records: its
    // length and the quad index of its first quad (len 0 past the end or for
    // a sub-chunk a short slice does not have).
    auto run_of = [&](uint32_t c, uint32_t& len, uint32_t& rs) {
      len = 0;
      rs = 0;
      if (c < nblk) {
        const uint32_t dw = c / (uint32_t)a.nbpw;
        const int w = (int)(w0 + dw);
        const int j = (int)(c - dw * (uint32_t)a.nbpw);
        const SliceShape shp = slice_shape(a, w);
        if (j < shp.nblocks) {
          const uint32_t s0 = col[c];
          len = ((uint32_t)col[c + nrows] - s0) >> 2;
          const int64_t r0 = block_base(shp, a, j) + ((int64_t)w * a.nbpw + j) * a.pad_row + s0;
          rs = (uint32_t)(r0 >> 2);
        }
      }
    };
    // Groups of 64 sub-chunks; with fewer groups than waves, wpg waves share
    // a group and take every wpg-th window of its quads.
    const uint32_t ngroups = (nblk + 63) / 64;
    uint32_t wpg = 1;
    while (wpg < nwaves && ngroups * wpg * 2 <= nwaves) wpg *= 2;
    const uint32_t gstride = nwaves / wpg;
    const uint32_t sub = wid % wpg;
    uint32_t nlen, nrs;  // the next group's run, read while this group is binned
    run_of((wid / wpg) * 64 + lane, nlen, nrs);
    for (uint32_t g = wid / wpg; g < ngroups; g += gstride) {
      const uint32_t len = nlen, rs = nrs;  // first quad of the lane's run
      run_of((g + gstride) * 64 + lane, nlen, nrs);
      uint32_t incl = len;
  #pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
      }
      // Wave-uniform scalars (readlane), so the window tests below stay on the
      // scalar unit: every vector instruction here costs 4 cycles per wave.
      const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
      const uint32_t start = rs - (incl - len);  // quad = start + q for q in the lane's run
      // R windows of 64 quads at a time: all their loads are issued before the
      // first LDS update, so R gathers of 4 records per lane are in flight.
      constexpr int R = sizeof(AT) == 8 ? 1 : 2;
      constexpr int N = 4 * R;
      for (uint32_t wb = 0; 64 * (sub + wpg * wb) < total; wb += R) {
        // The wave raises its issue priority while it maps its windows and
        // issues their loads, and drops it again for the LDS updates: a wave
        // about to issue gathers goes ahead of waves that only wait on the
        // LDS, so more loads are in flight (2.5% off this kernel on the
        // 2^27-particle 2048-square hotspot).
        __builtin_amdgcn_s_setprio(3);
        uint32_t quad[R];
  #pragma unroll
        for (int u = 0; u < R; ++u) {
          // Window of quads [w0q, w0q + 64): lane q's run is the number of
          // runs that end at or before q (incl is sorted), found by a
          // branch-free binary search over the wave's lanes (cross-lane reads
          // through ds_bpermute), so the R windows' searches overlap and the
          // cost does not grow with the number of runs a window spans.
          const uint32_t w0q = 64 * (sub + wpg * (wb + u));
          const uint32_t q = w0q + lane;
          int pos = 0;
  #pragma unroll
          for (int step = 32; step >= 1; step >>= 1) {
            const uint32_t e = (uint32_t)__builtin_amdgcn_ds_bpermute((pos + step - 1) << 2, (int)incl);
            pos += e <= q ? step : 0;
          }
          // pos == 64 only for q >= total
          const uint32_t st = (uint32_t)__builtin_amdgcn_ds_bpermute((pos & 63) << 2, (int)start);
          quad[u] = q < total ? st + q : 0xFFFFFFFFu;
        }
        // Every load of the R windows - bins and the first attributes - is
        // issued before the first LDS update: one 8-byte load of 4 bins and
        // 16-byte loads of their values per quad.
        constexpr int KV = sizeof(AT) == 8 ? 2 : 4;
        int lb[N];
        AT v[KV][N];
  #pragma unroll
        for (int u = 0; u < R; ++u) {
          u32x2 bq = {0xFFFFFFFFu, 0xFFFFFFFFu};
          if (quad[u] != 0xFFFFFFFFu) bq = reinterpret_cast<const u32x2*>(a.rec_bin)[quad[u]];
  #pragma unroll
          for (int e = 0; e < 4; ++e) {
            const uint32_t b = ((e < 2 ? bq.x : bq.y) >> (16 * (e & 1))) & 0xFFFFu;
            lb[4 * u + e] = b == 0xFFFFu ? -1 : (int)b;  // 0xFFFF: padding (or no quad)
          }
        }
  #pragma unroll
        for (int jj = 0; jj < KV; ++jj)
          if (jj < k) {
  #pragma unroll
            for (int u = 0; u < R; ++u) ld_quad<AT>(a.rec_val[jj], quad[u], v[jj] + 4 * u);
          }
        __builtin_amdgcn_s_setprio(0);
  #pragma unroll
        for (int e = 0; e < N; ++e)
          if (lb[e] >= 0) TL::count(smem, lb[e]);
  #pragma unroll
        for (int jj = 0; jj < KV; ++jj)
          if (jj < k) TL::template add_batch<N>(smem, a.lay, jj, lb, v[jj]);
        for (int jj = KV; jj < k; ++jj) {
          AT w[N];
  #pragma unroll
          for (int u = 0; u < R; ++u) ld_quad<AT>(a.rec_val[jj], quad[u], w + 4 * u);
          TL::template add_batch<N>(smem, a.lay, jj, lb, w);
        }
      }
    }
  } else {
    // Records one per lane (no padding): 64-record windows, each lane's run
    // picked among the window's runs with readlane.
    auto run_of = [&](uint32_t c, uint32_t& len, uint32_t& rs) {
      len = 0;
      rs = 0;
      if (c < nblk) {
        const uint32_t dw = c / (uint32_t)a.nbpw;
        const int w = (int)(w0 + dw);
        const int j = (int)(c - dw * (uint32_t)a.nbpw);
        const SliceShape shp = slice_shape(a, w);
        if (j < shp.nblocks) {
          const uint32_t s0 = col[c];
          len = (uint32_t)col[c + nrows] - s0;
          rs = (uint32_t)(block_base(shp, a, j) + s0);
        }
      }
    };
    // Groups of 64 sub-chunks; with fewer groups than waves, wpg waves share
    // a group and take every wpg-th window of its records.
    const uint32_t ngroups = (nblk + 63) / 64;
    uint32_t wpg = 1;
    while (wpg < nwaves && ngroups * wpg * 2 <= nwaves) wpg *= 2;
    const uint32_t gstride = nwaves / wpg;
    const uint32_t sub = wid % wpg;
    uint32_t nlen, nrs;  // the next group's run, read while this group is binned
    run_of((wid / wpg) * 64 + lane, nlen, nrs);
    for (uint32_t g = wid / wpg; g < ngroups; g += gstride) {
      const uint32_t len = nlen, rs = nrs;  // first record of the lane's run
      run_of((g + gstride) * 64 + lane, nlen, nrs);
      uint32_t incl = len;
  #pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
      }
      const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
      const uint32_t start = rs - (incl - len);  // record = start + q for q in the lane's run
      // R windows of 64 records at a time: all their loads are issued before
      // the first LDS update, so R gathers per wave are in flight.
      // (4 with f64 values, or with the compensated sum's 8-byte words in
      // flight, to stay within the registers of a 1024-thread workgroup)
      constexpr int R = (sizeof(AT) == 8 || PREC == PREC_COMP) ? 4 : 8;
      for (uint32_t wb = 0; 64 * (sub + wpg * wb) < total; wb += R) {
        __builtin_amdgcn_s_setprio(3);  // as in the quad gather: loads first
        uint32_t rec[R];
        int lb[R];
  #pragma unroll
        for (int u = 0; u < R; ++u) {
          // Window of records [w0q, w0q + 64): the runs holding its first and
          // last records are found with two ballots (wave-uniform), and each
          // lane picks the last run in that range starting at or before its
          // record, reading run starts with readlane (no LDS traffic).
          const uint32_t w0q = 64 * (sub + wpg * (wb + u));
          uint32_t recu = 0xFFFFFFFFu;
          if (w0q < total) {
            const uint32_t wl = w0q + 63 < total ? w0q + 63 : total - 1;
            const int la = __builtin_amdgcn_readfirstlane(__builtin_ctzll(__ballot(incl > w0q)));
            const int lb = __builtin_amdgcn_readfirstlane(__builtin_ctzll(__ballot(incl > wl)));
            const uint32_t q = w0q + lane;
            uint32_t st = (uint32_t)__builtin_amdgcn_readlane((int)start, la);
            for (int x = la + 1; x <= lb; ++x) {
              const uint32_t e = (uint32_t)__builtin_amdgcn_readlane((int)incl, x - 1);  // first record of run x
              const uint32_t sx = (uint32_t)__builtin_amdgcn_readlane((int)start, x);
              if (q >= e) st = sx;
            }
            if (q < total) recu = st + q;
          }
          rec[u] = recu;
        }
        // Every load of the R windows - bins and the first four attributes -
        // is issued before the first LDS update.
        constexpr int KV = sizeof(AT) == 8 ? 2 : 4;
        AT v[KV][R];
  #pragma unroll
        for (int u = 0; u < R; ++u)
          lb[u] = rec[u] != 0xFFFFFFFFu ? (int)a.rec_bin[rec[u]] : -1;
  #pragma unroll
        for (int jj = 0; jj < KV; ++jj)
          if (jj < k) {
  #pragma unroll
            for (int u = 0; u < R; ++u) v[jj][u] = rec[u] != 0xFFFFFFFFu ? ld_keep<AT>(a.rec_val[jj], rec[u]) : AT(0);
          }
        __builtin_amdgcn_s_setprio(0);
  #pragma unroll
        for (int u = 0; u < R; ++u)
          if (lb[u] >= 0) TL::count(smem, lb[u]);
  #pragma unroll
        for (int jj = 0; jj < KV; ++jj)
          if (jj < k) TL::template add_batch<R>(smem, a.lay, jj, lb, v[jj]);
        for (int jj = KV; jj < k; ++jj) {
          AT w[R];
  #pragma unroll
          for (int u = 0; u < R; ++u) w[u] = rec[u] != 0xFFFFFFFFu ? ld_keep<AT>(a.rec_val[jj], rec[u]) : AT(0);
          TL::template add_batch<R>(smem, a.lay, jj, lb, w);
        }
      }
    }
  }
  __syncthreads();
  if (a.tile_items[3 * t + 1] == 1u) {
    TL::emit_all(smem, a.lay, a.out, k, nbt, b0);
  } else {
    const uint32_t slot = a.tile_items[3 * t + 2] + (uint32_t)item - a.tile_items[3 * t];
    if (slot < (uint32_t)a.max_slots)  // proven bound; the guard only keeps stores in range
      TL::store_slot(smem, a.lay, k, nbt, static_cast<unsigned char*>(a.partial) + (int64_t)slot * a.lay.slot_bytes);
  }
}

// Workgroups are dispatched to the 8 XCDs round-robin; block b runs item
// (b % 8) * P + b / 8 with P = ceil(items / 8), so each XCD takes a
// contiguous range of tiles and neighbouring tiles' runs, which share cache
// lines, are read through the same L2.
template <typename AT, int PREC, bool QUAD>
__global__ __launch_bounds__(1024) void part_bin_kernel(PartArgs a) {
  const uint32_t n = *a.n_items;
  const uint32_t per = (n + 7) / 8;
  const uint32_t s = blockIdx.x / 8;
  if (s >= per) return;
  part_bin_body<AT, PREC, QUAD>(a, (int)((blockIdx.x % 8) * per + s));
}
// Batches: one gather form per launch (a group of requests that all pad
// their runs to quads, or none).
template <typename AT, int PREC, bool QUAD>
__global__ __launch_bounds__(1024) void part_bin_batched(const PartArgs* __restrict__ d,
                                                         const uint32_t* __restrict__ map) {
  const uint32_t m = map[blockIdx.x];
  if (m == 0xFFFFFFFFu) return;  // padding of the XCD-aware block order
  part_bin_body<AT, PREC, QUAD>(d[m >> 16], (int)(m & 0xFFFFu));
}

// Merge of split tiles: work unit u = (split tile, 1024-bin chunk), one bin
// per thread; merge_blocks workgroups stride over the units.
template <typename AT, int PREC>
__device__ __forceinline__ void part_merge_body(const PartArgs& a, int blk) {
  const uint32_t nsplit = a.split_list[a.ntiles];
  const int shift = a.lay.tile_shift;
  const int TB = 1 << shift;
  const uint32_t chunks = (uint32_t)((TB + 1023) >> 10);
  for (uint32_t u = blk; u < nsplit * chunks; u += (uint32_t)a.merge_blocks) {
    const uint32_t t = a.split_list[u / chunks];
    const int b = (int)(u % chunks) * 1024 + threadIdx.x;
    const uint32_t nit = a.tile_items[3 * t + 1];
    const uint32_t slot0 = a.tile_items[3 * t + 2];
    if (slot0 + nit > (uint32_t)a.max_slots) continue;  // cannot happen (proven bound)
    const int64_t b0 = (int64_t)t << shift;
    const int nbt = (int)((b0 + TB <= a.nbins) ? TB : a.nbins - b0);
    if (b < nbt)
      Tile<AT, PREC>::merge_emit(static_cast<const unsigned char*>(a.partial), a.lay.slot_bytes, slot0, nit, a.lay,
                                 a.out, a.k, b, b0 + b);
  }
}

template <typename AT, int PREC>
__global__ __launch_bounds__(1024) void part_merge_kernel(PartArgs a) {
  part_merge_body<AT, PREC>(a, blockIdx.x);
}
template <typename AT, int PREC>
__global__ __launch_bounds__(1024) void part_merge_batched(const PartArgs* __restrict__ d,
                                                           const uint32_t* __restrict__ map) {
  const uint32_t m = map[blockIdx.x];
  part_merge_body<AT, PREC>(d[m >> 16], (int)(m & 0xFFFFu));
}

// ---------------------------------------------------------------------------
// Launch sequences.
// ---------------------------------------------------------------------------
#define BK_LAUNCH(NAME, KERNEL, GRID, BLOCK, LDS, ...)                       \
  do {                                                                        \
    if ((GRID) > 0) {                                                         \
      if (tm) tm->begin(s);                                                   \
      hipLaunchKernelGGL(KERNEL, dim3(GRID), dim3(BLOCK), LDS, s, __VA_ARGS__); \
      if (tm) tm->end(NAME, s);                                               \
      if ((e = hipGetLastError()) != hipSuccess) return e;                    \
    }                                                                         \
  } while (0)

#define BK_SCATTER_SWITCH(KERNEL, GRID, ...)                                                  \
  switch (c.scatter_threads * 100 + c.ppt) {                                                  \
    BK_SC(KERNEL, GRID, 256, 4, __VA_ARGS__) BK_SC(KERNEL, GRID, 256, 8, __VA_ARGS__)         \
    BK_SC(KERNEL, GRID, 256, 16, __VA_ARGS__) BK_SC(KERNEL, GRID, 256, 32, __VA_ARGS__)       \
    BK_SC(KERNEL, GRID, 512, 4, __VA_ARGS__) BK_SC(KERNEL, GRID, 512, 8, __VA_ARGS__)         \
    BK_SC(KERNEL, GRID, 512, 16, __VA_ARGS__) BK_SC(KERNEL, GRID, 512, 32, __VA_ARGS__)       \
    BK_SC(KERNEL, GRID, 1024, 4, __VA_ARGS__) BK_SC(KERNEL, GRID, 1024, 8, __VA_ARGS__)       \
    BK_SC(KERNEL, GRID, 1024, 12, __VA_ARGS__) BK_SC(KERNEL, GRID, 1024, 16, __VA_ARGS__)     \
    default:                                                                                  \
      return hipErrorInvalidConfiguration;                                                    \
  }
#define BK_SC(KERNEL, GRID, NT, PPT, ...)                                                      \
  case NT * 100 + PPT:                                                                          \
    BK_LAUNCH("part_scatter_kernel", (KERNEL<CT, AT, PPT, NT>), GRID, NT, c.scatter_lds, __VA_ARGS__); \
    break;

template <typename CT, typename AT, int PREC>
static hipError_t launch_part_t(const PartArgs& a, const PartCfg& c, hipStream_t s, KTimer* tm) {
  hipError_t e;
  BK_SCATTER_SWITCH(part_scatter_kernel, a.nwg, a)
  BK_LAUNCH("part_items_walk_kernel", part_items_walk_kernel, (a.ntiles + 15) / 16, 1024, 0, a);
  BK_LAUNCH("part_items_kernel", part_items_kernel, 1, 1024, 0, a);
  if (a.quads)
    BK_LAUNCH("part_bin_kernel", (part_bin_kernel<AT, PREC, true>), (a.max_items + 7) / 8 * 8, c.bin_block, c.bin_lds,
              a);
  else
    BK_LAUNCH("part_bin_kernel", (part_bin_kernel<AT, PREC, false>), (a.max_items + 7) / 8 * 8, c.bin_block, c.bin_lds,
              a);
  BK_LAUNCH("part_merge_kernel", (part_merge_kernel<AT, PREC>), a.merge_blocks, 1024, 0, a);
  return hipSuccess;
}

template <typename CT, typename AT, int PREC>
static hipError_t launch_part_batch_t(const PartBatch& b, const PartCfg& c, hipStream_t s, KTimer* tm,
                                      bool scatter = true) {
  hipError_t e;
  if (scatter) {
    BK_SCATTER_SWITCH(part_scatter_batched, b.n_wg_blocks, b.descs, b.map_wg)
  }
  BK_LAUNCH("part_items_walk_kernel", part_items_walk_batched, b.n_walk_blocks, 1024, 0, b.descs, b.map_walk);
  BK_LAUNCH("part_items_kernel", part_items_batched, b.nreq, 1024, 0, b.descs);
  for (int q = 0; q < 4; ++q) {
    const int nb = b.cls_first[q + 1] - b.cls_first[q];
    if (c.quads)
      BK_LAUNCH("part_bin_kernel", (part_bin_batched<AT, PREC, true>), nb, b.cls_block[q], b.cls_lds[q], b.descs,
                b.map_item + b.cls_first[q]);
    else
      BK_LAUNCH("part_bin_kernel", (part_bin_batched<AT, PREC, false>), nb, b.cls_block[q], b.cls_lds[q], b.descs,
                b.map_item + b.cls_first[q]);
  }
  BK_LAUNCH("part_merge_kernel", (part_merge_batched<AT, PREC>), b.n_tile_blocks, 1024, 0, b.descs, b.map_tile);
  return hipSuccess;
}
#undef BK_SC
#undef BK_SCATTER_SWITCH

#define BK_PART_DISPATCH(FN, ...)                                              \
  if (coord_f64) {                                                             \
    if (attr_f64) return FN<double, double, PREC_F64>(__VA_ARGS__);            \
    switch (prec) {                                                            \
      case PREC_PLAIN: return FN<double, float, PREC_PLAIN>(__VA_ARGS__);      \
      case PREC_COMP: return FN<double, float, PREC_COMP>(__VA_ARGS__);        \
      default: return FN<double, float, PREC_F64>(__VA_ARGS__);                \
    }                                                                          \
  }                                                                            \
  if (attr_f64) return FN<float, double, PREC_F64>(__VA_ARGS__);               \
  switch (prec) {                                                              \
    case PREC_PLAIN: return FN<float, float, PREC_PLAIN>(__VA_ARGS__);         \
    case PREC_COMP: return FN<float, float, PREC_COMP>(__VA_ARGS__);           \
    default: return FN<float, float, PREC_F64>(__VA_ARGS__);                   \
  }

hipError_t launch_partition(const PartArgs& a, bool coord_f64, bool attr_f64, int prec, const PartCfg& c,
                            hipStream_t s, KTimer* tm) {
  BK_PART_DISPATCH(launch_part_t, a, c, s, tm)
}

hipError_t launch_partition_batch(const PartBatch& b, bool coord_f64, bool attr_f64, int prec, const PartCfg& c,
                                  hipStream_t s, KTimer* tm) {
  BK_PART_DISPATCH(launch_part_batch_t, b, c, s, tm)
}

hipError_t launch_partition_batch_after_scatter(const PartBatch& b, bool coord_f64, bool attr_f64, int prec,
                                                const PartCfg& c, hipStream_t s, KTimer* tm) {
  BK_PART_DISPATCH(launch_part_batch_t, b, c, s, tm, false)
}
#undef BK_PART_DISPATCH
#undef BK_LAUNCH

// ---------------------------------------------------------------------------
// Fused scatter of several grids over one table (MultiScatterArgs).  One
// workgroup of kMultiThreads per slice; per sub-chunk of kMultiSub
// particles the union of the columns is staged in LDS once (the first
// kMultiPrefetch columns of the next sub-chunk are read into registers while
// the grids of this one are processed).  The grids then go in groups of
// up to kMultiGroup: every thread ranks its particles within each grid's
// tiles, one wave per grid scans that grid's tile counts, the records' bins
// and source particles are placed in LDS in tile order (a stage per grid of
// the group), and each output column - the bins, then every attribute's
// values read from the staged columns through that permutation - is written
// back over the sub-chunk's own index range with 8- and 16-byte stores.  The
// layout, run table and per-slice counts are the single-grid scatter's; the
// particle table is read from HBM once for all grids.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kMultiThreads) void part_scatter_multi_kernel(const MultiScatterArgs* __restrict__ argp) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ uint32_t s_nsub[kMultiGroup];
  constexpr int NT = kMultiThreads;
  constexpr int S = kMultiSub;
  constexpr int PPT = S / NT;
  static_assert(S == 2 * NT, "each thread stages one pair of particles per column");
  typedef float f32x2 __attribute__((ext_vector_type(2)));
  const MultiScatterArgs& m = *argp;
  const int w = blockIdx.x;
  const PartArgs& a0 = m.grids[0];
  const int64_t lo = (int64_t)w * a0.chunk;
  const int64_t hi = lo + a0.chunk < a0.n ? lo + a0.chunk : a0.n;
  float* cols = reinterpret_cast<float*>(smem + m.cols_lds);
  for (int g = 0; g < m.ngrids; ++g) {
    const int T = m.grids[g].ntiles;
    uint32_t* c = reinterpret_cast<uint32_t*>(smem + m.grid_lds[g]);
    for (int t = threadIdx.x; t < 4 * T; t += NT) c[t] = 0u;  // cnt[2][T], off[T], tot[T]
  }
  // The first npf columns of a sub-chunk, a pair of particles per thread.
  const int npf = m.ncols < kMultiPrefetch ? m.ncols : kMultiPrefetch;
  f32x2 pf[kMultiPrefetch];
  auto fetch = [&](int64_t base) {
    const int len = hi - base < S ? (int)(hi - base) : S;
    const int p = 2 * threadIdx.x;
#pragma unroll
    for (int u = 0; u < kMultiPrefetch; ++u)
      if (u < npf) {
        const float* src = m.cols[u] + base;
        if (m.vec && p + 1 < len) {
          pf[u] = __builtin_nontemporal_load(reinterpret_cast<const f32x2*>(src + p));
        } else {
          pf[u].x = p < len ? __builtin_nontemporal_load(src + p) : 0.0f;
          pf[u].y = p + 1 < len ? __builtin_nontemporal_load(src + p + 1) : 0.0f;
        }
      }
  };
  if (lo < hi) fetch(lo);
  __syncthreads();
  const int nblocks = (int)((hi - lo + S - 1) / S);
  int j = 0;
  for (int64_t base = lo; base < hi; base += S, ++j) {
    const int len = hi - base < S ? (int)(hi - base) : S;
#pragma unroll
    for (int u = 0; u < kMultiPrefetch; ++u)
      if (u < npf) reinterpret_cast<f32x2*>(cols + (int64_t)u * S)[threadIdx.x] = pf[u];
    for (int u = npf; u < m.ncols; ++u) {
      const float* src = m.cols[u] + base;
      float* dst = cols + (int64_t)u * S;
      if (m.vec && len == S) {
        for (int q = threadIdx.x; q < S / 4; q += NT)
          reinterpret_cast<f32x4*>(dst)[q] = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(src) + q);
      } else {
        for (int p = threadIdx.x; p < S; p += NT) dst[p] = p < len ? __builtin_nontemporal_load(src + p) : 0.0f;
      }
    }
    __syncthreads();
    if (base + S < hi) fetch(base + S);  // in flight while the grids below run
    const int parity = j & 1;
    for (int g0 = 0; g0 < m.ngrids; g0 += m.group) {
      const int G = m.ngrids - g0 < m.group ? m.ngrids - g0 : m.group;
      // rank each particle within its tile, every grid of the group
      uint32_t tb[kMultiGroup][PPT], pos[kMultiGroup][PPT];
#pragma unroll
      for (int gi = 0; gi < kMultiGroup; ++gi) {
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
          tb[gi][q] = 0xFFFFFFFFu;
          pos[gi][q] = 0u;
        }
        if (gi < G) {
          const int g = g0 + gi;
          const PartArgs& a = m.grids[g];
          uint32_t* cnt = reinterpret_cast<uint32_t*>(smem + m.grid_lds[g]) + parity * a.ntiles;
          const int shift = a.lay.tile_shift;
          const uint32_t lmask = (1u << shift) - 1u;
          const float* xs = cols + (int64_t)m.gx[g] * S;
          const float* ys = cols + (int64_t)m.gy[g] * S;
          Axis ax = a.ax, ay = a.ay;
          resolve_axes(a.dyn, ax, ay);
#pragma unroll
          for (int q = 0; q < PPT; ++q) {
            const int p = q * NT + threadIdx.x;
            int ix, iy;
            if (p < len && locate((double)xs[p], ax, ix) && locate((double)ys[p], ay, iy)) {
              const uint32_t b = (uint32_t)(iy * a.nx + ix);
              tb[gi][q] = ((b >> shift) << 16) | (b & lmask);
              pos[gi][q] = atomicAdd(cnt + (tb[gi][q] >> 16), 1u);
            }
          }
        }
      }
      __syncthreads();
      // wave gi scans grid g0 + gi: lane l owns tiles [l * mt, l * mt + mt)
      const int wave = threadIdx.x >> 6;
      if (wave < G) {
        const int g = g0 + wave;
        const PartArgs& a = m.grids[g];
        const int T = a.ntiles;
        uint32_t* cbase = reinterpret_cast<uint32_t*>(smem + m.grid_lds[g]);
        uint32_t* cnt = cbase + parity * T;
        uint32_t* cprev = cbase + (parity ^ 1) * T;
        uint32_t* off = cbase + 2 * T;
        uint32_t* tot = off + T;
        const int lane = threadIdx.x & 63;
        const int mt = (T + 63) >> 6;
        const int t0 = lane * mt;
        const uint32_t padm = a.quads ? 3u : 0u;
        uint32_t own = 0;
        for (int q = 0; q < mt; ++q)
          if (t0 + q < T) own += (cnt[t0 + q] + padm) & ~padm;
        uint32_t x = own;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const uint32_t y = __shfl_up(x, o);
          if (lane >= o) x += y;
        }
        uint32_t o0 = x - own;
        for (int q = 0; q < mt; ++q) {
          const int t = t0 + q;
          if (t < T) {
            const uint32_t cc = (cnt[t] + padm) & ~padm;
            tot[t] += cc;
            cprev[t] = 0u;
            off[t] = o0;
            o0 += cc;
          }
        }
        if (lane == 63) s_nsub[wave] = x;
      }
      __syncthreads();
      // place the records in tile order: the local bin, and the particle
      // (its index in the sub-chunk) each slot takes its values from
#pragma unroll
      for (int gi = 0; gi < kMultiGroup; ++gi) {
        if (gi >= G) break;
        const int g = g0 + gi;
        const PartArgs& a = m.grids[g];
        const int T = a.ntiles;
        const uint32_t* cbase = reinterpret_cast<const uint32_t*>(smem + m.grid_lds[g]);
        const uint32_t* cnt = cbase + parity * T;
        const uint32_t* off = cbase + 2 * T;
        uint16_t* ost = reinterpret_cast<uint16_t*>(smem + m.grid_ost[g]);
        uint16_t* stg_b = reinterpret_cast<uint16_t*>(smem + m.stage + gi * 4 * S);
        uint16_t* perm = stg_b + S;
        const int F = 1 << a.off_shift;
        for (int t = threadIdx.x; t <= T; t += NT) {
          ost[(t << a.off_shift) + (j & (F - 1))] = (uint16_t)(t < T ? off[t] : s_nsub[gi]);
          if (a.quads && t < T) {  // pad the run to a whole quad (no particle: value 0)
            const uint32_t cc = cnt[t];
            const uint32_t e = off[t] + ((cc + 3u) & ~3u);
            for (uint32_t p = off[t] + cc; p < e; ++p) {
              stg_b[p] = 0xFFFFu;
              perm[p] = 0xFFFFu;
            }
          }
        }
#pragma unroll
        for (int q = 0; q < PPT; ++q)
          if (tb[gi][q] != 0xFFFFFFFFu) {
            const uint32_t p = pos[gi][q] + off[tb[gi][q] >> 16];
            stg_b[p] = (uint16_t)(tb[gi][q] & 0xFFFFu);
            perm[p] = (uint16_t)(q * NT + threadIdx.x);
          }
      }
      __syncthreads();
      // Write out the group's grids.  The next group's stages are filled
      // only after two more barriers, so no barrier follows.
      for (int gi = 0; gi < G; ++gi) {
        const int g = g0 + gi;
        const PartArgs& a = m.grids[g];
        const int T = a.ntiles;
        const uint16_t* ost = reinterpret_cast<const uint16_t*>(smem + m.grid_ost[g]);
        const uint16_t* stg_b = reinterpret_cast<const uint16_t*>(smem + m.stage + gi * 4 * S);
        const uint16_t* perm = stg_b + S;
        // run-table rows [j0, j] of the slice once F are staged or at its end
        const int F = 1 << a.off_shift;
        if (((j + 1) & (F - 1)) == 0 || j + 1 == nblocks) {
          const int j0 = j & ~(F - 1);
          const int f = j - j0 + 1;
          const int64_t nrows = (int64_t)a.nwg * a.nbpw;
          const int64_t r0 = (int64_t)w * a.nbpw + j0;
          for (int i2 = threadIdx.x; i2 < ((T + 1) << a.off_shift); i2 += NT) {
            const int t = i2 >> a.off_shift, jj = i2 & (F - 1);
            if (jj < f) a.blk_off[(int64_t)t * nrows + r0 + jj] = ost[i2];
          }
        }
        // One contiguous stream per output column, four records per thread.
        const uint32_t nsub = s_nsub[gi];
        const uint32_t nq = (nsub + 3u) >> 2;
        const int64_t rbase = base + ((int64_t)w * a.nbpw + j) * (int64_t)a.pad_row;
        const uint32_t nwork = (uint32_t)(a.k + 1) * nq;
        for (uint32_t i = threadIdx.x; i < nwork; i += NT) {
          const uint32_t c = i / nq;
          const uint32_t p = 4u * (i - c * nq);
          const uint32_t rem = nsub - p;  // records of this quad: 1..4 (p + 3 < S)
          const bool full = rem >= 4u;
          const u32x2 pp = *reinterpret_cast<const u32x2*>((c ? perm : stg_b) + p);
          if (c == 0) {
            uint16_t* rb = a.rec_bin + rbase + p;
            if (full && (reinterpret_cast<uintptr_t>(rb) & 7) == 0) {
              __builtin_nontemporal_store(pp, reinterpret_cast<u32x2*>(rb));
            } else {
              for (uint32_t e = 0; e < rem && e < 4u; ++e) rb[e] = stg_b[p + e];
            }
          } else {
            const float* vs = cols + (int64_t)m.attr_col[c - 1] * S;
            float* rv = static_cast<float*>(a.rec_val[c - 1]) + rbase + p;
            // slots past the sub-chunk's records hold stale entries: not read
            const uint32_t s0 = pp.x & 0xFFFFu, s1 = pp.x >> 16, s2 = pp.y & 0xFFFFu, s3 = pp.y >> 16;
            f32x4 v;
            v.x = s0 < (uint32_t)S ? vs[s0] : 0.0f;
            v.y = rem > 1u && s1 < (uint32_t)S ? vs[s1] : 0.0f;
            v.z = rem > 2u && s2 < (uint32_t)S ? vs[s2] : 0.0f;
            v.w = rem > 3u && s3 < (uint32_t)S ? vs[s3] : 0.0f;
            if (full && (reinterpret_cast<uintptr_t>(rv) & 15) == 0) {
              __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(rv));
            } else {
              const float ve[4] = {v.x, v.y, v.z, v.w};
              for (uint32_t e = 0; e < rem && e < 4u; ++e) rv[e] = ve[e];
            }
          }
        }
      }
    }
    __syncthreads();  // the staged columns are refilled by the next sub-chunk
  }
  for (int g = 0; g < m.ngrids; ++g) {
    const PartArgs& a = m.grids[g];
    const int T = a.ntiles;
    const uint32_t* tot = reinterpret_cast<const uint32_t*>(smem + m.grid_lds[g]) + 3 * T;
    for (int t = threadIdx.x; t < T; t += NT) a.counts[(int64_t)t * a.nwg + w] = tot[t];
  }
}

hipError_t launch_scatter_multi(const MultiScatterArgs* args, int nwg, size_t lds, hipStream_t s, KTimer* tm) {
  if (nwg <= 0) return hipSuccess;
  if (tm) tm->begin(s);
  hipLaunchKernelGGL(part_scatter_multi_kernel, dim3(nwg), dim3(kMultiThreads), lds, s, args);
  if (tm) tm->end("part_scatter_multi_kernel", s);
  return hipGetLastError();
}

hipError_t set_partition_lds_limit(size_t bytes) {
  hipError_t e = hipSuccess;
#define BK_SETF(...) \
  if (e == hipSuccess) e = set_dynamic_lds_limit(reinterpret_cast<const void*>(&__VA_ARGS__), bytes);
#define BK_SET_NT(K, CT, AT, NT) \
  BK_SETF(K<CT, AT, 4, NT>) BK_SETF(K<CT, AT, 8, NT>) BK_SETF(K<CT, AT, 16, NT>)
#define BK_SET_CA(K, CT, AT) \
  BK_SET_NT(K, CT, AT, 256) BK_SETF(K<CT, AT, 32, 256>) BK_SET_NT(K, CT, AT, 512) BK_SETF(K<CT, AT, 32, 512>) \
  BK_SET_NT(K, CT, AT, 1024) BK_SETF(K<CT, AT, 12, 1024>)
#define BK_SET_TYPES(K) \
  BK_SET_CA(K, float, float) BK_SET_CA(K, float, double) BK_SET_CA(K, double, float) BK_SET_CA(K, double, double)
  BK_SETF(part_scatter_multi_kernel)
  BK_SET_TYPES(part_scatter_kernel)
  BK_SET_TYPES(part_scatter_batched)
  BK_SETF(part_bin_kernel<float, PREC_F64, false>)
  BK_SETF(part_bin_kernel<float, PREC_COMP, false>)
  BK_SETF(part_bin_kernel<float, PREC_PLAIN, false>)
  BK_SETF(part_bin_kernel<double, PREC_F64, false>)
  BK_SETF(part_bin_kernel<float, PREC_F64, true>)
  BK_SETF(part_bin_kernel<float, PREC_COMP, true>)
  BK_SETF(part_bin_kernel<float, PREC_PLAIN, true>)
  BK_SETF(part_bin_kernel<double, PREC_F64, true>)
  BK_SETF(part_bin_batched<float, PREC_F64, false>)
  BK_SETF(part_bin_batched<float, PREC_COMP, false>)
  BK_SETF(part_bin_batched<float, PREC_PLAIN, false>)
  BK_SETF(part_bin_batched<double, PREC_F64, false>)
  BK_SETF(part_bin_batched<float, PREC_F64, true>)
  BK_SETF(part_bin_batched<float, PREC_COMP, true>)
  BK_SETF(part_bin_batched<float, PREC_PLAIN, true>)
  BK_SETF(part_bin_batched<double, PREC_F64, true>)
#undef BK_SET_TYPES
#undef BK_SET_CA
#undef BK_SET_NT
#undef BK_SETF
  return e;
}

}  // namespace bk
