// Partition strategy for grids too large for one LDS tile.
//
// Global atomics on gfx950 sustain only a few tens of G lane-ops/s across
// the whole device, while LDS atomics run two orders of magnitude faster, so
// large grids are binned without any per-particle global atomic:
//
//   part_count    per workgroup slice of particles: LDS histogram of tiles
//                 (a tile = TB consecutive flat bins, TB a power of two
//                 chosen so a tile's accumulators fill one LDS allocation);
//                 writes counts[tile][wg].
//   scan_*        exclusive scan of counts (tile-major) -> record offsets.
//   part_items    one work item per tile, heavy tiles split into items of at
//                 most L records; split tiles get partial slots.
//   part_scatter  re-reads the same slice, sorts each sub-chunk by tile in
//                 LDS and writes compact records (u16 local bin + attribute
//                 values) tile by tile, so stores are contiguous runs.
//   part_bin      one workgroup per item: LDS accumulators for the tile,
//                 then (single-item tile) the finished outputs - count, sum,
//                 min, max, avg - written once, or (split tile) a partial.
//   part_merge    combines the partials of split tiles into outputs.
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
// Block-wide exclusive scans.
// ---------------------------------------------------------------------------
// Generic block size; tmp: blockDim.x words of LDS.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* tmp, uint32_t* total) {
  const int t = threadIdx.x;
  tmp[t] = v;
  __syncthreads();
  for (int off = 1; off < (int)blockDim.x; off <<= 1) {
    const uint32_t add = t >= off ? tmp[t - off] : 0u;
    __syncthreads();
    tmp[t] += add;
    __syncthreads();
  }
  const uint32_t incl = tmp[t];
  *total = tmp[blockDim.x - 1];
  __syncthreads();
  return incl - v;
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
// Tile histogram of workgroup slice wg.
// ---------------------------------------------------------------------------
template <typename CT>
__device__ __forceinline__ void part_count_body(const PartArgs& a, int wg) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint32_t* h = reinterpret_cast<uint32_t*>(smem);
  Axis ax = a.ax, ay = a.ay;
  resolve_axes(a.dyn, ax, ay);
  const int T = a.ntiles;
  for (int t = threadIdx.x; t < T; t += blockDim.x) h[t] = 0u;
  __syncthreads();
  const int64_t lo = (int64_t)wg * a.chunk;
  const int64_t hi = lo + a.chunk < a.n ? lo + a.chunk : a.n;
  const int shift = a.lay.tile_shift;
  const bool vec = a.vec != 0;
  // Each lane takes groups of 4 consecutive particles (16-byte loads).
  constexpr int G = 4;
  const int64_t step = (int64_t)4 * G * blockDim.x;
  for (int64_t base = lo; base < hi; base += step) {
    CT xs[4 * G], ys[4 * G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int64_t i = base + 4 * ((int64_t)g * blockDim.x + threadIdx.x);
      ld4<CT>(a.x, i, hi, vec, xs + 4 * g);
      ld4<CT>(a.y, i, hi, vec, ys + 4 * g);
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int64_t i = base + 4 * ((int64_t)g * blockDim.x + threadIdx.x);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int ix, iy;
        if (i + e < hi && locate((double)xs[4 * g + e], ax, ix) && locate((double)ys[4 * g + e], ay, iy))
          atomicAdd(h + ((iy * a.nx + ix) >> shift), 1u);
      }
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < T; t += blockDim.x) a.counts[(int64_t)t * a.nwg + wg] = h[t];
}

template <typename CT>
__global__ __launch_bounds__(1024) void part_count_kernel(PartArgs a) {
  part_count_body<CT>(a, blockIdx.x);
}
template <typename CT>
__global__ __launch_bounds__(1024) void part_count_batched(const PartArgs* __restrict__ d,
                                                           const uint32_t* __restrict__ map) {
  const uint32_t m = map[blockIdx.x];
  part_count_body<CT>(d[m >> 16], (int)(m & 0xFFFFu));
}

// ---------------------------------------------------------------------------
// Exclusive scan of m u32 values in place (three launches).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void scan_block_sums_kernel(const uint32_t* v, int64_t m, int64_t per,
                                                               uint32_t* bsum) {
  __shared__ uint32_t red[1024];
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = lo + per < m ? lo + per : m;
  uint32_t s = 0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) s += v[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}

// One block: exclusive scan of nb block sums in place; total at bsum[nb].
__global__ __launch_bounds__(1024) void scan_top_kernel(uint32_t* bsum, int nb) {
  __shared__ uint32_t wave_tot[16];
  uint32_t carry = 0;
  for (int base = 0; base < nb; base += 1024) {
    const int i = base + threadIdx.x;
    uint32_t tot;
    const uint32_t ex = block_scan_excl<1024>(i < nb ? bsum[i] : 0u, wave_tot, tot);
    if (i < nb) bsum[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ __launch_bounds__(1024) void scan_apply_kernel(uint32_t* v, int64_t m, int64_t per,
                                                          const uint32_t* bsum) {
  __shared__ uint32_t wave_tot[16];
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = lo + per < m ? lo + per : m;
  uint32_t carry = bsum[blockIdx.x];
  for (int64_t base = lo; base < hi; base += 1024) {
    const int64_t i = base + threadIdx.x;
    uint32_t tot;
    const uint32_t ex = block_scan_excl<1024>(i < hi ? v[i] : 0u, wave_tot, tot);
    if (i < hi) v[i] = carry + ex;
    carry += tot;
  }
}

// ---------------------------------------------------------------------------
// Work items: one per tile, heavy tiles split into ranges of <= split_len.
// tile_items[3t] = first item, [3t+1] = items, [3t+2] = first partial slot
// (split tiles only).  counts[] holds the exclusive scan; *inside is the
// end of this request's records.  One block (1024 threads) per request.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void part_items_body(const PartArgs& a) {
  __shared__ uint32_t wave_tot[16];
  const uint32_t total = *a.inside;
  uint32_t carry = 0, scarry = 0;
  for (int base = 0; base < a.ntiles; base += 1024) {
    const int t = base + threadIdx.x;
    uint32_t start = 0, end = 0, ni = 0;
    if (t < a.ntiles) {
      start = a.counts[(int64_t)t * a.nwg];
      end = t + 1 < a.ntiles ? a.counts[(int64_t)(t + 1) * a.nwg] : total;
      const uint32_t c = end - start;
      ni = c == 0 ? 1u : (c + a.split_len - 1) / a.split_len;
    }
    uint32_t tot, stot;
    const uint32_t first = carry + block_scan_excl<1024>(ni, wave_tot, tot);
    const uint32_t slot0 = scarry + block_scan_excl<1024>(ni > 1 ? ni : 0u, wave_tot, stot);
    if (t < a.ntiles) {
      a.tile_items[3 * t] = first;
      a.tile_items[3 * t + 1] = ni;
      a.tile_items[3 * t + 2] = slot0;
      for (uint32_t q = 0; q < ni; ++q) {
        const uint32_t it = first + q;
        if (it >= (uint32_t)a.max_items) break;  // max_items is a proven upper bound
        const uint32_t b = start + q * a.split_len;
        a.items[3 * it] = (uint32_t)t;
        a.items[3 * it + 1] = b;
        a.items[3 * it + 2] = (end - b) < a.split_len ? end : b + a.split_len;
      }
    }
    carry += tot;
    scarry += stot;
  }
  if (threadIdx.x == 0) *a.n_items = carry < (uint32_t)a.max_items ? carry : (uint32_t)a.max_items;
}

__global__ __launch_bounds__(1024) void part_items_kernel(PartArgs a) { part_items_body(a); }
__global__ __launch_bounds__(1024) void part_items_batched(const PartArgs* __restrict__ d) {
  part_items_body(d[blockIdx.x]);
}

// ---------------------------------------------------------------------------
// Scatter: per sub-chunk of S = NT * PPT particles, rank each inside
// particle within its tile (LDS atomic), scan the tile counts, place records
// in LDS in tile order, then copy each tile's run to its global segment.
// Lane t takes the groups of 4 consecutive particles starting at
// base + 4 * (q * NT + t), q < PPT / 4.  Whole sub-chunks of an aligned
// request are read with 16-byte loads and no bounds tests, and the next
// one's coordinates are loaded while the current one is sorted and written;
// the remainder (and unaligned requests) take a bounds-tested path.
// Three barriers per sub-chunk: the tile counters are double-buffered, and
// one wave scans them, advances the run heads by the previous sub-chunk's
// counts and clears that buffer.
// LDS: cnt[2][T] | off[T] | delta[T] | run[T] | (tile << 16 | local bin)[S] |
//      values[k][S]
// ---------------------------------------------------------------------------
struct ScatterShared {
  uint32_t nsub;
};

template <typename CT, typename AT, int PPT, int NT, bool FULL>
__device__ __forceinline__ void scatter_sub(const PartArgs& a, unsigned char* smem, ScatterShared& sh,
                                            const Axis& ax, const Axis& ay, int64_t base, int64_t hi,
                                            int64_t full_end, int parity, CT* px, CT* py) {
  constexpr int S = NT * PPT;
  constexpr int Q = PPT / 4;
  const int T = a.ntiles;
  uint32_t* cnt = reinterpret_cast<uint32_t*>(smem) + parity * T;
  uint32_t* cprev = reinterpret_cast<uint32_t*>(smem) + (parity ^ 1) * T;
  uint32_t* off = reinterpret_cast<uint32_t*>(smem) + 2 * T;
  uint32_t* delta = off + T;
  uint32_t* run = delta + T;
  uint32_t* stg_tb = run + T;
  AT* stg_v = reinterpret_cast<AT*>(smem + a.stage_val_off);
  const int shift = a.lay.tile_shift;
  const uint32_t lmask = (1u << shift) - 1u;
  const int k = a.k;

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
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int64_t i = base + S + 4 * ((int64_t)q * NT + threadIdx.x);
        ld4v<CT>(a.x, i, px + 4 * q);
        ld4v<CT>(a.y, i, py + 4 * q);
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < 64) {  // one wave: lane l owns tiles [l * m, l * m + m)
    const int lane = threadIdx.x;
    const int m = (T + 63) >> 6;
    const int t0 = lane * m;
    uint32_t own = 0;
    for (int q = 0; q < m; ++q)
      if (t0 + q < T) own += cnt[t0 + q];
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
        const uint32_t c = cnt[t];
        const uint32_t r = run[t] + cprev[t];
        run[t] = r;
        cprev[t] = 0u;
        off[t] = o0;
        delta[t] = r - o0;
        o0 += c;
      }
    }
    if (lane == 63) sh.nsub = x;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    if (tb[u] == 0xFFFFFFFFu) continue;
    pos[u] += off[tb[u] >> 16];
    stg_tb[pos[u]] = tb[u];
  }
  for (int j = 0; j < k; ++j) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t i = base + 4 * ((int64_t)q * NT + threadIdx.x);
      AT v[4];
      if constexpr (FULL)
        ld4v<AT>(a.attr[j], i, v);
      else
        ld4<AT>(a.attr[j], i, hi, false, v);
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (tb[4 * q + e] != 0xFFFFFFFFu) stg_v[(int64_t)j * S + pos[4 * q + e]] = v[e];
    }
  }
  __syncthreads();
  // Consecutive p of one tile go to consecutive record addresses.
  const uint32_t nsub = sh.nsub;
  for (uint32_t p = threadIdx.x; p < nsub; p += NT) {
    const uint32_t v = stg_tb[p];
    const uint32_t dst = delta[v >> 16] + p;
    a.rec_bin[dst] = (uint16_t)(v & 0xFFFFu);
    for (int j = 0; j < k; ++j) static_cast<AT*>(a.rec_val[j])[dst] = stg_v[(int64_t)j * S + p];
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
  uint32_t* run = cnt + 4 * T;
  Axis ax = a.ax, ay = a.ay;
  resolve_axes(a.dyn, ax, ay);
  for (int t = threadIdx.x; t < T; t += NT) {
    cnt[t] = 0u;
    cnt[T + t] = 0u;
    run[t] = a.counts[(int64_t)t * a.nwg + wg];
  }
  const int64_t lo = (int64_t)wg * a.chunk;
  const int64_t hi = lo + a.chunk < a.n ? lo + a.chunk : a.n;
  const int64_t full_end = a.vec ? lo + (hi - lo) / S * S : lo;
  CT px[PPT], py[PPT];
  if (lo < full_end) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t i = lo + 4 * ((int64_t)q * NT + threadIdx.x);
      ld4v<CT>(a.x, i, px + 4 * q);
      ld4v<CT>(a.y, i, py + 4 * q);
    }
  }
  __syncthreads();
  int parity = 0;
  for (int64_t base = lo; base < full_end; base += S, parity ^= 1)
    scatter_sub<CT, AT, PPT, NT, true>(a, smem, sh, ax, ay, base, hi, full_end, parity, px, py);
  for (int64_t base = full_end; base < hi; base += S, parity ^= 1) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int64_t i = base + 4 * ((int64_t)q * NT + threadIdx.x);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        px[4 * q + e] = i + e < hi ? ld<CT>(a.x, i + e) : CT(0);
        py[4 * q + e] = i + e < hi ? ld<CT>(a.y, i + e) : CT(0);
      }
    }
    scatter_sub<CT, AT, PPT, NT, false>(a, smem, sh, ax, ay, base, hi, full_end, parity, px, py);
  }
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
// Per-item tile binning; fused finalize for tiles binned by one item.
// ---------------------------------------------------------------------------
template <typename AT, int PREC>
__device__ __forceinline__ void part_bin_body(const PartArgs& a, int item) {
  using TL = Tile<AT, PREC>;
  extern __shared__ __align__(16) unsigned char smem[];
  if (item >= (int)*a.n_items) return;
  const uint32_t t = a.items[3 * item];
  const uint32_t rb = a.items[3 * item + 1];
  const uint32_t re = a.items[3 * item + 2];
  const int shift = a.lay.tile_shift;
  const int64_t b0 = (int64_t)t << shift;
  const int TB = 1 << shift;
  const int nbt = (int)((b0 + TB <= a.nbins) ? TB : a.nbins - b0);
  const int k = a.k;
  TL::init(smem, a.lay, k);
  __syncthreads();

  // Groups of 4 consecutive records from rb rounded down to a multiple of 4
  // (record arrays are 256-byte aligned): 8-byte bin and 16-byte value loads.
  constexpr int G = 2;
  const uint32_t r0 = rb & ~3u;
  for (uint32_t base = r0; base < re; base += 4 * G * blockDim.x) {
    uint32_t lb[4 * G];
    bool full[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const uint32_t r = base + 4 * (g * blockDim.x + threadIdx.x);
      full[g] = r >= rb && r + 4 <= re;
      if (full[g]) {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        const u32x2 w = __builtin_nontemporal_load(reinterpret_cast<const u32x2*>(a.rec_bin + r));
        lb[4 * g] = w.x & 0xFFFFu;
        lb[4 * g + 1] = w.x >> 16;
        lb[4 * g + 2] = w.y & 0xFFFFu;
        lb[4 * g + 3] = w.y >> 16;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          lb[4 * g + e] = (r + e >= rb && r + e < re) ? (uint32_t)__builtin_nontemporal_load(a.rec_bin + r + e)
                                                      : 0xFFFFFFFFu;
      }
    }
#pragma unroll
    for (int u = 0; u < 4 * G; ++u)
      if (lb[u] != 0xFFFFFFFFu) TL::count(smem, (int)lb[u]);
    for (int j = 0; j < k; ++j) {
      AT v[4 * G];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const uint32_t r = base + 4 * (g * blockDim.x + threadIdx.x);
        if (full[g]) {
          ld4<AT>(a.rec_val[j], r, re, true, v + 4 * g);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            v[4 * g + e] = lb[4 * g + e] != 0xFFFFFFFFu ? ld<AT>(a.rec_val[j], r + e) : AT(0);
        }
      }
#pragma unroll
      for (int u = 0; u < 4 * G; ++u)
        if (lb[u] != 0xFFFFFFFFu) TL::add(smem, a.lay, j, (int)lb[u], v[u]);
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

template <typename AT, int PREC>
__global__ __launch_bounds__(1024) void part_bin_kernel(PartArgs a) {
  part_bin_body<AT, PREC>(a, blockIdx.x);
}
template <typename AT, int PREC>
__global__ __launch_bounds__(1024) void part_bin_batched(const PartArgs* __restrict__ d,
                                                         const uint32_t* __restrict__ map) {
  const uint32_t m = map[blockIdx.x];
  part_bin_body<AT, PREC>(d[m >> 16], (int)(m & 0xFFFFu));
}

// One block per tile; only split tiles do work.
template <typename AT, int PREC>
__device__ __forceinline__ void part_merge_body(const PartArgs& a, int t) {
  const uint32_t nit = a.tile_items[3 * t + 1];
  if (nit <= 1) return;
  const uint32_t slot0 = a.tile_items[3 * t + 2];
  if (slot0 + nit > (uint32_t)a.max_slots) return;  // cannot happen (proven bound)
  const int shift = a.lay.tile_shift;
  const int64_t b0 = (int64_t)t << shift;
  const int TB = 1 << shift;
  const int nbt = (int)((b0 + TB <= a.nbins) ? TB : a.nbins - b0);
  for (int b = threadIdx.x; b < nbt; b += blockDim.x)
    Tile<AT, PREC>::merge_emit(static_cast<const unsigned char*>(a.partial), a.lay.slot_bytes, slot0, nit, a.lay,
                               a.out, a.k, b, b0 + b);
}

template <typename AT, int PREC>
__global__ __launch_bounds__(256) void part_merge_kernel(PartArgs a) {
  part_merge_body<AT, PREC>(a, blockIdx.x);
}
template <typename AT, int PREC>
__global__ __launch_bounds__(256) void part_merge_batched(const PartArgs* __restrict__ d,
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
    BK_SC(KERNEL, GRID, 1024, 16, __VA_ARGS__)                                                \
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
  BK_LAUNCH("part_count_kernel", (part_count_kernel<CT>), a.nwg, 1024, c.count_lds, a);
  const int64_t m = (int64_t)a.ntiles * a.nwg;
  BK_LAUNCH("scan_block_sums_kernel", scan_block_sums_kernel, c.scan_blocks, 1024, 0, a.counts, m, c.scan_per,
            a.bsum);
  BK_LAUNCH("scan_top_kernel", scan_top_kernel, 1, 1024, 0, a.bsum, c.scan_blocks);
  BK_LAUNCH("scan_apply_kernel", scan_apply_kernel, c.scan_blocks, 1024, 0, a.counts, m, c.scan_per, a.bsum);
  BK_LAUNCH("part_items_kernel", part_items_kernel, 1, 1024, 0, a);
  BK_SCATTER_SWITCH(part_scatter_kernel, a.nwg, a)
  BK_LAUNCH("part_bin_kernel", (part_bin_kernel<AT, PREC>), a.max_items, c.bin_block, c.bin_lds, a);
  BK_LAUNCH("part_merge_kernel", (part_merge_kernel<AT, PREC>), a.ntiles, 256, 0, a);
  return hipSuccess;
}

template <typename CT, typename AT, int PREC>
static hipError_t launch_part_batch_t(const PartBatch& b, const PartCfg& c, hipStream_t s, KTimer* tm) {
  hipError_t e;
  BK_LAUNCH("part_count_kernel", (part_count_batched<CT>), b.n_wg_blocks, 1024, c.count_lds, b.descs,
            b.map_wg);
  BK_LAUNCH("scan_block_sums_kernel", scan_block_sums_kernel, c.scan_blocks, 1024, 0, b.counts, b.m, c.scan_per,
            b.bsum);
  BK_LAUNCH("scan_top_kernel", scan_top_kernel, 1, 1024, 0, b.bsum, c.scan_blocks);
  BK_LAUNCH("scan_apply_kernel", scan_apply_kernel, c.scan_blocks, 1024, 0, b.counts, b.m, c.scan_per, b.bsum);
  BK_LAUNCH("part_items_kernel", part_items_batched, b.nreq, 1024, 0, b.descs);
  BK_SCATTER_SWITCH(part_scatter_batched, b.n_wg_blocks, b.descs, b.map_wg)
  BK_LAUNCH("part_bin_kernel", (part_bin_batched<AT, PREC>), b.n_item_blocks, c.bin_block, c.bin_lds, b.descs,
            b.map_item);
  BK_LAUNCH("part_merge_kernel", (part_merge_batched<AT, PREC>), b.n_tile_blocks, 256, 0, b.descs, b.map_tile);
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
#undef BK_PART_DISPATCH
#undef BK_LAUNCH

hipError_t set_partition_lds_limit(size_t bytes) {
  hipError_t e = hipSuccess;
#define BK_SETF(...) \
  if (e == hipSuccess) e = set_dynamic_lds_limit(reinterpret_cast<const void*>(&__VA_ARGS__), bytes);
#define BK_SET_NT(K, CT, AT, NT) \
  BK_SETF(K<CT, AT, 4, NT>) BK_SETF(K<CT, AT, 8, NT>) BK_SETF(K<CT, AT, 16, NT>)
#define BK_SET_CA(K, CT, AT) \
  BK_SET_NT(K, CT, AT, 256) BK_SETF(K<CT, AT, 32, 256>) BK_SET_NT(K, CT, AT, 512) BK_SETF(K<CT, AT, 32, 512>) \
  BK_SET_NT(K, CT, AT, 1024)
#define BK_SET_TYPES(K) \
  BK_SET_CA(K, float, float) BK_SET_CA(K, float, double) BK_SET_CA(K, double, float) BK_SET_CA(K, double, double)
  BK_SETF(part_count_kernel<float>)
  BK_SETF(part_count_kernel<double>)
  BK_SETF(part_count_batched<float>)
  BK_SETF(part_count_batched<double>)
  BK_SET_TYPES(part_scatter_kernel)
  BK_SET_TYPES(part_scatter_batched)
  BK_SETF(part_bin_kernel<float, PREC_F64>)
  BK_SETF(part_bin_kernel<float, PREC_COMP>)
  BK_SETF(part_bin_kernel<float, PREC_PLAIN>)
  BK_SETF(part_bin_kernel<double, PREC_F64>)
  BK_SETF(part_bin_batched<float, PREC_F64>)
  BK_SETF(part_bin_batched<float, PREC_COMP>)
  BK_SETF(part_bin_batched<float, PREC_PLAIN>)
  BK_SETF(part_bin_batched<double, PREC_F64>)
#undef BK_SET_TYPES
#undef BK_SET_CA
#undef BK_SET_NT
#undef BK_SETF
  return e;
}

}  // namespace bk
