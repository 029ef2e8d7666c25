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
//                 most L records.
//   part_scatter  re-reads the same slice, sorts each sub-chunk by tile in
//                 LDS and writes compact records (u16 local bin + attribute
//                 values) tile by tile, so stores are contiguous runs.
//   part_bin      one workgroup per item: LDS accumulators for the tile,
//                 then (single-item tile) the finished outputs - count, sum,
//                 min, max, avg - written once, or (split tile) a partial.
//   part_merge    combines the partials of split tiles into outputs.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"
#include "kernels.h"

namespace bk {

// ---------------------------------------------------------------------------
// Tile histogram.
// ---------------------------------------------------------------------------
template <typename CT>
__global__ __launch_bounds__(1024) void part_count_kernel(PartArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint32_t* h = reinterpret_cast<uint32_t*>(smem);
  Axis ax = a.ax, ay = a.ay;
  resolve_axes(a.dyn, ax, ay);
  for (int t = threadIdx.x; t < a.ntiles; t += blockDim.x) h[t] = 0u;
  __syncthreads();
  const int64_t lo = (int64_t)blockIdx.x * a.chunk;
  const int64_t hi = lo + a.chunk < a.n ? lo + a.chunk : a.n;
  const int shift = a.lay.tile_shift;
  constexpr int U = 4;
  for (int64_t base = lo; base < hi; base += (int64_t)U * blockDim.x) {
    double xs[U], ys[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = base + (int64_t)u * blockDim.x + threadIdx.x;
      xs[u] = i < hi ? (double)ld<CT>(a.x, i) : __builtin_nan("");
      ys[u] = i < hi ? (double)ld<CT>(a.y, i) : __builtin_nan("");
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int ix, iy;
      if (locate(xs[u], ax, ix) && locate(ys[u], ay, iy)) atomicAdd(h + ((iy * a.nx + ix) >> shift), 1u);
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < a.ntiles; t += blockDim.x) a.counts[(int64_t)t * a.nwg + blockIdx.x] = h[t];
}

// ---------------------------------------------------------------------------
// Exclusive scan of m u32 values in place (three launches).
// ---------------------------------------------------------------------------
// Block-wide exclusive scan of one value per thread (tmp: blockDim.x words
// of LDS).  Called by every thread of the block.
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
  __shared__ uint32_t tmp[1024];
  uint32_t carry = 0;
  for (int base = 0; base < nb; base += blockDim.x) {
    const int i = base + threadIdx.x;
    const uint32_t v = i < nb ? bsum[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(v, tmp, &tot);
    if (i < nb) bsum[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ __launch_bounds__(1024) void scan_apply_kernel(uint32_t* v, int64_t m, int64_t per,
                                                          const uint32_t* bsum) {
  __shared__ uint32_t tmp[1024];
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = lo + per < m ? lo + per : m;
  uint32_t carry = bsum[blockIdx.x];
  for (int64_t base = lo; base < hi; base += blockDim.x) {
    const int64_t i = base + threadIdx.x;
    const uint32_t x = i < hi ? v[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(x, tmp, &tot);
    if (i < hi) v[i] = carry + ex;
    carry += tot;
  }
}

// ---------------------------------------------------------------------------
// Work items: one per tile, heavy tiles split into ranges of <= split_len.
// One block.  counts[] already holds the exclusive scan; *inside = total.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void part_items_kernel(PartArgs a) {
  __shared__ uint32_t tmp[1024];
  const uint32_t total = *a.inside;
  uint32_t carry = 0;
  for (int base = 0; base < a.ntiles; base += blockDim.x) {
    const int t = base + threadIdx.x;
    uint32_t start = 0, end = 0, ni = 0;
    if (t < a.ntiles) {
      start = a.counts[(int64_t)t * a.nwg];
      end = t + 1 < a.ntiles ? a.counts[(int64_t)(t + 1) * a.nwg] : total;
      const uint32_t c = end - start;
      ni = c == 0 ? 1u : (c + a.split_len - 1) / a.split_len;
    }
    uint32_t tot;
    const uint32_t first = carry + block_exclusive_scan(ni, tmp, &tot);
    if (t < a.ntiles) {
      a.tile_items[2 * t] = first;
      a.tile_items[2 * t + 1] = ni;
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
  }
  if (threadIdx.x == 0) *a.n_items = carry < (uint32_t)a.max_items ? carry : (uint32_t)a.max_items;
}

// ---------------------------------------------------------------------------
// Scatter: per sub-chunk of S = blockDim * PPT particles, rank each inside
// particle within its tile (LDS atomic), scan the tile counts, place records
// in LDS in tile order, then copy each tile's run to its global segment.
// LDS: cnt[T] | off[T] | run[T] | (tile << 16 | local bin)[S] | values[k][S]
// ---------------------------------------------------------------------------
template <typename CT, typename AT, int PPT>
__global__ __launch_bounds__(512) void part_scatter_kernel(PartArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ uint32_t scan_tmp[512];
  const int T = a.ntiles;
  const int S = blockDim.x * PPT;
  uint32_t* cnt = reinterpret_cast<uint32_t*>(smem);
  uint32_t* off = cnt + T;
  uint32_t* run = off + T;
  uint32_t* stg_tb = run + T;
  AT* stg_v = reinterpret_cast<AT*>(smem + a.stage_val_off);
  Axis ax = a.ax, ay = a.ay;
  resolve_axes(a.dyn, ax, ay);

  for (int t = threadIdx.x; t < T; t += blockDim.x) {
    cnt[t] = 0u;
    run[t] = a.counts[(int64_t)t * a.nwg + blockIdx.x];
  }
  __syncthreads();
  const int64_t lo = (int64_t)blockIdx.x * a.chunk;
  const int64_t hi = lo + a.chunk < a.n ? lo + a.chunk : a.n;
  const int shift = a.lay.tile_shift;
  const uint32_t lmask = (1u << shift) - 1u;
  for (int64_t base = lo; base < hi; base += S) {
    uint32_t tb[PPT], rank[PPT];
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
      const int64_t i = base + (int64_t)u * blockDim.x + threadIdx.x;
      tb[u] = 0xFFFFFFFFu;
      rank[u] = 0u;
      if (i < hi) {
        int ix, iy;
        const double x = (double)ld<CT>(a.x, i);
        const double y = (double)ld<CT>(a.y, i);
        if (locate(x, ax, ix) && locate(y, ay, iy)) {
          const uint32_t b = (uint32_t)(iy * a.nx + ix);
          tb[u] = ((b >> shift) << 16) | (b & lmask);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < PPT; ++u)
      if (tb[u] != 0xFFFFFFFFu) rank[u] = atomicAdd(cnt + (tb[u] >> 16), 1u);
    __syncthreads();
    uint32_t carry = 0;
    for (int t0 = 0; t0 < T; t0 += blockDim.x) {
      const int t = t0 + threadIdx.x;
      const uint32_t c = t < T ? cnt[t] : 0u;
      uint32_t tot;
      const uint32_t ex = block_exclusive_scan(c, scan_tmp, &tot);
      if (t < T) off[t] = carry + ex;
      carry += tot;
    }
    const uint32_t nsub = carry;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
      if (tb[u] == 0xFFFFFFFFu) continue;
      const uint32_t p = off[tb[u] >> 16] + rank[u];
      stg_tb[p] = tb[u];
      const int64_t i = base + (int64_t)u * blockDim.x + threadIdx.x;
      for (int j = 0; j < a.k; ++j) stg_v[(int64_t)j * S + p] = ld<AT>(a.attr[j], i);
    }
    __syncthreads();
    // Consecutive p of one tile go to consecutive record addresses.
    for (uint32_t p = threadIdx.x; p < nsub; p += blockDim.x) {
      const uint32_t v = stg_tb[p];
      const uint32_t t = v >> 16;
      const uint32_t dst = run[t] + (p - off[t]);
      a.rec_bin[dst] = (uint16_t)(v & 0xFFFFu);
      for (int j = 0; j < a.k; ++j) static_cast<AT*>(a.rec_val[j])[dst] = stg_v[(int64_t)j * S + p];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < T; t += blockDim.x) {
      run[t] += cnt[t];
      cnt[t] = 0u;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Per-item tile binning; fused finalize for tiles binned by one item.
// ---------------------------------------------------------------------------
template <typename AT, int PREC>
__global__ __launch_bounds__(1024) void part_bin_kernel(PartArgs a) {
  using TL = Tile<AT, PREC>;
  extern __shared__ __align__(16) unsigned char smem[];
  const int item = blockIdx.x;
  if (item >= (int)*a.n_items) return;
  const uint32_t t = a.items[3 * item];
  const uint32_t rb = a.items[3 * item + 1];
  const uint32_t re = a.items[3 * item + 2];
  const int shift = a.lay.tile_shift;
  const int64_t b0 = (int64_t)t << shift;
  const int TB = 1 << shift;
  const int nbt = (int)((b0 + TB <= a.nbins) ? TB : a.nbins - b0);
  TL::init(smem, a.lay, a.k);
  __syncthreads();

  constexpr int U = 4;
  for (uint32_t base = rb; base < re; base += U * blockDim.x) {
    uint32_t lb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t r = base + u * blockDim.x + threadIdx.x;
      lb[u] = r < re ? (uint32_t)__builtin_nontemporal_load(a.rec_bin + r) : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (lb[u] != 0xFFFFFFFFu) TL::count(smem, (int)lb[u]);
    for (int j = 0; j < a.k; ++j) {
      AT v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const uint32_t r = base + u * blockDim.x + threadIdx.x;
        v[u] = lb[u] != 0xFFFFFFFFu ? __builtin_nontemporal_load(static_cast<const AT*>(a.rec_val[j]) + r) : AT(0);
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (lb[u] != 0xFFFFFFFFu) TL::add(smem, a.lay, j, (int)lb[u], v[u]);
    }
  }
  __syncthreads();
  if (a.tile_items[2 * t + 1] == 1u)
    TL::emit_all(smem, a.lay, a.out, a.k, nbt, b0);
  else
    TL::store_slot(smem, a.lay, a.k, nbt, static_cast<unsigned char*>(a.partial) + (int64_t)item * a.lay.slot_bytes);
}

// One block per tile; only split tiles do work.
template <typename AT, int PREC>
__global__ __launch_bounds__(256) void part_merge_kernel(PartArgs a) {
  const int t = blockIdx.x;
  const uint32_t first = a.tile_items[2 * t];
  const uint32_t nit = a.tile_items[2 * t + 1];
  if (nit <= 1) return;
  const int shift = a.lay.tile_shift;
  const int64_t b0 = (int64_t)t << shift;
  const int TB = 1 << shift;
  const int nbt = (int)((b0 + TB <= a.nbins) ? TB : a.nbins - b0);
  for (int b = threadIdx.x; b < nbt; b += blockDim.x)
    Tile<AT, PREC>::merge_emit(static_cast<const unsigned char*>(a.partial), a.lay.slot_bytes, first, nit, a.lay,
                               a.out, a.k, b, b0 + b);
}

// ---------------------------------------------------------------------------
// Launch sequence.
// ---------------------------------------------------------------------------
#define BK_LAUNCH(NAME, KERNEL, GRID, BLOCK, LDS, ...)                 \
  do {                                                                  \
    if (tm) tm->begin(s);                                               \
    hipLaunchKernelGGL(KERNEL, dim3(GRID), dim3(BLOCK), LDS, s, __VA_ARGS__); \
    if (tm) tm->end(NAME, s);                                           \
    if ((e = hipGetLastError()) != hipSuccess) return e;                \
  } while (0)

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
  switch (c.ppt) {
    case 16: BK_LAUNCH("part_scatter_kernel", (part_scatter_kernel<CT, AT, 16>), a.nwg, 512, c.scatter_lds, a); break;
    case 8: BK_LAUNCH("part_scatter_kernel", (part_scatter_kernel<CT, AT, 8>), a.nwg, 512, c.scatter_lds, a); break;
    default: BK_LAUNCH("part_scatter_kernel", (part_scatter_kernel<CT, AT, 4>), a.nwg, 512, c.scatter_lds, a); break;
  }
  BK_LAUNCH("part_bin_kernel", (part_bin_kernel<AT, PREC>), a.max_items, c.bin_block, c.bin_lds, a);
  BK_LAUNCH("part_merge_kernel", (part_merge_kernel<AT, PREC>), a.ntiles, 256, 0, a);
  return hipSuccess;
}
#undef BK_LAUNCH

hipError_t launch_partition(const PartArgs& a, bool coord_f64, bool attr_f64, int prec, const PartCfg& c,
                            hipStream_t s, KTimer* tm) {
  if (coord_f64) {
    if (attr_f64) return launch_part_t<double, double, PREC_F64>(a, c, s, tm);
    switch (prec) {
      case PREC_PLAIN: return launch_part_t<double, float, PREC_PLAIN>(a, c, s, tm);
      case PREC_COMP: return launch_part_t<double, float, PREC_COMP>(a, c, s, tm);
      default: return launch_part_t<double, float, PREC_F64>(a, c, s, tm);
    }
  }
  if (attr_f64) return launch_part_t<float, double, PREC_F64>(a, c, s, tm);
  switch (prec) {
    case PREC_PLAIN: return launch_part_t<float, float, PREC_PLAIN>(a, c, s, tm);
    case PREC_COMP: return launch_part_t<float, float, PREC_COMP>(a, c, s, tm);
    default: return launch_part_t<float, float, PREC_F64>(a, c, s, tm);
  }
}

hipError_t set_partition_lds_limit(size_t bytes) {
  hipError_t e = hipSuccess;
#define BK_SETF(...) \
  if (e == hipSuccess) e = set_dynamic_lds_limit(reinterpret_cast<const void*>(&__VA_ARGS__), bytes);
#define BK_SET_CA(CT, AT)                   \
  BK_SETF(part_scatter_kernel<CT, AT, 4>)   \
  BK_SETF(part_scatter_kernel<CT, AT, 8>)   \
  BK_SETF(part_scatter_kernel<CT, AT, 16>)
  BK_SETF(part_count_kernel<float>)
  BK_SETF(part_count_kernel<double>)
  BK_SET_CA(float, float)
  BK_SET_CA(float, double)
  BK_SET_CA(double, float)
  BK_SET_CA(double, double)
  BK_SETF(part_bin_kernel<float, PREC_F64>)
  BK_SETF(part_bin_kernel<float, PREC_COMP>)
  BK_SETF(part_bin_kernel<float, PREC_PLAIN>)
  BK_SETF(part_bin_kernel<double, PREC_F64>)
#undef BK_SET_CA
#undef BK_SETF
  return e;
}

}  // namespace bk
