// HIP kernels (gfx950) for 2D particle data binning: global-atomic and
// whole-grid-in-LDS strategies.  (The partition strategy for large grids is
// in partition.hip.)
//
// The computation is the per-bin scatter-reduction of Section 4.2 of the
// paper: locate the mesh cell of every particle from two coordinate columns,
// then count particles per cell and reduce the attribute columns by sum, min,
// max and average.  Races between threads on one bin need atomic updates
// (Section 4.4).  On gfx950 those are cheap in LDS and expensive in device
// memory, so:
//
//  * bin_lds_kernel: each workgroup privatises the whole grid in LDS, bins a
//    contiguous slice of the particles with LDS atomics, then writes either
//    the finished outputs (one workgroup) or its partial accumulators to a
//    slot; lds_merge_kernel combines the slots with plain loads and stores.
//  * bin_global_kernel: grid-stride loop with device-scope atomics straight
//    into the result grids (only for very sparse requests: few particles on
//    a huge grid), between bin_init_kernel (identities) and
//    bin_finalize_kernel (binary64 S + C sums and averages).
//
// Compiled with -ffp-contract=off: the binary64 index and the TwoSum error
// term must be evaluated exactly as written.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"
#include "kernels.h"
#include "lds_body.h"

namespace bk {

// ---------------------------------------------------------------------------
// Global-atomic strategy.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void bin_init_kernel(InitArgs a) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < a.nbins; b += stride) {
    if (a.cnt) a.cnt[b] = 0u;
    for (int j = 0; j < a.k; ++j) {
      const AccPtrs& p = a.acc[j];
      if (p.sum) {
        if (p.sum_is_f64) static_cast<double*>(p.sum)[b] = 0.0;
        else static_cast<float*>(p.sum)[b] = 0.0f;
      }
      if (p.comp) p.comp[b] = 0.0f;
      if (p.mn) {
        if (p.minmax_f64) static_cast<uint64_t*>(p.mn)[b] = 0x7FF0000000000000ull;  // +Inf
        else static_cast<uint32_t*>(p.mn)[b] = 0x7F800000u;
      }
      if (p.mx) {
        if (p.minmax_f64) static_cast<uint64_t*>(p.mx)[b] = 0xFFF0000000000000ull;  // -Inf
        else static_cast<uint32_t*>(p.mx)[b] = 0xFF800000u;
      }
    }
  }
}

template <typename AT, int PREC>
__device__ __forceinline__ void global_update(const AccPtrs& p, int b, AT v) {
  if (p.sum) {
    if constexpr (PREC == PREC_F64) {
      atomicAdd(static_cast<double*>(p.sum) + b, (double)v);
    } else if constexpr (PREC == PREC_PLAIN) {
      atomicAdd(static_cast<float*>(p.sum) + b, (float)v);
    } else {  // compensated FP32: the returning add gives the old value
      const float fv = (float)v;
      const float old = atomicAdd(static_cast<float*>(p.sum) + b, fv);
      const float e = two_sum_err(old, fv, old + fv);
      if (e != 0.0f) atomicAdd(p.comp + b, e);
    }
  }
  using I = typename KeyOf<AT>::T;
  if (p.mn && beats_min<AT, I>(static_cast<AT*>(p.mn) + b, v)) atomic_min_fp(static_cast<AT*>(p.mn) + b, v);
  if (p.mx && beats_max<AT, I>(static_cast<AT*>(p.mx) + b, v)) atomic_max_fp(static_cast<AT*>(p.mx) + b, v);
}

template <typename CT, typename AT, int PREC, int PPT>
__global__ __launch_bounds__(1024) void bin_global_kernel(BinArgs a) {
  Axis ax = a.ax, ay = a.ay;
  resolve_axes(a.dyn, ax, ay);
  const int64_t tile = (int64_t)blockDim.x * PPT;
  const int64_t step = (int64_t)gridDim.x * tile;
  for (int64_t base = (int64_t)blockIdx.x * tile; base < a.n; base += step) {
    int bin[PPT];
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
      const int64_t i = base + (int64_t)u * blockDim.x + threadIdx.x;
      bin[u] = -1;
      if (i < a.n) {
        int ix, iy;
        const double x = (double)ld<CT>(a.x, i);
        const double y = (double)ld<CT>(a.y, i);
        if (locate(x, ax, ix) && locate(y, ay, iy)) bin[u] = iy * a.nx + ix;
      }
    }
    if (a.cnt) {
#pragma unroll
      for (int u = 0; u < PPT; ++u)
        if (bin[u] >= 0) atomicAdd(a.cnt + bin[u], 1u);
    }
    for (int j = 0; j < a.k; ++j) {
      AT v[PPT];
#pragma unroll
      for (int u = 0; u < PPT; ++u) {
        const int64_t i = base + (int64_t)u * blockDim.x + threadIdx.x;
        v[u] = bin[u] >= 0 ? ld<AT>(a.attr[j], i) : AT(0);
      }
      const AccPtrs p = a.acc[j];
#pragma unroll
      for (int u = 0; u < PPT; ++u)
        if (bin[u] >= 0) global_update<AT, PREC>(p, bin[u], v[u]);
    }
  }
}

// binary64 sum (S + C for the compensated words) and avg = sum / count.
__global__ __launch_bounds__(256) void bin_finalize_kernel(FinArgs a) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < a.nbins; b += stride) {
    const unsigned int c = a.cnt ? a.cnt[b] : 0u;
    for (int j = 0; j < a.k; ++j) {
      const FinAttr& f = a.attr[j];
      double s;
      if (f.src_kind == SRC_F64) s = static_cast<const double*>(f.src)[b];
      else if (f.src_kind == SRC_F32) s = (double)static_cast<const float*>(f.src)[b];
      else s = (double)static_cast<const float*>(f.src)[b] + (double)f.comp[b];
      if (f.sum_out) static_cast<double*>(f.sum_out)[b] = s;  // only the S + C case
      if (f.avg_out) {
        const double av = c ? s / (double)c : __builtin_nan("");
        if (f.avg_f64) static_cast<double*>(f.avg_out)[b] = av;
        else static_cast<float*>(f.avg_out)[b] = (float)av;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// LDS strategy: the whole grid in one workgroup's LDS (body in lds_body.h).
// ---------------------------------------------------------------------------
template <typename CT, typename AT, int PREC>
__global__ __launch_bounds__(1024) void bin_lds_kernel(LdsArgs a) {
  bin_lds_body<CT, AT, PREC>(a, blockIdx.x);
}
template <typename CT, typename AT, int PREC>
__global__ __launch_bounds__(1024) void bin_lds_batched(const LdsArgs* __restrict__ d,
                                                        const uint32_t* __restrict__ map) {
  const uint32_t m = map[blockIdx.x];
  bin_lds_body<CT, AT, PREC>(d[m >> 16], (int)(m & 0xFFFFu));
}

// Merge the slots of bins [b0, b0 + 64) (1024-thread workgroups).
template <typename AT, int PREC>
__global__ __launch_bounds__(1024) void lds_merge_kernel(LdsArgs a) {
  __shared__ __align__(16) unsigned char red[Tile<AT, PREC>::kMergeLds];
  for (int64_t b0 = (int64_t)blockIdx.x * 64; b0 < a.nbins; b0 += (int64_t)gridDim.x * 64)
    Tile<AT, PREC>::merge_emit64(static_cast<const unsigned char*>(a.partial), a.lay.slot_bytes, 0u,
                                 (uint32_t)a.nslots, a.lay, a.out, a.k, b0, a.nbins, 0, red);
}
template <typename AT, int PREC>
__global__ __launch_bounds__(1024) void lds_merge_batched(const LdsArgs* __restrict__ d,
                                                          const uint32_t* __restrict__ map) {
  __shared__ __align__(16) unsigned char red[Tile<AT, PREC>::kMergeLds];
  const uint32_t m = map[blockIdx.x];
  const LdsArgs& a = d[m >> 16];
  if (a.nslots > 1)
    Tile<AT, PREC>::merge_emit64(static_cast<const unsigned char*>(a.partial), a.lay.slot_bytes, 0u,
                                 (uint32_t)a.nslots, a.lay, a.out, a.k, (int64_t)(m & 0xFFFFu) * 64, a.nbins, 0, red);
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------
template <typename CT, typename AT, int PREC>
static hipError_t launch_global_t(const BinArgs& a, const LaunchCfg& c, hipStream_t s, KTimer* tm) {
  if (tm) tm->begin(s);
  hipLaunchKernelGGL((bin_global_kernel<CT, AT, PREC, 4>), dim3(c.grid), dim3(c.block), 0, s, a);
  if (tm) tm->end("bin_global_kernel", s);
  return hipGetLastError();
}

template <typename CT, typename AT, int PREC>
static hipError_t launch_lds_t(const LdsArgs& a, const LaunchCfg& c, hipStream_t s, KTimer* tm) {
  hipError_t e;
  if (tm) tm->begin(s);
  hipLaunchKernelGGL((bin_lds_kernel<CT, AT, PREC>), dim3(c.grid), dim3(c.block), c.lds_bytes, s, a);
  if (tm) tm->end("bin_lds_kernel", s);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (a.nslots > 1) {
    const int64_t g = (a.nbins + 63) / 64;
    if (tm) tm->begin(s);
    hipLaunchKernelGGL((lds_merge_kernel<AT, PREC>), dim3((int)(g < 4096 ? g : 4096)), dim3(1024), 0, s, a);
    if (tm) tm->end("lds_merge_kernel", s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename CT, typename AT, int PREC>
static hipError_t launch_lds_batch_t(const LdsBatch& b, hipStream_t s, KTimer* tm) {
  hipError_t e;
  for (int q = 0; q < 3; ++q) {
    const int nb = b.cls_first[q + 1] - b.cls_first[q];
    if (nb <= 0) continue;
    if (tm) tm->begin(s);
    hipLaunchKernelGGL((bin_lds_batched<CT, AT, PREC>), dim3(nb), dim3(b.cls_block[q]), (size_t)b.cls_lds[q], s,
                       b.descs, b.map_slot + b.cls_first[q]);
    if (tm) tm->end("bin_lds_kernel", s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (b.n_merge_blocks > 0) {
    if (tm) tm->begin(s);
    hipLaunchKernelGGL((lds_merge_batched<AT, PREC>), dim3(b.n_merge_blocks), dim3(1024), 0, s, b.descs, b.map_merge);
    if (tm) tm->end("lds_merge_kernel", s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

#define BK_DISPATCH(FN, ...)                                                        \
  if (coord_f64) {                                                                  \
    if (attr_f64) return FN<double, double, PREC_F64>(__VA_ARGS__);                 \
    switch (prec) {                                                                 \
      case PREC_PLAIN: return FN<double, float, PREC_PLAIN>(__VA_ARGS__);           \
      case PREC_COMP: return FN<double, float, PREC_COMP>(__VA_ARGS__);             \
      default: return FN<double, float, PREC_F64>(__VA_ARGS__);                     \
    }                                                                               \
  } else {                                                                          \
    if (attr_f64) return FN<float, double, PREC_F64>(__VA_ARGS__);                  \
    switch (prec) {                                                                 \
      case PREC_PLAIN: return FN<float, float, PREC_PLAIN>(__VA_ARGS__);            \
      case PREC_COMP: return FN<float, float, PREC_COMP>(__VA_ARGS__);              \
      default: return FN<float, float, PREC_F64>(__VA_ARGS__);                      \
    }                                                                               \
  }

hipError_t launch_bin_global(const BinArgs& a, bool coord_f64, bool attr_f64, int prec, const LaunchCfg& c,
                             hipStream_t s, KTimer* tm) {
  BK_DISPATCH(launch_global_t, a, c, s, tm)
}

hipError_t launch_bin_lds(const LdsArgs& a, bool coord_f64, bool attr_f64, int prec, const LaunchCfg& c,
                          hipStream_t s, KTimer* tm) {
  BK_DISPATCH(launch_lds_t, a, c, s, tm)
}

hipError_t launch_lds_batch(const LdsBatch& b, bool coord_f64, bool attr_f64, int prec, hipStream_t s, KTimer* tm) {
  BK_DISPATCH(launch_lds_batch_t, b, s, tm)
}
#undef BK_DISPATCH

hipError_t launch_init(const InitArgs& a, int grid, hipStream_t s, KTimer* tm) {
  if (tm) tm->begin(s);
  hipLaunchKernelGGL(bin_init_kernel, dim3(grid), dim3(256), 0, s, a);
  if (tm) tm->end("bin_init_kernel", s);
  return hipGetLastError();
}

hipError_t launch_finalize(const FinArgs& a, int grid, hipStream_t s, KTimer* tm) {
  if (tm) tm->begin(s);
  hipLaunchKernelGGL(bin_finalize_kernel, dim3(grid), dim3(256), 0, s, a);
  if (tm) tm->end("bin_finalize_kernel", s);
  return hipGetLastError();
}

// Allow a kernel up to 'total' bytes of LDS per workgroup: its static LDS
// plus dynamic LDS.
hipError_t set_dynamic_lds_limit(const void* fn, size_t total) {
  hipFuncAttributes attr;
  hipError_t e = hipFuncGetAttributes(&attr, fn);
  if (e != hipSuccess) return e;
  const size_t stat = attr.sharedSizeBytes;
  const size_t dyn = total > stat ? total - stat : 0;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
}

hipError_t set_lds_limit(size_t bytes) {
  hipError_t e = hipSuccess;
#define BK_SET(CT, AT, P)                                                                                        \
  if (e == hipSuccess) e = set_dynamic_lds_limit(reinterpret_cast<const void*>(&bin_lds_kernel<CT, AT, P>), bytes); \
  if (e == hipSuccess) e = set_dynamic_lds_limit(reinterpret_cast<const void*>(&bin_lds_batched<CT, AT, P>), bytes);
  BK_SET(float, float, PREC_PLAIN)
  BK_SET(float, float, PREC_COMP)
  BK_SET(float, float, PREC_F64)
  BK_SET(float, double, PREC_F64)
  BK_SET(double, float, PREC_PLAIN)
  BK_SET(double, float, PREC_COMP)
  BK_SET(double, float, PREC_F64)
  BK_SET(double, double, PREC_F64)
#undef BK_SET
  if (e == hipSuccess) e = set_partition_lds_limit(bytes);
  return e;
}

}  // namespace bk
