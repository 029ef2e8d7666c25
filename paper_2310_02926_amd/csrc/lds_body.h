// Body of the whole-grid LDS strategy, shared by its single-request and
// batched kernels: one workgroup bins particles [wg * chunk,
// (wg + 1) * chunk) of a request into the grid held in LDS, then writes the
// finished outputs (a lone workgroup) or its accumulators as partial slot wg.
#ifndef BINNING_LDS_BODY_H
#define BINNING_LDS_BODY_H

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"
#include "kernels.h"

namespace bk {

template <typename CT, typename AT, int PREC>
__device__ __forceinline__ void bin_lds_body(const LdsArgs& a, int wg) {
  using TL = Tile<AT, PREC>;
  extern __shared__ __align__(16) unsigned char smem[];
  Axis ax = a.ax, ay = a.ay;
  resolve_axes(a.dyn, ax, ay);
  TL::init(smem, a.lay, a.k);
  __syncthreads();

  const int64_t lo = (int64_t)wg * a.chunk;
  const int64_t hi = lo + a.chunk < a.n ? lo + a.chunk : a.n;
  // Groups of 4 consecutive particles per lane (16-byte loads).
  const bool vec = a.vec != 0;
  constexpr int G = 2;
  for (int64_t base = lo; base < hi; base += (int64_t)4 * G * blockDim.x) {
    int bin[4 * G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int64_t i = base + 4 * ((int64_t)g * blockDim.x + threadIdx.x);
      CT xs[4], ys[4];
      ld4<CT>(a.x, i, hi, vec, xs);
      ld4<CT>(a.y, i, hi, vec, ys);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int ix, iy;
        bin[4 * g + e] = -1;
        if (i + e < hi && locate((double)xs[e], ax, ix) && locate((double)ys[e], ay, iy))
          bin[4 * g + e] = iy * a.nx + ix;
      }
    }
#pragma unroll
    for (int u = 0; u < 4 * G; ++u)
      if (bin[u] >= 0) TL::count(smem, bin[u]);
    for (int j = 0; j < a.k; ++j) {
      AT v[4 * G];
#pragma unroll
      for (int g = 0; g < G; ++g)
        ld4<AT>(a.attr[j], base + 4 * ((int64_t)g * blockDim.x + threadIdx.x), hi, vec, v + 4 * g);
#pragma unroll
      for (int u = 0; u < 4 * G; ++u)
        if (bin[u] >= 0) TL::add(smem, a.lay, j, bin[u], v[u]);
    }
  }
  __syncthreads();
  if (a.nslots <= 1)
    TL::emit_all(smem, a.lay, a.out, a.k, a.nbins, 0);
  else
    TL::store_slot(smem, a.lay, a.k, a.nbins, static_cast<unsigned char*>(a.partial) + (int64_t)wg * a.lay.slot_bytes);
}

}  // namespace bk

#endif
