// Meshes of three axes (Section 4.2: the mesh axes are any chosen subset of
// the particle variables).  Axes 1 and 2 are folded into one composite
// coordinate before binning: per particle, c = iz * ny + iy when it is
// inside on both axes, NaN otherwise.  c is an integer below ny * nz, held
// exactly in the coordinate type, so binning (x, c) on an nx by ny * nz mesh
// whose second axis is [0, ny * nz] with scale 1 reproduces the bin
// (iz * ny + iy) * nx + ix and the inside test of the three-axis mesh
// exactly; the binning kernels are the two-axis ones.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"
#include "kernels.h"

namespace bk {

template <typename CT>
__device__ __forceinline__ void st4(void* p, int64_t i, int64_t hi, bool vec, const CT* v) {
  CT* q = static_cast<CT*>(p) + i;
  if (vec && i + 4 <= hi) {
    if constexpr (sizeof(CT) == 4) {
      *reinterpret_cast<f32x4*>(q) = f32x4{v[0], v[1], v[2], v[3]};
    } else {
      reinterpret_cast<f64x2*>(q)[0] = f64x2{v[0], v[1]};
      reinterpret_cast<f64x2*>(q)[1] = f64x2{v[2], v[3]};
    }
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (i + e < hi) q[e] = v[e];
  }
}

// Keys: with dyn_in set, axis 1 is [dyn_in[2], dyn_in[3]] and axis 2
// [dyn_in[4], dyn_in[5]] (bounds from the data); block 0 then writes the
// four keys the binning kernels read: axis 0 copied from dyn_in[0..1], the
// composite axis [0, ny * nz].
template <typename CT>
__global__ __launch_bounds__(256) void fold_axes_kernel(FoldArgs a) {
  Axis ay = a.ay, az = a.az;
  if (a.dyn_in) resolve_axes(a.dyn_in + 2, ay, az);
  if (a.dyn_out && blockIdx.x == 0 && threadIdx.x == 0) {
    a.dyn_out[0] = a.dyn_in[0];
    a.dyn_out[1] = a.dyn_in[1];
    a.dyn_out[2] = fkey(0.0);
    a.dyn_out[3] = fkey((double)ay.n * (double)az.n);
  }
  const bool vec = a.vec != 0;
  constexpr int G = 2;
  const int64_t step = (int64_t)gridDim.x * blockDim.x * 4 * G;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x * 4 * G; base < a.n; base += step) {
    CT ys[G][4], zs[G][4];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int64_t i = base + 4 * ((int64_t)g * blockDim.x + threadIdx.x);
      ld4<CT>(a.y, i, a.n, vec, ys[g]);
      ld4<CT>(a.z, i, a.n, vec, zs[g]);
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int64_t i = base + 4 * ((int64_t)g * blockDim.x + threadIdx.x);
      CT c[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        int iy, iz;
        const bool in = locate((double)ys[g][e], ay, iy) && locate((double)zs[g][e], az, iz);
        c[e] = in ? (CT)(iz * ay.n + iy) : (CT)__builtin_nan("");
      }
      st4<CT>(a.out, i, a.n, vec, c);
    }
  }
}

hipError_t launch_fold(const FoldArgs& a, bool coord_f64, int cus, hipStream_t s, KTimer* tm) {
  if (a.n == 0 && !a.dyn_out) return hipSuccess;
  const int64_t per_block = 256 * 4 * 2;
  const int64_t want = (a.n + per_block - 1) / per_block;
  const int64_t cap = (int64_t)cus * 8;
  const int grid = (int)(want < 1 ? 1 : (want > cap ? cap : want));
  if (tm) tm->begin(s);
  if (coord_f64)
    hipLaunchKernelGGL((fold_axes_kernel<double>), dim3(grid), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((fold_axes_kernel<float>), dim3(grid), dim3(256), 0, s, a);
  if (tm) tm->end("fold_axes_kernel", s);
  return hipGetLastError();
}

}  // namespace bk
