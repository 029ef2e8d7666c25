// Mesh bounds computed on the fly (Section 4.2: the low and high bounds of
// each axis may be obtained from the minimum and maximum of the coordinate
// variable).  Only finite coordinates count; the result is kept as four
// totalOrder keys (xmin, xmax, ymin, ymax) in device memory, from which the
// binning kernels derive their axes (resolve_axes).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"
#include "kernels.h"

namespace bk {

__global__ void bounds_init_kernel(long long* keys) {
  if (threadIdx.x == 0) {
    keys[0] = fkey((double)INFINITY);
    keys[1] = fkey((double)-INFINITY);
    keys[2] = fkey((double)INFINITY);
    keys[3] = fkey((double)-INFINITY);
  }
}

template <typename CT>
__global__ __launch_bounds__(256) void bounds_reduce_kernel(const void* x, const void* y, int64_t n, long long* keys) {
  __shared__ double red[4][256];
  double xmn = INFINITY, xmx = -INFINITY, ymn = INFINITY, ymx = -INFINITY;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double vx = (double)ld<CT>(x, i);
    const double vy = (double)ld<CT>(y, i);
    if (__builtin_isfinite(vx)) {
      xmn = vx < xmn ? vx : xmn;
      xmx = vx > xmx ? vx : xmx;
    }
    if (__builtin_isfinite(vy)) {
      ymn = vy < ymn ? vy : ymn;
      ymx = vy > ymx ? vy : ymx;
    }
  }
  red[0][threadIdx.x] = xmn;
  red[1][threadIdx.x] = xmx;
  red[2][threadIdx.x] = ymn;
  red[3][threadIdx.x] = ymx;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      const int t = threadIdx.x;
      red[0][t] = red[0][t + off] < red[0][t] ? red[0][t + off] : red[0][t];
      red[1][t] = red[1][t + off] > red[1][t] ? red[1][t + off] : red[1][t];
      red[2][t] = red[2][t + off] < red[2][t] ? red[2][t + off] : red[2][t];
      red[3][t] = red[3][t + off] > red[3][t] ? red[3][t + off] : red[3][t];
    }
    __syncthreads();
  }
  // -0 and +0 compare equal above; totalOrder keys pick -0 for the minimum
  // and +0 for the maximum only when that value was seen, which cannot move
  // any particle across a bin edge (both are the same coordinate).
  if (threadIdx.x == 0) {
    atomicMin(keys + 0, fkey(red[0][0]));
    atomicMax(keys + 1, fkey(red[1][0]));
    atomicMin(keys + 2, fkey(red[2][0]));
    atomicMax(keys + 3, fkey(red[3][0]));
  }
}

hipError_t launch_bounds(const void* x, const void* y, bool coord_f64, int64_t n, long long* keys, int cus,
                         hipStream_t s, KTimer* tm) {
  if (tm) tm->begin(s);
  hipLaunchKernelGGL(bounds_init_kernel, dim3(1), dim3(64), 0, s, keys);
  if (tm) tm->end("bounds_init_kernel", s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t want = (n + 4095) / 4096;
  const int grid = (int)(want < 1 ? 1 : (want > (int64_t)cus * 4 ? (int64_t)cus * 4 : want));
  if (tm) tm->begin(s);
  if (coord_f64)
    hipLaunchKernelGGL((bounds_reduce_kernel<double>), dim3(grid), dim3(256), 0, s, x, y, n, keys);
  else
    hipLaunchKernelGGL((bounds_reduce_kernel<float>), dim3(grid), dim3(256), 0, s, x, y, n, keys);
  if (tm) tm->end("bounds_reduce_kernel", s);
  return hipGetLastError();
}

}  // namespace bk
