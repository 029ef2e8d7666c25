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
__device__ __forceinline__ void minmax_finite(CT v, CT& mn, CT& mx) {
  if (__builtin_isfinite(v)) {
    mn = v < mn ? v : mn;
    mx = v > mx ? v : mx;
  }
}

// Grid-stride min/max of the finite values of both columns, in the column
// type (exact).  With both columns 16-byte aligned, groups of 4 values are
// read with 16-byte loads, U groups per column in flight per thread; the
// rest (and unaligned columns) element by element.  Each block reduces
// across its waves and folds its result into the keys with 4 atomics.
template <typename CT>
__global__ __launch_bounds__(256) void bounds_reduce_kernel(const void* x, const void* y, int64_t n, int vec,
                                                            long long* keys) {
  __shared__ CT red[4][4];
  CT xmn = (CT)INFINITY, xmx = (CT)-INFINITY, ymn = (CT)INFINITY, ymx = (CT)-INFINITY;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  int64_t done = 0;
  if (vec) {
    constexpr int U = 2;
    const int64_t nq = n / 4;
    int64_t q = tid;
    for (; q + (U - 1) * nth < nq; q += U * nth) {
      CT vx[U][4], vy[U][4];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        ld4v<CT>(x, 4 * (q + u * nth), vx[u]);
        ld4v<CT>(y, 4 * (q + u * nth), vy[u]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          minmax_finite(vx[u][e], xmn, xmx);
          minmax_finite(vy[u][e], ymn, ymx);
        }
    }
    for (; q < nq; q += nth) {
      CT vx[4], vy[4];
      ld4v<CT>(x, 4 * q, vx);
      ld4v<CT>(y, 4 * q, vy);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        minmax_finite(vx[e], xmn, xmx);
        minmax_finite(vy[e], ymn, ymx);
      }
    }
    done = 4 * nq;
  }
  for (int64_t i = done + tid; i < n; i += nth) {
    minmax_finite(ld<CT>(x, i), xmn, xmx);
    minmax_finite(ld<CT>(y, i), ymn, ymx);
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const CT a = __shfl_xor(xmn, o), b = __shfl_xor(xmx, o), c = __shfl_xor(ymn, o), d = __shfl_xor(ymx, o);
    xmn = a < xmn ? a : xmn;
    xmx = b > xmx ? b : xmx;
    ymn = c < ymn ? c : ymn;
    ymx = d > ymx ? d : ymx;
  }
  const int wid = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wid] = xmn;
    red[1][wid] = xmx;
    red[2][wid] = ymn;
    red[3][wid] = ymx;
  }
  __syncthreads();
  // -0 and +0 compare equal above; totalOrder keys pick -0 for the minimum
  // and +0 for the maximum only when that value was seen, which cannot move
  // any particle across a bin edge (both are the same coordinate).
  if (threadIdx.x == 0) {
    const int nw = (int)(blockDim.x >> 6);
    for (int w = 1; w < nw; ++w) {
      xmn = red[0][w] < xmn ? red[0][w] : xmn;
      xmx = red[1][w] > xmx ? red[1][w] : xmx;
      ymn = red[2][w] < ymn ? red[2][w] : ymn;
      ymx = red[3][w] > ymx ? red[3][w] : ymx;
    }
    atomicMin(keys + 0, fkey((double)xmn));
    atomicMax(keys + 1, fkey((double)xmx));
    atomicMin(keys + 2, fkey((double)ymn));
    atomicMax(keys + 3, fkey((double)ymx));
  }
}

hipError_t launch_bounds(const void* x, const void* y, bool coord_f64, int64_t n, long long* keys, int cus,
                         hipStream_t s, KTimer* tm) {
  if (tm) tm->begin(s);
  hipLaunchKernelGGL(bounds_init_kernel, dim3(1), dim3(64), 0, s, keys);
  if (tm) tm->end("bounds_init_kernel", s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // One block per 32768 values, at most 2 per CU: fewer, longer-lived
  // workgroups stream faster here (6.2 TB/s against 5.0 with 8 per CU).
  const int64_t want = (n + 32767) / 32768;
  const int grid = (int)(want < 1 ? 1 : (want > (int64_t)cus * 2 ? (int64_t)cus * 2 : want));
  const int vec = (reinterpret_cast<uintptr_t>(x) % 16 == 0 && reinterpret_cast<uintptr_t>(y) % 16 == 0) ? 1 : 0;
  if (tm) tm->begin(s);
  if (coord_f64)
    hipLaunchKernelGGL((bounds_reduce_kernel<double>), dim3(grid), dim3(256), 0, s, x, y, n, vec, keys);
  else
    hipLaunchKernelGGL((bounds_reduce_kernel<float>), dim3(grid), dim3(256), 0, s, x, y, n, vec, keys);
  if (tm) tm->end("bounds_reduce_kernel", s);
  return hipGetLastError();
}

}  // namespace bk
