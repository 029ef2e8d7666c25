// Device helpers shared by the binning kernels: bin location, totalOrder
// min/max, TwoSum, streaming loads.
#ifndef BINNING_DEVICE_COMMON_H
#define BINNING_DEVICE_COMMON_H

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace bk {

// Bin location (Section 4.2): inside test with a closed upper edge, then
// trunc((x - lo) * scale) clamped to n-1, all in binary64.  A zero scale
// (zero-extent axis, or an extent from the data too large or too small for
// a finite binary64 scale) maps every inside value to cell 0: the product
// is then 0, or NaN where v - lo overflows, and max(NaN, 0) is 0.
__device__ __forceinline__ bool locate(double v, const Axis& a, int& idx) {
  if (!(v >= a.lo && v <= a.hi)) return false;  // NaN fails both tests
  const double f = __builtin_fmax((v - a.lo) * a.scale, 0.0);
  const int i = (int)f;  // v_cvt_i32_f64 truncates; 0 <= f <= n (1 + 2^-52) here
  idx = i < a.n ? i : a.n - 1;
  return true;
}

// Scale of an axis whose bounds come from the data: n / (hi - lo), or 0
// when the extent is zero or either quantity is not finite in binary64.
__device__ __forceinline__ double data_scale(int n, double lo, double hi) {
  if (!(hi > lo)) return 0.0;
  const double w = hi - lo;
  const double s = (double)n / w;
  return (__builtin_isfinite(w) && __builtin_isfinite(s)) ? s : 0.0;
}

__device__ __forceinline__ double fkey_decode(long long k);

// Axes from bounds computed on the device (four totalOrder keys: xmin,
// xmax, ymin, ymax), or left as passed when keys is null.  A zero-extent
// axis, or one whose extent or scale is not finite, gets scale 0 (every
// inside value in cell 0); an axis that saw no finite value has
// lo = +Inf > hi = -Inf, so nothing is inside.
__device__ __forceinline__ void resolve_axes(const long long* keys, Axis& ax, Axis& ay) {
  if (!keys) return;
  ax.lo = fkey_decode(keys[0]);
  ax.hi = fkey_decode(keys[1]);
  ay.lo = fkey_decode(keys[2]);
  ay.hi = fkey_decode(keys[3]);
  ax.scale = data_scale(ax.n, ax.lo, ax.hi);
  ay.scale = data_scale(ay.n, ay.lo, ay.hi);
}

// totalOrder min/max on float bit patterns held directly in a result array.
// For a non-negative value (sign bit clear) signed-integer order of the bit
// patterns equals IEEE totalOrder; for a value with the sign bit set,
// unsigned order of the bits is the reverse of totalOrder.  One integer
// atomic per lane, no key decoding pass.
// totalOrder keys of raw float bits (signed order of the key = totalOrder).
__device__ __forceinline__ int total_key(int b) { return b >= 0 ? b : (b ^ 0x7FFFFFFF); }
__device__ __forceinline__ long long total_key(long long b) { return b >= 0 ? b : (b ^ 0x7FFFFFFFFFFFFFFFLL); }

// Skip the atomic when the value cannot beat the value read from the result
// array: min/max only move one way, so even a stale read is a safe filter.
template <typename T, typename I>
__device__ __forceinline__ bool beats_min(const T* p, T v) {
  const I cur = __hip_atomic_load(reinterpret_cast<const I*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  I vb;
  __builtin_memcpy(&vb, &v, sizeof vb);
  return total_key(vb) < total_key(cur);
}
template <typename T, typename I>
__device__ __forceinline__ bool beats_max(const T* p, T v) {
  const I cur = __hip_atomic_load(reinterpret_cast<const I*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  I vb;
  __builtin_memcpy(&vb, &v, sizeof vb);
  return total_key(vb) > total_key(cur);
}

__device__ __forceinline__ void atomic_min_fp(float* p, float v) {
  const int b = __float_as_int(v);
  if (b >= 0)
    atomicMin(reinterpret_cast<int*>(p), b);
  else
    atomicMax(reinterpret_cast<unsigned int*>(p), static_cast<unsigned int>(b));
}
__device__ __forceinline__ void atomic_max_fp(float* p, float v) {
  const int b = __float_as_int(v);
  if (b >= 0)
    atomicMax(reinterpret_cast<int*>(p), b);
  else
    atomicMin(reinterpret_cast<unsigned int*>(p), static_cast<unsigned int>(b));
}
__device__ __forceinline__ void atomic_min_fp(double* p, double v) {
  const long long b = __double_as_longlong(v);
  if (b >= 0)
    atomicMin(reinterpret_cast<long long*>(p), b);
  else
    atomicMax(reinterpret_cast<unsigned long long*>(p), static_cast<unsigned long long>(b));
}
__device__ __forceinline__ void atomic_max_fp(double* p, double v) {
  const long long b = __double_as_longlong(v);
  if (b >= 0)
    atomicMax(reinterpret_cast<long long*>(p), b);
  else
    atomicMin(reinterpret_cast<unsigned long long*>(p), static_cast<unsigned long long>(b));
}

// Order-preserving integer keys (one LDS atomic per lane whatever the sign).
// Signed order of the key equals totalOrder of the value.
__device__ __forceinline__ int fkey(float v) {
  const int b = __float_as_int(v);
  return b >= 0 ? b : (b ^ 0x7FFFFFFF);
}
__device__ __forceinline__ float fkey_decode(int k) { return __int_as_float(k >= 0 ? k : (k ^ 0x7FFFFFFF)); }
__device__ __forceinline__ long long fkey(double v) {
  const long long b = __double_as_longlong(v);
  return b >= 0 ? b : (b ^ 0x7FFFFFFFFFFFFFFFLL);
}
__device__ __forceinline__ double fkey_decode(long long k) {
  return __longlong_as_double(k >= 0 ? k : (k ^ 0x7FFFFFFFFFFFFFFFLL));
}
template <typename AT> struct KeyOf;
template <> struct KeyOf<float> { using T = int; };
template <> struct KeyOf<double> { using T = long long; };

// Error-free transformation (Knuth's TwoSum): with s = fl(a + b), returns
// e such that a + b = s + e exactly (round-to-nearest, no overflow).
__device__ __forceinline__ float two_sum_err(float a, float b, float s) {
  const float bb = s - a;
  return (a - (s - bb)) + (b - bb);
}

// Streaming column load (read once; keep caches for accumulators).
template <typename T>
__device__ __forceinline__ T ld(const void* p, int64_t i) {
  return __builtin_nontemporal_load(static_cast<const T*>(p) + i);
}
// Plain (temporal) load: for data that other workgroups read soon after.
template <typename T>
__device__ __forceinline__ T ld_keep(const void* p, int64_t i) {
  return static_cast<const T*>(p)[i];
}

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Elements i .. i+3 of a 16-byte aligned column (i a multiple of 4), read
// with 16-byte loads: HBM streams at full rate only with wide loads.
template <typename T, typename I>
__device__ __forceinline__ void ld4v(const void* p, I i, T* out) {
  if constexpr (sizeof(T) == 4) {
    const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(static_cast<const T*>(p) + i));
    out[0] = v.x;
    out[1] = v.y;
    out[2] = v.z;
    out[3] = v.w;
  } else {
    const f64x2* q = reinterpret_cast<const f64x2*>(static_cast<const T*>(p) + i);
    const f64x2 a = __builtin_nontemporal_load(q);
    const f64x2 b = __builtin_nontemporal_load(q + 1);
    out[0] = a.x;
    out[1] = a.y;
    out[2] = b.x;
    out[3] = b.y;
  }
}

// Elements i .. i+3 of a column into out[0..3], zero past hi; wide loads
// when vec (column 16-byte aligned, i a multiple of 4) and the group is full.
template <typename T>
__device__ __forceinline__ void ld4(const void* p, int64_t i, int64_t hi, bool vec, T* out) {
  if (vec && i + 4 <= hi) {
    ld4v<T, int64_t>(p, i, out);
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) out[e] = i + e < hi ? ld<T>(p, i + e) : T(0);
  }
}

// ---------------------------------------------------------------------------
// LDS tile accumulators (layout in TileLayout).  All functions are called by
// every thread of the workgroup; tb = bins of the tile held in LDS.
// ---------------------------------------------------------------------------
template <typename AT, int PREC>
struct Tile {
  using K = typename KeyOf<AT>::T;
  static constexpr int kSumBytes = (PREC == PREC_PLAIN) ? 4 : 8;
  // Element of local bin b in the min (or max) array: interleaved pairs
  // when both are kept.
  __device__ static int mm(const TileLayout& L, int b) { return L.mm_pair ? 2 * b : b; }

  __device__ static void init(unsigned char* smem, const TileLayout& L, int k) {
    const int tb = L.tb;
    uint32_t* cnt = reinterpret_cast<uint32_t*>(smem);
    for (int b = threadIdx.x; b < tb; b += blockDim.x) cnt[b] = 0u;
    for (int j = 0; j < k; ++j) {
      if (L.want_sum) {
        uint32_t* w = reinterpret_cast<uint32_t*>(smem + L.lds_sum_off[j]);
        const int words = tb * kSumBytes / 4;
        for (int b = threadIdx.x; b < words; b += blockDim.x) w[b] = 0u;
      }
      if (L.want_min) {
        K* m = reinterpret_cast<K*>(smem + L.lds_min_off[j]);
        for (int b = threadIdx.x; b < tb; b += blockDim.x) m[mm(L, b)] = fkey((AT)INFINITY);
      }
      if (L.want_max) {
        K* m = reinterpret_cast<K*>(smem + L.lds_max_off[j]);
        for (int b = threadIdx.x; b < tb; b += blockDim.x) m[mm(L, b)] = fkey((AT)-INFINITY);
      }
    }
  }

  __device__ static void count(unsigned char* smem, int b) { atomicAdd(reinterpret_cast<uint32_t*>(smem) + b, 1u); }

  // Plain binary32 sum: S' = fl(S + v) by a 4-byte compare-and-swap (on
  // gfx950 a float add in LDS runs at a fraction of the rate of the integer
  // operations; the swap and its read are two of those).  'seen' is the
  // word as last read; a failed swap returns the current word.
  __device__ static void plain_update(uint32_t* p, uint32_t seen, float v) {
    for (;;) {
      const uint32_t want = __float_as_uint(__uint_as_float(seen) + v);
      if (__hip_atomic_compare_exchange_strong(p, &seen, want, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP))
        return;
    }
  }

  // Compensated binary32 sum (TwoSum): a bin's running sum S and its
  // compensation C share one 8-byte word, low half S, high half C, and are
  // updated together by compare-and-swap: S' = fl(S + v), C' = fl(C + e)
  // with e the exact rounding error of S + v.  'seen' is the word as last
  // read; a failed swap returns the current word and the update is redone
  // on it, so every attempt that fails lets another one succeed.
  __device__ static void comp_update(unsigned long long* p, unsigned long long seen, float v) {
    for (;;) {
      const float s = __uint_as_float((uint32_t)seen);
      const float c = __uint_as_float((uint32_t)(seen >> 32));
      const float ns = s + v;
      const float nc = c + two_sum_err(s, v, ns);
      const unsigned long long want =
          (unsigned long long)__float_as_uint(ns) | ((unsigned long long)__float_as_uint(nc) << 32);
      if (__hip_atomic_compare_exchange_strong(p, &seen, want, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP))
        return;
    }
  }

  __device__ static void add(unsigned char* smem, const TileLayout& L, int j, int b, AT v) {
    if (L.want_sum) {
      unsigned char* base = smem + L.lds_sum_off[j];
      if constexpr (PREC == PREC_F64) {
        atomicAdd(reinterpret_cast<double*>(base) + b, (double)v);
      } else if constexpr (PREC == PREC_PLAIN) {
        uint32_t* P = reinterpret_cast<uint32_t*>(base) + b;
        plain_update(P, __hip_atomic_load(P, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP), (float)v);
      } else {
        unsigned long long* P = reinterpret_cast<unsigned long long*>(base) + b;
        comp_update(P, __hip_atomic_load(P, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP), (float)v);
      }
    }
    // min/max keys only move one way, so a value that does not beat the key
    // read (however stale) cannot change it: skip its atomic.  Once a bin has
    // seen m values, a new one changes its min with probability ~1/m.
    if (L.want_min || L.want_max) {
      const K kv = fkey(v);
      if (L.want_min) {
        K* m = reinterpret_cast<K*>(smem + L.lds_min_off[j]) + mm(L, b);
        if (kv < __hip_atomic_load(m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) atomicMin(m, kv);
      }
      if (L.want_max) {
        K* m = reinterpret_cast<K*>(smem + L.lds_max_off[j]) + mm(L, b);
        if (kv > __hip_atomic_load(m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) atomicMax(m, kv);
      }
    }
  }

  // add() for R records at once (lb[u] < 0: no record).  Every LDS read
  // of the R records (the min/max filter, the compensated sum's old value)
  // is issued before any of them is used, so the wave waits for LDS once
  // per group instead of once per record.
  template <int R>
  __device__ static void add_batch(unsigned char* smem, const TileLayout& L, int j, const int* lb, const AT* v) {
    if (L.want_sum) {
      unsigned char* base = smem + L.lds_sum_off[j];
      if constexpr (PREC == PREC_F64) {
#pragma unroll
        for (int u = 0; u < R; ++u)
          if (lb[u] >= 0) atomicAdd(reinterpret_cast<double*>(base) + lb[u], (double)v[u]);
      } else if constexpr (PREC == PREC_PLAIN) {
        uint32_t* P = reinterpret_cast<uint32_t*>(base);
        uint32_t seen[R];
#pragma unroll
        for (int u = 0; u < R; ++u)
          seen[u] = lb[u] >= 0 ? __hip_atomic_load(P + lb[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : 0u;
#pragma unroll
        for (int u = 0; u < R; ++u)
          if (lb[u] >= 0) plain_update(P + lb[u], seen[u], (float)v[u]);
      } else {
        unsigned long long* P = reinterpret_cast<unsigned long long*>(base);
        unsigned long long seen[R];
#pragma unroll
        for (int u = 0; u < R; ++u)
          seen[u] = lb[u] >= 0 ? __hip_atomic_load(P + lb[u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : 0ull;
#pragma unroll
        for (int u = 0; u < R; ++u)
          if (lb[u] >= 0) comp_update(P + lb[u], seen[u], (float)v[u]);
      }
    }
    if (L.want_min || L.want_max) {
      K kv[R], cmin[R], cmax[R];
      K* mn = reinterpret_cast<K*>(smem + L.lds_min_off[j]);
      K* mx = reinterpret_cast<K*>(smem + L.lds_max_off[j]);
#pragma unroll
      for (int u = 0; u < R; ++u) {
        kv[u] = fkey(v[u]);
        const int b = lb[u] >= 0 ? lb[u] : 0;
        if constexpr (sizeof(K) == 4) {
          if (L.mm_pair) {  // both keys of the bin in one 8-byte read
            const long long pr = __hip_atomic_load(reinterpret_cast<const long long*>(mn + 2 * b), __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WORKGROUP);
            cmin[u] = (K)(int)(pr & 0xFFFFFFFFll);
            cmax[u] = (K)(int)(pr >> 32);
            continue;
          }
        }
        cmin[u] = L.want_min ? __hip_atomic_load(mn + mm(L, b), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : K(0);
        cmax[u] = L.want_max ? __hip_atomic_load(mx + mm(L, b), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) : K(0);
      }
#pragma unroll
      for (int u = 0; u < R; ++u) {
        if (lb[u] < 0) continue;
        if (L.want_min && kv[u] < cmin[u]) atomicMin(mn + mm(L, lb[u]), kv[u]);
        if (L.want_max && kv[u] > cmax[u]) atomicMax(mx + mm(L, lb[u]), kv[u]);
      }
    }
  }

  __device__ static uint32_t cnt_get(const unsigned char* smem, int b) {
    return reinterpret_cast<const uint32_t*>(smem)[b];
  }
  // binary64 value of the sum (S + C for the compensated words).
  __device__ static double sum_get(const unsigned char* smem, const TileLayout& L, int j, int b) {
    const unsigned char* base = smem + L.lds_sum_off[j];
    if constexpr (PREC == PREC_F64) return reinterpret_cast<const double*>(base)[b];
    else if constexpr (PREC == PREC_PLAIN) return (double)reinterpret_cast<const float*>(base)[b];
    else {
      const float* SC = reinterpret_cast<const float*>(base) + 2 * b;
      return (double)SC[0] + (double)SC[1];
    }
  }
  __device__ static K min_get(const unsigned char* smem, const TileLayout& L, int j, int b) {
    return reinterpret_cast<const K*>(smem + L.lds_min_off[j])[mm(L, b)];
  }
  __device__ static K max_get(const unsigned char* smem, const TileLayout& L, int j, int b) {
    return reinterpret_cast<const K*>(smem + L.lds_max_off[j])[mm(L, b)];
  }

  // Final values of attribute j in one bin: sum (binary64 or float), min/max
  // decoded from keys, avg = sum / count (NaN if empty).
  __device__ static void emit_attr(const Outs& o, int j, int64_t gb, uint32_t c, double s, K kmin, K kmax) {
    if (o.sum[j]) {
      if constexpr (PREC == PREC_PLAIN) static_cast<float*>(o.sum[j])[gb] = (float)s;
      else static_cast<double*>(o.sum[j])[gb] = s;
    }
    if (o.mn[j]) static_cast<AT*>(o.mn[j])[gb] = fkey_decode(kmin);
    if (o.mx[j]) static_cast<AT*>(o.mx[j])[gb] = fkey_decode(kmax);
    if (o.avg[j]) {
      const double av = c ? s / (double)c : __builtin_nan("");
      if constexpr (PREC == PREC_PLAIN) static_cast<float*>(o.avg[j])[gb] = (float)av;
      else static_cast<double*>(o.avg[j])[gb] = av;
    }
  }

  // Write the finished outputs of local bins [0, nbt) -> global b0 + b.
  __device__ static void emit_all(const unsigned char* smem, const TileLayout& L, const Outs& o, int k, int nbt,
                                  int64_t b0) {
    for (int b = threadIdx.x; b < nbt; b += blockDim.x) {
      const uint32_t c = cnt_get(smem, b);
      if (o.cnt) o.cnt[b0 + b] = c;
      for (int j = 0; j < k; ++j)
        emit_attr(o, j, b0 + b, c, L.want_sum ? sum_get(smem, L, j, b) : 0.0,
                  L.want_min ? min_get(smem, L, j, b) : K(0), L.want_max ? max_get(smem, L, j, b) : K(0));
    }
  }

  // Store this workgroup's accumulators of local bins [0, nbt) as a slot.
  __device__ static void store_slot(const unsigned char* smem, const TileLayout& L, int k, int nbt,
                                    unsigned char* slot) {
    for (int b = threadIdx.x; b < nbt; b += blockDim.x) {
      reinterpret_cast<uint32_t*>(slot)[b] = cnt_get(smem, b);
      for (int j = 0; j < k; ++j) {
        if (L.want_sum) {
          const double s = sum_get(smem, L, j, b);
          if constexpr (PREC == PREC_PLAIN) reinterpret_cast<float*>(slot + L.slot_sum_off[j])[b] = (float)s;
          else reinterpret_cast<double*>(slot + L.slot_sum_off[j])[b] = s;
        }
        if (L.want_min) reinterpret_cast<K*>(slot + L.slot_min_off[j])[b] = min_get(smem, L, j, b);
        if (L.want_max) reinterpret_cast<K*>(slot + L.slot_max_off[j])[b] = max_get(smem, L, j, b);
      }
    }
  }

  // Combine slots first..first+nslot-1 for 64 consecutive bins [b0, b0+64)
  // (local index lb = gb - goff) with a 1024-thread workgroup: 16 threads
  // per bin each fold every 16th slot, then the 16 partials are combined in
  // LDS and the finished bin is emitted.  Many slots are merged in
  // parallel instead of one slot after another.
  // LDS workspace for merge_emit64: 16 x 64 partial sums, keys and counts.
  static constexpr int kMergeLds = 16 * 64 * (8 + 2 * (int)sizeof(K) + 4);
  __device__ static void merge_emit64(const unsigned char* slots, int64_t slot_bytes, uint32_t first, uint32_t nslot,
                                      const TileLayout& L, const Outs& o, int k, int64_t b0, int64_t nb,
                                      int64_t goff, unsigned char* lds) {
    double(*red_s)[64] = reinterpret_cast<double(*)[64]>(lds);
    K(*red_mn)[64] = reinterpret_cast<K(*)[64]>(lds + 16 * 64 * 8);
    K(*red_mx)[64] = reinterpret_cast<K(*)[64]>(lds + 16 * 64 * (8 + sizeof(K)));
    uint32_t(*red_c)[64] = reinterpret_cast<uint32_t(*)[64]>(lds + 16 * 64 * (8 + 2 * sizeof(K)));
    const int bl = threadIdx.x & 63;
    const int sg = threadIdx.x >> 6;  // 16 slot groups (blockDim.x == 1024)
    const int64_t gb = b0 + bl;
    const bool live = gb < nb;
    const int lb = (int)(gb - goff);
    uint32_t c = 0;
    if (live)
      for (uint32_t q = sg; q < nslot; q += 16)
        c += reinterpret_cast<const uint32_t*>(slots + (int64_t)(first + q) * slot_bytes)[lb];
    red_c[sg][bl] = c;
    __syncthreads();
    if (sg == 0) {
      for (int g = 1; g < 16; ++g) c += red_c[g][bl];
      red_c[0][bl] = c;
      if (live && o.cnt) o.cnt[gb] = c;
    }
    __syncthreads();
    c = red_c[0][bl];
    for (int j = 0; j < k; ++j) {
      double s = 0.0;
      K kmin = fkey((AT)INFINITY), kmax = fkey((AT)-INFINITY);
      if (live)
        for (uint32_t q = sg; q < nslot; q += 16) {
          const unsigned char* slot = slots + (int64_t)(first + q) * slot_bytes;
          if (L.want_sum) {
            if constexpr (PREC == PREC_PLAIN) s += (double)reinterpret_cast<const float*>(slot + L.slot_sum_off[j])[lb];
            else s += reinterpret_cast<const double*>(slot + L.slot_sum_off[j])[lb];
          }
          if (L.want_min) {
            const K m = reinterpret_cast<const K*>(slot + L.slot_min_off[j])[lb];
            kmin = m < kmin ? m : kmin;
          }
          if (L.want_max) {
            const K m = reinterpret_cast<const K*>(slot + L.slot_max_off[j])[lb];
            kmax = m > kmax ? m : kmax;
          }
        }
      red_s[sg][bl] = s;
      red_mn[sg][bl] = kmin;
      red_mx[sg][bl] = kmax;
      __syncthreads();
      if (sg == 0 && live) {
        for (int g = 1; g < 16; ++g) {
          s += red_s[g][bl];
          kmin = red_mn[g][bl] < kmin ? red_mn[g][bl] : kmin;
          kmax = red_mx[g][bl] > kmax ? red_mx[g][bl] : kmax;
        }
        emit_attr(o, j, gb, c, s, kmin, kmax);
      }
      __syncthreads();
    }
  }

  // Combine slots first..first+nslot-1 for local bin b and emit it.
  __device__ static void merge_emit(const unsigned char* slots, int64_t slot_bytes, uint32_t first, uint32_t nslot,
                                    const TileLayout& L, const Outs& o, int k, int b, int64_t gb) {
    uint32_t c = 0;
    for (uint32_t q = 0; q < nslot; ++q)
      c += reinterpret_cast<const uint32_t*>(slots + (int64_t)(first + q) * slot_bytes)[b];
    if (o.cnt) o.cnt[gb] = c;
    for (int j = 0; j < k; ++j) {
      double s = 0.0;
      K kmin = fkey((AT)INFINITY), kmax = fkey((AT)-INFINITY);
      for (uint32_t q = 0; q < nslot; ++q) {
        const unsigned char* slot = slots + (int64_t)(first + q) * slot_bytes;
        if (L.want_sum) {
          if constexpr (PREC == PREC_PLAIN) s += (double)reinterpret_cast<const float*>(slot + L.slot_sum_off[j])[b];
          else s += reinterpret_cast<const double*>(slot + L.slot_sum_off[j])[b];
        }
        if (L.want_min) {
          const K m = reinterpret_cast<const K*>(slot + L.slot_min_off[j])[b];
          kmin = m < kmin ? m : kmin;
        }
        if (L.want_max) {
          const K m = reinterpret_cast<const K*>(slot + L.slot_max_off[j])[b];
          kmax = m > kmax ? m : kmax;
        }
      }
      emit_attr(o, j, gb, c, s, kmin, kmax);
    }
  }
};

}  // namespace bk

#endif
