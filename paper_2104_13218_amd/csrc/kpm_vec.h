// Vector-access and reduction helpers shared by the gfx950 step kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "kpm_internal.h"

namespace kpm {

// ------------------------------------------------------------------ helpers

template <typename T, int N>
struct alignas(sizeof(T) * N >= 16 ? 16 : sizeof(T) * N) VecT {
  T v[N];
};

template <typename T, int N>
__device__ __forceinline__ VecT<T, N> vload(const T* p) {
  return *reinterpret_cast<const VecT<T, N>*>(p);
}
template <typename T, int N>
__device__ __forceinline__ void vstore(T* p, const VecT<T, N>& x) {
  *reinterpret_cast<VecT<T, N>*>(p) = x;
}

// Non-temporal (streaming) 16-byte accesses for data touched once per step:
// v_{n-1} is read once and v_{n+1} written once, so they should not displace
// the gathered rows of v_n from the caches.
template <typename T, int N>
struct NtVec;
template <> struct NtVec<float, 4> { typedef float type __attribute__((ext_vector_type(4))); };
template <> struct NtVec<float, 2> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct NtVec<float, 1> { typedef float type; };
template <> struct NtVec<double, 2> { typedef double type __attribute__((ext_vector_type(2))); };
template <> struct NtVec<double, 1> { typedef double type; };

template <typename T, int N>
__device__ __forceinline__ VecT<T, N> vload_nt(const T* p) {
  VecT<T, N> r;
  if constexpr (N == 4 && sizeof(T) == 8) {
    typedef typename NtVec<double, 2>::type V;
    const V a = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
    const V b = __builtin_nontemporal_load(reinterpret_cast<const V*>(p) + 1);
    r.v[0] = a[0]; r.v[1] = a[1]; r.v[2] = b[0]; r.v[3] = b[1];
  } else if constexpr (N == 1) {
    r.v[0] = __builtin_nontemporal_load(p);
  } else {
    typedef typename NtVec<T, N>::type V;
    const V a = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
#pragma unroll
    for (int i = 0; i < N; ++i) r.v[i] = a[i];
  }
  return r;
}

template <typename T, int N>
__device__ __forceinline__ void vstore_nt(T* p, const VecT<T, N>& x) {
  if constexpr (N == 4 && sizeof(T) == 8) {
    typedef typename NtVec<double, 2>::type V;
    V a, b;
    a[0] = x.v[0]; a[1] = x.v[1]; b[0] = x.v[2]; b[1] = x.v[3];
    __builtin_nontemporal_store(a, reinterpret_cast<V*>(p));
    __builtin_nontemporal_store(b, reinterpret_cast<V*>(p) + 1);
  } else if constexpr (N == 1) {
    __builtin_nontemporal_store(x.v[0], p);
  } else {
    typedef typename NtVec<T, N>::type V;
    V a;
#pragma unroll
    for (int i = 0; i < N; ++i) a[i] = x.v[i];
    __builtin_nontemporal_store(a, reinterpret_cast<V*>(p));
  }
}

constexpr int kGatherBatch = 4;   // neighbour loads in flight per lane

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of tiles so neighbour rows with small rank offsets are
// found in that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int grid_tiles) {
  const int per = grid_tiles >> 3;
  return (b & 7) * per + (b >> 3);
}

// Deterministic workgroup sum (valid in thread 0). sh: >= 4 doubles of LDS.
__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = ((sh[0] + sh[1]) + sh[2]) + sh[3];
  return r;
}

// Float32 storage with a 16-bit residual: x is kept as hi = float32(x)
// (round to nearest) and q = rint((x - hi) 2^(165 - e)), e = max(1, biased
// exponent of hi), so that hi + q 2^(e - 165) (exact in float64) is x to
// within 2^(e - 166), half a unit of hi's last place times 2^-15.
__device__ __forceinline__ double res_unit(float hi) {
  const uint32_t e = max((__float_as_uint(hi) >> 23) & 0xFFu, 1u);
  return __longlong_as_double((long long)(e + 858u) << 52);     // 2^(e - 165)
}
__device__ __forceinline__ double res_inv_unit(float hi) {
  const uint32_t e = max((__float_as_uint(hi) >> 23) & 0xFFu, 1u);
  return __longlong_as_double((long long)(1188u - e) << 52);    // 2^(165 - e)
}
__device__ __forceinline__ void res_encode(double x, float& hi, int16_t& q) {
  hi = (float)x;
  q = (int16_t)rint((x - (double)hi) * res_inv_unit(hi));
}
__device__ __forceinline__ double res_decode(float hi, int16_t q) {
  return fma((double)q, res_unit(hi), (double)hi);
}

// p[first] + p[first + stride] + ... (indices < n) in a fixed association:
// eight running sums, so that eight loads are in flight per lane, added in
// index order at the end.
__device__ __forceinline__ double strided_sum(const double* p, int n, int first, int stride) {
  double s[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) s[j] = 0.0;
  int t = first;
  for (; t + 7 * stride < n; t += 8 * stride) {
#pragma unroll
    for (int j = 0; j < 8; ++j) s[j] += p[t + j * stride];
  }
#pragma unroll
  for (int j = 0; j < 7; ++j)
    if (t + j * stride < n) s[j] += p[t + j * stride];
  return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// Sum of n partials in a fixed order (strided per thread, then tree).
__device__ __forceinline__ double sum_partials(const double* p, int n, double* sh) {
  return block_sum(strided_sum(p, n, threadIdx.x, kThreads), sh);
}

}  // namespace kpm
