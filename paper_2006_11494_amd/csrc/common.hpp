// Shared device helpers for the AOT kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aot {

constexpr int kWave = 64;
constexpr int kBlock = 256;                 // threads per workgroup everywhere
constexpr int kWavesPerBlock = kBlock / kWave;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// The wave's lanes where p holds (the builtin takes the predicate as is,
// without turning it into an int and back).
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Number of set lanes strictly below this lane in `mask`.
__device__ __forceinline__ int popc_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// The bits of `mask` that belong to this lane's aligned group of G lanes,
// shifted down to bit 0.
template <int G>
__device__ __forceinline__ uint64_t group_bits(uint64_t mask) {
  if constexpr (G == kWave) return mask;
  const int base = lane_id() & ~(G - 1);
  return (mask >> base) & ((1ull << G) - 1ull);
}

// Set lanes below this one inside its G-lane group.
template <int G>
__device__ __forceinline__ int popc_below_in_group(uint64_t mask) {
  if constexpr (G == kWave) return popc_below(mask);
  const int in = lane_id() & (G - 1);
  return __popcll(group_bits<G>(mask) & ((1ull << in) - 1ull));
}

template <int G, typename T>
__device__ __forceinline__ T group_sum(T x) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, G);
  return x;
}

// Sum of x over the lanes below this one inside its G-lane group.
template <int G, typename T>
__device__ __forceinline__ T group_exclusive_sum(T x) {
  const int in = lane_id() & (G - 1);
  T inc = x;
#pragma unroll
  for (int o = 1; o < G; o <<= 1) {
    const T y = __shfl_up(inc, o, G);
    if (in >= o) inc += y;
  }
  return inc - x;
}

// Inclusive prefix sum across the 64 lanes of a wave.
template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T y = __shfl_up(x, o, kWave);
    if (l >= o) x += y;
  }
  return x;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

// Exclusive prefix over a 256-thread block; returns this thread's exclusive
// prefix and writes the block total to *total.  `tmp` holds kWavesPerBlock+1.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T x, T* tmp, T* total) {
  const int w = threadIdx.x / kWave;
  T inc = wave_inclusive_scan(x);
  if (lane_id() == kWave - 1) tmp[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T run = 0;
    for (int i = 0; i < kWavesPerBlock; ++i) {
      T t = tmp[i];
      tmp[i] = run;
      run += t;
    }
    tmp[kWavesPerBlock] = run;
  }
  __syncthreads();
  T r = tmp[w] + inc - x;
  *total = tmp[kWavesPerBlock];
  __syncthreads();
  return r;
}

template <typename T>
__device__ __forceinline__ T block_sum(T x, T* tmp) {
  const int w = threadIdx.x / kWave;
  x = wave_sum(x);
  if (lane_id() == 0) tmp[w] = x;
  __syncthreads();
  T s = 0;
#pragma unroll
  for (int i = 0; i < kWavesPerBlock; ++i) s += tmp[i];
  __syncthreads();
  return s;
}

// First index in a[0, len) whose value is >= key (a ascending).
__device__ __forceinline__ int64_t lower_bound(const int32_t* __restrict__ a, int64_t len,
                                               int32_t key) {
  int64_t lo = 0, hi = len;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ bool contains_sorted(const int32_t* __restrict__ a, int64_t len,
                                                int32_t key) {
  int64_t i = lower_bound(a, len, key);
  return i < len && a[i] == key;
}

__device__ __forceinline__ void sort3(int32_t& a, int32_t& b, int32_t& c) {
  int32_t t;
  if (a > b) { t = a; a = b; b = t; }
  if (b > c) { t = b; b = c; c = t; }
  if (a > b) { t = a; a = b; b = t; }
}

__host__ __device__ __forceinline__ int ceil_log2(int64_t x) {
  int k = 0;
  while ((int64_t(1) << k) < x) ++k;
  return k;
}

}  // namespace aot
