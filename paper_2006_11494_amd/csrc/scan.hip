// Device-wide exclusive prefix sum (int32 or int64 in, int64 out).
//
// Three phases over tiles of 4096 items: per-tile sums, a (recursive) scan of
// the tile sums, then a per-tile scan seeded with the tile's offset.  Inside a
// tile each thread owns 16 consecutive items; lanes combine with a wave-level
// shuffle scan and the four waves through LDS.
#include "kernels.hpp"

namespace aot {

namespace {

constexpr int kItems = 16;
constexpr int kTile = kBlock * kItems;

template <typename T>
__device__ __forceinline__ void load_items(const T* __restrict__ in, int64_t n, int64_t base,
                                           T (&v)[kItems], bool aligned) {
  const int64_t i0 = base + (int64_t)threadIdx.x * kItems;
  if (aligned && i0 + kItems <= n) {
    if constexpr (sizeof(T) == 4) {
      const int4* p = reinterpret_cast<const int4*>(in + i0);
#pragma unroll
      for (int q = 0; q < kItems / 4; ++q) {
        int4 x = p[q];
        v[4 * q] = x.x; v[4 * q + 1] = x.y; v[4 * q + 2] = x.z; v[4 * q + 3] = x.w;
      }
    } else {
      const longlong2* p = reinterpret_cast<const longlong2*>(in + i0);
#pragma unroll
      for (int q = 0; q < kItems / 2; ++q) {
        longlong2 x = p[q];
        v[2 * q] = x.x; v[2 * q + 1] = x.y;
      }
    }
  } else {
#pragma unroll
    for (int k = 0; k < kItems; ++k) v[k] = (i0 + k < n) ? in[i0 + k] : T(0);
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_tile_sums(const T* __restrict__ in, int64_t n,
                                                      int64_t* __restrict__ sums, bool aligned) {
  __shared__ int64_t tmp[kWavesPerBlock + 1];
  T v[kItems];
  load_items(in, n, (int64_t)blockIdx.x * kTile, v, aligned);
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) s += (int64_t)v[k];
  s = block_sum(s, tmp);
  if (threadIdx.x == 0) sums[blockIdx.x] = s;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_tile_scan(const T* __restrict__ in, int64_t n,
                                                      const int64_t* __restrict__ offs,
                                                      int64_t* __restrict__ out, bool aligned) {
  __shared__ int64_t tmp[kWavesPerBlock + 1];
  T v[kItems];
  const int64_t base = (int64_t)blockIdx.x * kTile;
  load_items(in, n, base, v, aligned);
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < kItems; ++k) s += (int64_t)v[k];
  int64_t total;
  int64_t run = block_exclusive_scan(s, tmp, &total) + (offs ? offs[blockIdx.x] : 0);
  const int64_t i0 = base + (int64_t)threadIdx.x * kItems;
  if (aligned && i0 + kItems <= n) {
    longlong2* p = reinterpret_cast<longlong2*>(out + i0);
#pragma unroll
    for (int q = 0; q < kItems / 2; ++q) {
      longlong2 x;
      x.x = run; run += (int64_t)v[2 * q];
      x.y = run; run += (int64_t)v[2 * q + 1];
      p[q] = x;
    }
  } else {
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
      if (i0 + k < n) out[i0 + k] = run;
      run += (int64_t)v[k];
    }
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
    out[n] = (offs ? offs[blockIdx.x] : 0) + total;
}

int64_t num_tiles(int64_t n) { return (n + kTile - 1) / kTile; }

template <typename T>
hipError_t scan_impl(const T* in, int64_t* out, int64_t n, char* tmp, hipStream_t s) {
  if (n <= 0) return fill_i64(out, 1, 0, s);
  const bool aligned = ((uintptr_t)in % 16 == 0) && ((uintptr_t)out % 16 == 0);
  const int64_t nt = num_tiles(n);
  if (nt == 1) {
    k_tile_scan<T><<<1, kBlock, 0, s>>>(in, n, nullptr, out, aligned);
    return hipGetLastError();
  }
  int64_t* sums = reinterpret_cast<int64_t*>(tmp);
  int64_t* offs = sums + align_up(nt, 32);
  char* next = reinterpret_cast<char*>(offs + align_up(nt + 1, 32));
  k_tile_sums<T><<<(unsigned)nt, kBlock, 0, s>>>(in, n, sums, aligned);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = scan_impl<int64_t>(sums, offs, nt, next, s);
  if (e != hipSuccess) return e;
  k_tile_scan<T><<<(unsigned)nt, kBlock, 0, s>>>(in, n, offs, out, aligned);
  return hipGetLastError();
}

}  // namespace

size_t scan_workspace(int64_t n) {
  size_t bytes = 0;
  int64_t nt = num_tiles(n);
  while (nt > 1) {
    bytes += sizeof(int64_t) * (size_t)(align_up(nt, 32) + align_up(nt + 1, 32));
    nt = num_tiles(nt);
  }
  return bytes + 256;
}

hipError_t exclusive_scan(const int32_t* in, int64_t* out, int64_t n, void* tmp, hipStream_t s) {
  return scan_impl<int32_t>(in, out, n, static_cast<char*>(tmp), s);
}

hipError_t exclusive_scan(const int64_t* in, int64_t* out, int64_t n, void* tmp, hipStream_t s) {
  return scan_impl<int64_t>(in, out, n, static_cast<char*>(tmp), s);
}

}  // namespace aot
