// Fill kernels (used instead of hipMemsetAsync so that every clear is an
// ordinary kernel node when a caller captures the stream into a graph).
#include "kernels.hpp"

namespace aot {

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(T* __restrict__ p, int64_t n, T v) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    p[i] = v;
}

template <typename T>
static hipError_t fill(T* p, int64_t n, T v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = cdiv(n, kBlock);
  if (blocks > 8192) blocks = 8192;
  k_fill<T><<<(unsigned)blocks, kBlock, 0, s>>>(p, n, v);
  return hipGetLastError();
}

hipError_t fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) { return fill(p, n, v, s); }
hipError_t fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t s) { return fill(p, n, v, s); }

}  // namespace aot
