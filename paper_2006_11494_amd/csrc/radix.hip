// Stable LSD radix sort of (int32 key, int32 value) pairs, 8 bits per pass.
//
// A tile is 2048 pairs: each of the four waves of a workgroup walks 512
// consecutive pairs in eight coalesced steps of 64.  Within a step, lanes
// holding the same digit find each other with eight ballots (one per digit
// bit); the lowest such lane adds the group's size to the wave's digit
// counter in LDS, so no LDS atomic ever contends.  A pass is a histogram
// kernel, a device-wide scan of the digit-major [256][tiles] counts, and a
// scatter kernel that recomputes the same ranks; the order inside a tile is
// (wave, step, lane) = input order, which makes every pass stable.
#include "kernels.hpp"

namespace aot {

namespace {

constexpr int kDigits = 256;
constexpr int kSteps = 8;
constexpr int kTileKeys = kBlock * kSteps;          // 2048
constexpr int kWaveKeys = kWave * kSteps;           // 512

// Lanes (among the valid ones) whose 8-bit digit equals this lane's.
__device__ __forceinline__ uint64_t match_digit(int d, bool valid) {
  uint64_t peers = ballot(valid);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1;
    const uint64_t m = ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

__global__ __launch_bounds__(kBlock) void k_radix_hist(const int32_t* __restrict__ keys, int64_t n,
                                                       int shift, int32_t* __restrict__ hist,
                                                       int64_t ntiles) {
  __shared__ int32_t h[kDigits];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int w = threadIdx.x / kWave;
  const int64_t base = (int64_t)blockIdx.x * kTileKeys + (int64_t)w * kWaveKeys + lane_id();
#pragma unroll
  for (int st = 0; st < kSteps; ++st) {
    const int64_t i = base + st * kWave;
    const bool valid = i < n;
    const int d = valid ? (keys[i] >> shift) & (kDigits - 1) : 0;
    const uint64_t peers = match_digit(d, valid);
    if (valid && popc_below(peers) == 0) atomicAdd(&h[d], (int32_t)__popcll(peers));
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kBlock) void k_radix_scatter(
    const int32_t* __restrict__ kin, const int32_t* __restrict__ vin, int32_t* __restrict__ kout,
    int32_t* __restrict__ vout, int64_t n, int shift, const int64_t* __restrict__ offs,
    int64_t ntiles) {
  __shared__ int32_t wc[kWavesPerBlock][kDigits];
  for (int i = threadIdx.x; i < kWavesPerBlock * kDigits; i += kBlock) (&wc[0][0])[i] = 0;
  __syncthreads();
  const int w = threadIdx.x / kWave;
  const int64_t base = (int64_t)blockIdx.x * kTileKeys + (int64_t)w * kWaveKeys + lane_id();
  int32_t k[kSteps], v[kSteps], pos[kSteps];
#pragma unroll
  for (int st = 0; st < kSteps; ++st) {
    const int64_t i = base + st * kWave;
    const bool valid = i < n;
    k[st] = valid ? kin[i] : 0;
    v[st] = valid ? vin[i] : 0;
    const int d = (k[st] >> shift) & (kDigits - 1);
    const uint64_t peers = match_digit(d, valid);
    const int r = popc_below(peers);
    if (valid) {
      const int b = wc[w][d];            // every lane reads before the leader writes
      pos[st] = b + r;
      if (r == 0) wc[w][d] = b + (int32_t)__popcll(peers);
    }
  }
  __syncthreads();
  {
    int32_t run = 0;
    for (int q = 0; q < kWavesPerBlock; ++q) {
      const int32_t t = wc[q][threadIdx.x];
      wc[q][threadIdx.x] = run;
      run += t;
    }
  }
  __syncthreads();
#pragma unroll
  for (int st = 0; st < kSteps; ++st) {
    const int64_t i = base + st * kWave;
    if (i < n) {
      const int d = (k[st] >> shift) & (kDigits - 1);
      const int64_t o = offs[(int64_t)d * ntiles + blockIdx.x] + wc[w][d] + pos[st];
      kout[o] = k[st];
      vout[o] = v[st];
    }
  }
}

}  // namespace

size_t radix_workspace(int64_t n) {
  const int64_t ntiles = cdiv(n > 0 ? n : 1, kTileKeys);
  const int64_t cells = kDigits * ntiles;
  return (size_t)(align_up(cells * 4, 256) + align_up((cells + 1) * 8, 256)) +
         scan_workspace(cells);
}

hipError_t radix_sort_pairs(int32_t* keys, int32_t* vals, int32_t* keys_alt, int32_t* vals_alt,
                            int64_t n, int bits, void* tmp, hipStream_t s, int32_t** keys_out,
                            int32_t** vals_out) {
  *keys_out = keys;
  *vals_out = vals;
  if (n <= 1 || bits <= 0) return hipSuccess;
  const int64_t ntiles = cdiv(n, kTileKeys);
  const int64_t cells = kDigits * ntiles;
  char* t = static_cast<char*>(tmp);
  int32_t* hist = reinterpret_cast<int32_t*>(t);
  int64_t* offs = reinterpret_cast<int64_t*>(t + align_up(cells * 4, 256));
  void* stmp = t + align_up(cells * 4, 256) + align_up((cells + 1) * 8, 256);
  int32_t *ck = keys, *cv = vals, *ak = keys_alt, *av = vals_alt;
  for (int shift = 0; shift < bits; shift += 8) {
    k_radix_hist<<<(unsigned)ntiles, kBlock, 0, s>>>(ck, n, shift, hist, ntiles);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = exclusive_scan(hist, offs, cells, stmp, s);
    if (e != hipSuccess) return e;
    k_radix_scatter<<<(unsigned)ntiles, kBlock, 0, s>>>(ck, cv, ak, av, n, shift, offs, ntiles);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    int32_t* x = ck; ck = ak; ak = x;
    x = cv; cv = av; av = x;
  }
  *keys_out = ck;
  *vals_out = cv;
  return hipSuccess;
}

}  // namespace aot
