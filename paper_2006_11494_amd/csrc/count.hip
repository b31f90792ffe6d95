// Adaptive-orientation probe passes (Algorithm 3's two loops; Section 3.1,
// "The main idea"; Section 3.2, Correctness and Time Complexity).
//
// Every directed edge e = <u,v> of the oriented graph is charged to its owner
// b, the endpoint with the larger (deg+, label) (equal out-degrees go by the
// label, the footnote of Section 3.2; labels are ranks, or original ids); the
// other endpoint s is probed: each w in N+(s) is looked up in an index of
// N+(b), so edge e costs min(deg+(u), deg+(v)) look-ups.
//
// Edges fall into buckets:
//  * heavy owner classes (deg+(b) >= heavy_min), one per ceil(log2 deg+(b)):
//    owner-grouped as in Algorithm 3, where a pivot builds its index once
//    (Section 3.2, the remark on the bitmap).  A workgroup takes a work item
//    = an owner and its whole row if that holds at most kItemSpan
//    neighbours, else a window of up to kItemSpan of its out-neighbours or of
//    its in-neighbours (with in-lists sorted by label, the in-items of a long
//    in-list each hold a narrow run of the edge order), compacts the
//    neighbours it owns into LDS with a prefix sum
//    of their out-degrees, stages N+(b) in LDS (bitmap over [min, max] of the
//    list, open-addressing hash, or a sorted copy; a list too long or too
//    wide for its launch's LDS takes the sorted copy, then a global binary
//    search), and then spreads the
//    flattened probes over all its lanes: each lane takes consecutive probes,
//    so reads of the probed out-lists are coalesced and no lane idles on
//    short lists.
//  * light bins by c = min(deg+) (owners below heavy_min): edge-centric, G
//    lanes per edge, each lane binary-searching the short sorted N+(b).
// The count pass writes cnt[e]; an exclusive scan gives each edge its slot in
// the global triangle list; the write pass repeats the probes and stores the
// hits of an edge in ascending w at those slots.
//
// The same passes take the comparison costs of Section 2 as strategies (the
// fixed orientation of kClist, CF's merge, CF-Hash's per-edge probing) with
// the same output, and, in digest mode, count each triangle once for its
// three edges (the per-edge support) instead of storing it.
#include <algorithm>
#include <climits>
#include <cmath>
#include <vector>

#include "kernels.hpp"

namespace aot {

namespace {

constexpr int kLightBins = 8;       // c in {1}, {2}, (2,4], (4,8], ..., last bin open-ended
constexpr int kHeavyClasses = 16;   // owner classes by ceil(log2 deg+(b))
constexpr int kHeavyBase = 16;      // bucket id of heavy class 0
constexpr int kItemSpan = 512;      // neighbours of one owner per work item
constexpr int kLine = 32;           // int32 entries per 128-byte line (count-pass skip)
constexpr int32_t kSkipMin = 2 * kLine;  // shorter probed lists are probed whole
#ifndef AOT_MAX_INDEX_WORDS
#define AOT_MAX_INDEX_WORDS 12288
#endif
constexpr int kMaxIndexWords = AOT_MAX_INDEX_WORDS;  // LDS index cap (12288: 48 KiB, a bitmap
                                                     // window of 393216 ids)
#ifndef AOT_PROBE_UNROLL
#define AOT_PROBE_UNROLL 8
#endif
#ifndef AOT_EMIT_UNROLL
#define AOT_EMIT_UNROLL 8
#endif
constexpr int kUnroll = AOT_PROBE_UNROLL;       // 64-probe windows in flight per wave: count pass
constexpr int kEmitUnroll = AOT_EMIT_UNROLL;    // and write pass
constexpr int kGrid = 4096;
constexpr int kDefaultHeavyMin = 64;
#ifndef AOT_SPLIT_ITEMS
#define AOT_SPLIT_ITEMS 1
#endif
// rows longer than this are windowed separately over out- and in-list
constexpr int kSplitAbove = AOT_SPLIT_ITEMS ? kItemSpan : (1 << 30);
constexpr int kPlanWords = 64;      // resolved table [32], learned flag, valid flag, strategy
constexpr int kFeatures = AOT_NUM_FEATURES;
constexpr int kOptions = AOT_NUM_OPTIONS;

static_assert(kNumBuckets == kHeavyBase + kHeavyClasses, "bucket layout");

// per-bucket statistics (int64, device), bucket = light bin or kHeavyBase + class
enum : int {
  kSEdges = 0, kSProbes, kSTriangles, kSItems, kSStaged, kSCursor, kSItemBase, kSSpan, kSDb,
  kSLookups,   // heavy: probes the write pass makes (the hit spans of the count pass)
  kSCountLooks,  // heavy: probes the count pass makes (each list from its line below min N+(b))
  kStats,
};
constexpr int kStatWords = kNumBuckets * kStats;

enum Arm : int { kArmBitmap = 0, kArmHash = 1, kArmGlobal = 2, kArmSorted = 3, kNumArms = 4 };

__host__ __device__ __forceinline__ int light_bin(int32_t c) {
  const int k = c <= 1 ? 0 : ceil_log2(c);
  return k < kLightBins ? k : kLightBins - 1;
}

__host__ __device__ __forceinline__ int heavy_class(int32_t db) {
  const int h = ceil_log2(db);
  return h < kHeavyClasses ? h : kHeavyClasses - 1;
}

// Probe strategies (the comparisons of Sections 4.1 and 4.2 and the costs of Section 2):
// which list an edge probes and into what.  All list the same triangles in
// the same order.
constexpr int kStratAdaptive = 0;   // Algorithm 3: min side into the owner's index
constexpr int kStratHead = 1;       // fixed orientation: N+(v) into N+(u) (kClist cost)
constexpr int kStratMerge = 2;      // Algorithm 1: merge N+(u) with N+(v)
constexpr int kStratPerEdge = 3;    // min side into the larger list, edge by edge
constexpr int kNumStrategies = 4;

struct EdgeEnds {
  int32_t s, b;      // probe side, owner
  int32_t c, db;     // deg+(s), deg+(b)
};

// head = false: the adaptive rule.  head = true: the fixed orientation, where
// the tail u always owns the edge and its head's list is probed.
__device__ __forceinline__ EdgeEnds edge_ends(const int64_t* __restrict__ orow, int32_t u,
                                              int32_t v, bool head) {
  const int32_t du = (int32_t)(orow[u + 1] - orow[u]);
  const int32_t dv = (int32_t)(orow[v + 1] - orow[v]);
  // u < v in rank, so on a tie u has the smaller (deg+, id) and is probed
  EdgeEnds r;
  if (!head && du <= dv) { r.s = u; r.b = v; r.c = du; r.db = dv; }
  else { r.s = v; r.b = u; r.c = dv; r.db = du; }
  return r;
}

__device__ __forceinline__ unsigned long long* u64p(int64_t* p) {
  return reinterpret_cast<unsigned long long*>(p);
}

__device__ __forceinline__ int32_t block_min(int32_t x, int32_t* tmp) {
  for (int o = kWave / 2; o > 0; o >>= 1) x = min(x, __shfl_xor(x, o, kWave));
  if (lane_id() == 0) tmp[threadIdx.x / kWave] = x;
  __syncthreads();
  int32_t r = tmp[0];
  for (int q = 1; q < kWavesPerBlock; ++q) r = min(r, tmp[q]);
  __syncthreads();
  return r;
}

__device__ __forceinline__ int32_t block_max(int32_t x, int32_t* tmp) {
  for (int o = kWave / 2; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o, kWave));
  if (lane_id() == 0) tmp[threadIdx.x / kWave] = x;
  __syncthreads();
  int32_t r = tmp[0];
  for (int q = 1; q < kWavesPerBlock; ++q) r = max(r, tmp[q]);
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------- binning

// Per-bucket edge and probe counts, and the probe total.
// Also stores each edge's light bin (or 0xFF) for the scatter.
__global__ __launch_bounds__(kBlock) void k_bin_count(int64_t m, const int64_t* __restrict__ orow,
                                                      const int32_t* __restrict__ ocol,
                                                      const int32_t* __restrict__ otail,
                                                      int32_t heavy_min, int32_t strategy,
                                                      int32_t* __restrict__ cnt,
                                                      uint8_t* __restrict__ code,
                                                      int64_t* __restrict__ stats,
                                                      unsigned long long* __restrict__ probes) {
  __shared__ unsigned long long se[kNumBuckets], sp[kNumBuckets], sd[kNumBuckets], sk;
  if (threadIdx.x < kNumBuckets) { se[threadIdx.x] = 0; sp[threadIdx.x] = 0; sd[threadIdx.x] = 0; }
  if (threadIdx.x == 0) sk = 0;
  __syncthreads();
  const bool merge = strategy == kStratMerge;
  unsigned long long skipped = 0;       // merge cost of edges with an empty list
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * kBlock) {
    const EdgeEnds x = edge_ends(orow, otail[e], ocol[e], strategy == kStratHead);
    // the edge's cost: probes of N+(s), or both lists for a merge
    const int32_t cost = merge ? x.c + x.db : x.c;
    int bucket;
    if (x.db >= heavy_min) bucket = kHeavyBase + heavy_class(x.db);
    else if (x.c == 0) { cnt[e] = 0; code[e] = 0xFF; skipped += (unsigned)cost; continue; }
    else bucket = light_bin(cost);
    code[e] = bucket < kLightBins ? (uint8_t)bucket : (uint8_t)0xFF;
    atomicAdd(&se[bucket], 1ull);
    atomicAdd(&sp[bucket], (unsigned long long)cost);
    atomicAdd(&sd[bucket], (unsigned long long)x.db);
  }
  if (merge) {
    skipped = wave_sum(skipped);
    if (lane_id() == 0 && skipped) atomicAdd(&sk, skipped);
  }
  __syncthreads();
  if (threadIdx.x == 0 && sk) atomicAdd(probes, sk);
  if (threadIdx.x < kNumBuckets && se[threadIdx.x]) {
    atomicAdd(u64p(&stats[threadIdx.x * kStats + kSEdges]), se[threadIdx.x]);
    atomicAdd(u64p(&stats[threadIdx.x * kStats + kSProbes]), sp[threadIdx.x]);
    atomicAdd(u64p(&stats[threadIdx.x * kStats + kSDb]), sd[threadIdx.x]);
    atomicAdd(probes, sp[threadIdx.x]);
  }
}

// Light edges into their bins, in edge order inside every bin, so that a
// window of the edge order is one contiguous run of each bin.  k_bin_hist
// counts every chunk's edges per bin; an exclusive scan over (bin, chunk)
// gives each chunk's first slot in each bin; k_bin_place writes each chunk's
// edges in order, ranked with per-wave ballots.
constexpr int kScatterChunk = 8192;

__global__ __launch_bounds__(kBlock) void k_bin_hist(int64_t m, const uint8_t* __restrict__ code,
                                                     int64_t nchunks, int32_t* __restrict__ hist) {
  __shared__ int32_t cnt[kLightBins];
  int32_t mine[kLightBins];
  for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    if (threadIdx.x < kLightBins) cnt[threadIdx.x] = 0;
#pragma unroll
    for (int q = 0; q < kLightBins; ++q) mine[q] = 0;
    __syncthreads();
    const int64_t c0 = c * kScatterChunk, c1 = min(m, c0 + kScatterChunk);
    for (int64_t e = c0 + threadIdx.x; e < c1; e += kBlock) {
      const int bin = code[e];
#pragma unroll
      for (int q = 0; q < kLightBins; ++q) mine[q] += (int32_t)__popcll(ballot(bin == q));
    }
    if (lane_id() == 0)
#pragma unroll
      for (int q = 0; q < kLightBins; ++q)
        if (mine[q]) atomicAdd(&cnt[q], mine[q]);
    __syncthreads();
    if (threadIdx.x < kLightBins) hist[threadIdx.x * nchunks + c] = cnt[threadIdx.x];
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_bin_place(int64_t m, const uint8_t* __restrict__ code,
                                                      int64_t nchunks,
                                                      const int64_t* __restrict__ hoff,
                                                      int32_t* __restrict__ elist) {
  __shared__ int64_t run[kLightBins];
  __shared__ int32_t wc[kWavesPerBlock][kLightBins];
  const int w = threadIdx.x / kWave;
  for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
    if (threadIdx.x < kLightBins) run[threadIdx.x] = hoff[threadIdx.x * nchunks + c];
    __syncthreads();
    const int64_t c0 = c * kScatterChunk, c1 = min(m, c0 + kScatterChunk);
    for (int64_t r0 = c0; r0 < c1; r0 += kBlock) {
      const int64_t e = r0 + threadIdx.x;
      const int bin = e < c1 ? code[e] : 0xFF;
      uint64_t same = 0;
#pragma unroll
      for (int q = 0; q < kLightBins; ++q) {
        const uint64_t mask = ballot(bin == q);
        if (lane_id() == 0) wc[w][q] = (int32_t)__popcll(mask);
        if (bin == q) same = mask;
      }
      __syncthreads();
      if (bin < kLightBins) {
        int64_t pos = run[bin] + popc_below(same);
        for (int x = 0; x < w; ++x) pos += wc[x][bin];
        elist[pos] = (int32_t)e;
      }
      __syncthreads();
      if (threadIdx.x < kLightBins) {
        int32_t t = 0;
        for (int x = 0; x < kWavesPerBlock; ++x) t += wc[x][threadIdx.x];
        run[threadIdx.x] += t;
      }
      __syncthreads();
    }
  }
}

// lsamp[q] = ocol[kLine * q]: one entry per line of the oriented out-lists,
// which the count pass searches for where to start probing a list.
__global__ __launch_bounds__(kBlock) void k_line_samples(int64_t m, const int32_t* __restrict__ ocol,
                                                         int32_t* __restrict__ lsamp) {
  const int64_t lines = (m + kLine - 1) / kLine;
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < lines;
       q += (int64_t)gridDim.x * kBlock)
    lsamp[q] = ocol[q * kLine];
}

// The items of one class whose owned edges hold triangles in [first, first +
// count) (their smallest and largest owned edge, from the count pass, bound
// the item's part of the list), appended to list in any order (each item
// writes fixed slots) with one atomic per wave.  A write window then visits
// only these instead of testing every item of the class on one workgroup each.
__global__ __launch_bounds__(kBlock) void k_window_items(int64_t base, int64_t items,
                                                         const int2* __restrict__ item_e,
                                                         const int64_t* __restrict__ tri_off,
                                                         int64_t first, int64_t count,
                                                         int32_t* __restrict__ list,
                                                         int32_t* __restrict__ n) {
  for (int64_t i0 = (int64_t)blockIdx.x * kBlock; i0 < items; i0 += (int64_t)gridDim.x * kBlock) {
    const int64_t i = i0 + threadIdx.x;
    bool in = false;
    if (i < items) {
      const int2 r = item_e[base + i];
      if (r.y >= r.x) {
        const int64_t t0 = tri_off[r.x], t1 = tri_off[r.y + 1];
        in = t1 > first && t0 < first + count && t1 > t0;
      }
    }
    const uint64_t m = ballot(in);
    if (!m) continue;
    const int leader = __ffsll((long long)m) - 1;
    int32_t at = 0;
    if (lane_id() == leader) at = atomicAdd(n, (int32_t)__popcll(m));
    at = __shfl(at, leader, kWave);
    if (in) list[at + popc_below(m)] = (int32_t)(base + i);
  }
}

// Work items per heavy class, the owner-list entries they stage, and the
// largest owner-list span of the class (which sizes the bitmap arm's LDS).
__global__ __launch_bounds__(kBlock) void k_item_count(int32_t n, const int64_t* __restrict__ orow,
                                                       const int32_t* __restrict__ ocol,
                                                       const int64_t* __restrict__ irow,
                                                       int32_t heavy_min, bool head,
                                                       int64_t* __restrict__ stats) {
  __shared__ unsigned long long si[kHeavyClasses], ss[kHeavyClasses], sx[kHeavyClasses];
  if (threadIdx.x < kHeavyClasses) { si[threadIdx.x] = 0; ss[threadIdx.x] = 0; sx[threadIdx.x] = 0; }
  __syncthreads();
  for (int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x; b < n;
       b += (int64_t)gridDim.x * kBlock) {
    const int64_t ob = orow[b];
    const int64_t db = orow[b + 1] - ob;
    if (db < heavy_min) continue;
    const int64_t din = head ? 0 : irow[b + 1] - irow[b];
    const int64_t k = db + din <= kSplitAbove
                          ? (db + din + kItemSpan - 1) / kItemSpan
                          : (db + kItemSpan - 1) / kItemSpan + (din + kItemSpan - 1) / kItemSpan;
    const int h = heavy_class((int32_t)db);
    const unsigned long long span = (unsigned long long)(ocol[ob + db - 1] - ocol[ob] + 1);
    atomicAdd(&si[h], (unsigned long long)k);
    atomicAdd(&ss[h], (unsigned long long)(k * db));
    atomicMax(&sx[h], span);
  }
  __syncthreads();
  if (threadIdx.x < kHeavyClasses && si[threadIdx.x]) {
    int64_t* st = stats + (kHeavyBase + threadIdx.x) * kStats;
    atomicAdd(u64p(&st[kSItems]), si[threadIdx.x]);
    atomicAdd(u64p(&st[kSStaged]), ss[threadIdx.x]);
    atomicMax(u64p(&st[kSSpan]), sx[threadIdx.x]);
  }
}

// Work items into their classes; one global atomic per wave and class.
__global__ __launch_bounds__(kBlock) void k_item_scatter(int32_t n, const int64_t* __restrict__ orow,
                                                         const int64_t* __restrict__ irow,
                                                         int32_t heavy_min, bool head,
                                                         int64_t* __restrict__ stats,
                                                         int2* __restrict__ items) {
  __shared__ int64_t base[kHeavyClasses];
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int q = 0; q < kHeavyClasses; ++q) {
      base[q] = run;
      run += stats[(kHeavyBase + q) * kStats + kSItems];
    }
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x < kHeavyClasses)
    stats[(kHeavyBase + threadIdx.x) * kStats + kSItemBase] = base[threadIdx.x];
  for (int64_t b0 = (int64_t)blockIdx.x * kBlock; b0 < n; b0 += (int64_t)gridDim.x * kBlock) {
    const int64_t b = b0 + threadIdx.x;
    int h = -1;
    int32_t k = 0, kout = 0;
    int32_t dbo = 0;
    if (b < n) {
      const int64_t db = orow[b + 1] - orow[b];
      if (db >= heavy_min) {
        const int64_t din = head ? 0 : irow[b + 1] - irow[b];
        if (db + din <= kSplitAbove) {        // windows over the whole row
          k = (int32_t)((db + din + kItemSpan - 1) / kItemSpan);
          kout = k;
        } else {
          kout = (int32_t)((db + kItemSpan - 1) / kItemSpan);
          k = kout + (int32_t)((din + kItemSpan - 1) / kItemSpan);
        }
        h = heavy_class((int32_t)db);
        dbo = (int32_t)db;
      }
    }
    if (!ballot(h >= 0)) continue;
    for (int q = 0; q < kHeavyClasses; ++q) {
      const uint64_t mask = ballot(h == q);
      if (!mask) continue;
      // exclusive prefix of k over the lanes of this class
      int32_t kin = h == q ? k : 0;
      int32_t inc = wave_inclusive_scan(kin);
      const int32_t tot = __shfl(inc, 63, kWave);
      const int leader = __ffsll((long long)mask) - 1;
      long long at = 0;
      if (lane_id() == leader)
        at = (long long)atomicAdd(u64p(&stats[(kHeavyBase + q) * kStats + kSCursor]),
                                  (unsigned long long)tot);
      at = __shfl(at, leader, kWave);
      if (h == q) {
        const int64_t first = base[q] + at + (inc - kin);
        // out-list windows, then in-list windows: an item of a longer row
        // never mixes the two
        for (int32_t r = 0; r < k; ++r)
          items[first + r] = make_int2((int32_t)b, r < kout ? r * kItemSpan
                                                            : dbo + (r - kout) * kItemSpan);
        (void)dbo;
      }
    }
  }
}

// ---------------------------------------------------------------- LDS index

__device__ __forceinline__ uint32_t hash_slot(int32_t w) { return (uint32_t)w * 0x9E3779B1u; }

struct Index {
  int32_t lo, span;   // bitmap window
  uint32_t mask;      // hash table size - 1
  int shift;          // hash: 32 - log2(size)
  const int32_t* list;
  int32_t len;
};

__host__ __device__ __forceinline__ int64_t floor_pow2(int64_t x) {
  int64_t p = 1;
  while (p * 2 <= x) p *= 2;
  return p;
}

// The arm an owner actually uses: the requested one if its list fits that
// arm in `words` LDS words, else the next that fits (bitmap or hash ->
// sorted -> global).  A bitmap too wide for its window goes to the sorted
// copy, which needs the fewest words and probes faster than the hash on
// every workload measured.
__host__ __device__ __forceinline__ int resolve_arm(int arm, int64_t db, int64_t span, int words) {
  if (arm == kArmBitmap && span > (int64_t)words * 32) arm = kArmSorted;
  if (arm == kArmHash && 2 * db > floor_pow2(words)) arm = kArmSorted;
  if (arm == kArmSorted && db > words) arm = kArmGlobal;
  return arm;
}

template <int ARM>
__device__ __forceinline__ Index build_index(const int32_t* __restrict__ a, int32_t db,
                                             uint32_t* lds) {
  Index ix;
  ix.list = a;
  ix.len = db;
  ix.lo = a[0];
  ix.span = a[db - 1] - ix.lo + 1;
  ix.mask = 0;
  ix.shift = 0;
  if constexpr (ARM == kArmBitmap) {
    const int words = (ix.span + 31) >> 5;
    for (int i = threadIdx.x; i < words; i += kBlock) lds[i] = 0u;
    __syncthreads();
    for (int i = threadIdx.x; i < db; i += kBlock) {
      const int32_t off = a[i] - ix.lo;
      atomicOr(&lds[off >> 5], 1u << (off & 31));
    }
  } else if constexpr (ARM == kArmHash) {
    int size = 2;
    while (size < 2 * db) size <<= 1;
    ix.mask = (uint32_t)size - 1u;
    ix.shift = 32 - ceil_log2(size);
    for (int i = threadIdx.x; i < size; i += kBlock) lds[i] = 0xFFFFFFFFu;
    __syncthreads();
    for (int i = threadIdx.x; i < db; i += kBlock) {
      const uint32_t w = (uint32_t)a[i];
      uint32_t h = hash_slot((int32_t)w) >> ix.shift;
      while (atomicCAS(&lds[h], 0xFFFFFFFFu, w) != 0xFFFFFFFFu) h = (h + 1) & ix.mask;
    }
  } else if constexpr (ARM == kArmSorted) {
    for (int i = threadIdx.x; i < db; i += kBlock) lds[i] = (uint32_t)a[i];
  }
  __syncthreads();
  return ix;
}

template <int ARM>
__device__ __forceinline__ bool index_has(const Index& ix, const uint32_t* lds, int32_t w) {
  if constexpr (ARM == kArmBitmap) {
    // branchless: an id outside the window reads word 0 and is masked off
    const uint32_t off = (uint32_t)(w - ix.lo);
    const bool in = off < (uint32_t)ix.span;
    const uint32_t word = lds[(in ? off : 0u) >> 5];
    return in & ((word >> (off & 31)) & 1u);
  } else if constexpr (ARM == kArmHash) {
    uint32_t h = hash_slot(w) >> ix.shift;
    while (true) {
      const uint32_t k = lds[h];
      if (k == (uint32_t)w) return true;
      if (k == 0xFFFFFFFFu) return false;
      h = (h + 1) & ix.mask;
    }
  } else if constexpr (ARM == kArmSorted) {
    const int32_t* l = reinterpret_cast<const int32_t*>(lds);
    int lo = 0, hi = ix.len;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (l[mid] < w) lo = mid + 1; else hi = mid;
    }
    return lo < ix.len && l[lo] == w;
  } else {
    return contains_sorted(ix.list, ix.len, w);
  }
}

// index_has for U probes at once.  The sorted copy takes a branchless search
// whose trip count depends only on the owner's deg+ (the same on every lane):
// each step narrows [b, b + n) to the half holding the last entry <= w with
// one LDS read, a compare and a select, and the U searches advance together so
// their reads issue back to back.
template <int ARM, int U>
__device__ __forceinline__ void index_has_all(const Index& ix, const uint32_t* lds,
                                              const int32_t (&w)[U], bool (&has)[U]) {
  if constexpr (ARM == kArmSorted) {
    typedef const __attribute__((address_space(3))) int32_t* LdsPtr;   // 32-bit LDS address
    const LdsPtr l = (LdsPtr)lds;
    const int len = __builtin_amdgcn_readfirstlane(ix.len);   // >= 1: an owner has out-neighbours
    constexpr int G = U < 4 ? U : 4;     // searches in step together (register budget)
#pragma unroll
    for (int g = 0; g < U; g += G) {
      LdsPtr b[G];
#pragma unroll
      for (int u = 0; u < G; ++u) b[u] = l;
      for (int n = len; n > 1;) {
        const int half = n >> 1;
#pragma unroll
        for (int u = 0; u < G; ++u) b[u] = b[u][half] <= w[g + u] ? b[u] + half : b[u];
        n -= half;
      }
#pragma unroll
      for (int u = 0; u < G; ++u) has[g + u] = *b[u] == w[g + u];
    }
  } else {
#pragma unroll
    for (int u = 0; u < U; ++u) has[u] = index_has<ARM>(ix, lds, w[u]);
  }
}

// ---------------------------------------------------------------- heavy path

// Largest k in [kc, K) with pre[k] <= p, given pre[kc] <= p < pre[K].
__device__ __forceinline__ int advance(const int32_t* pre, int kc, int K, int32_t p) {
  if (pre[kc + 1] > p) return kc;
  int lo = kc + 1, step = 1, hi;
  while (true) {
    hi = lo + step;
    if (hi >= K || pre[hi] > p) break;
    lo = hi;
    step <<= 1;
  }
  if (hi > K) hi = K;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= p) lo = mid; else hi = mid;
  }
  return lo;
}

struct HeavyArgs {
  int32_t arms[kHeavyClasses];  // requested arm of each heavy class
  int idx_words;                // LDS words of the index (dynamic shared memory)
  const int2* items;
  int2* item_e;                 // per item: smallest and largest owned edge id with
                                // probes (count pass writes, write pass reads)
  int32_t* ieid;                // per in-list entry: the id of an owned in-edge
                                // (count pass writes, write pass reads)
  int32_t* hfirst;              // per owned edge with triangles: the ocol index of its
                                // first hit (count pass writes, write pass reads)
  int64_t* look_stat;           // count pass: the bucket's write-pass probes
  int64_t* made_stat = nullptr; // count pass: the bucket's own probes
  const int32_t* lsamp = nullptr;  // count pass: lsamp[q] = ocol[kLine * q], the first
                                   // entry of every kLine-entry line of the out-lists
  int64_t item_base, item_count;
  const int32_t* item_list = nullptr;     // write pass, windows: the items to visit,
  const int32_t* item_list_n = nullptr;   // and how many (device), instead of them all
  const int64_t* orow;
  const int32_t* ocol;
  const int64_t* irow;
  const int32_t* icol;
  int32_t* cnt;                 // count pass
  int64_t* tri_stat;            // count pass: the bucket's triangle total
  const int64_t* tri_off;       // write pass
  const int32_t* perm;
  int64_t first, count;
  int64_t e_lo, e_hi;           // write pass: the edge range the window can touch, and
  int32_t y_lo, y_hi;           // the rows of its first and last edge
  int32_t* out;
  unsigned long long* digest;   // write pass in digest mode: {triangles, hash sum, hash xor}
  uint32_t* esup = nullptr;     // digest mode, optional: per-edge support
  int32_t head = 0;             // fixed orientation: b owns its out-edges only
};

// Digest mode with per-edge support: a triangle adds one to each of its three
// oriented edges (ids = indices into the out-lists).
__device__ __forceinline__ void add_support(uint32_t* esup, int64_t e0, int64_t e1, int64_t e2) {
  atomicAdd(&esup[e0], 1u);
  atomicAdd(&esup[e1], 1u);
  atomicAdd(&esup[e2], 1u);
}

// SplitMix64's output function (Steele, Lea and Flood, 2014) on state z.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Order-independent digest of a triangle list: each ascending triple
// (a, b, c) hashes to splitmix64(splitmix64(splitmix64(a) ^ b) ^ c); the
// digest is the count, the sum (mod 2^64) and the xor of the hashes.
struct Digest {
  uint64_t count = 0, sum = 0, xr = 0;
  __device__ __forceinline__ void add(int32_t a, int32_t b, int32_t c) {
    const uint64_t h = splitmix64(splitmix64(splitmix64((uint64_t)(uint32_t)a) ^
                                             (uint64_t)(uint32_t)b) ^ (uint64_t)(uint32_t)c);
    count += 1;
    sum += h;
    xr ^= h;
  }
};

// Block-wide reduction of the per-thread digests into the global one.
__device__ void flush_digest(const Digest& d, unsigned long long* out) {
  __shared__ unsigned long long red[3][kWavesPerBlock];
  uint64_t c = d.count, s = d.sum, x = d.xr;
  for (int o = kWave / 2; o > 0; o >>= 1) {
    c += __shfl_xor(c, o, kWave);
    s += __shfl_xor(s, o, kWave);
    x ^= __shfl_xor(x, o, kWave);
  }
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) { red[0][w] = c; red[1][w] = s; red[2][w] = x; }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t tc = 0, ts = 0, tx = 0;
    for (int q = 0; q < kWavesPerBlock; ++q) { tc += red[0][q]; ts += red[1][q]; tx ^= red[2][q]; }
    if (tc) {
      atomicAdd(&out[0], tc);
      atomicAdd(&out[1], ts);
      atomicXor(&out[2], tx);
    }
  }
}

// Write pass: a triangle at global index pos is stored if the window holds it.
__device__ __forceinline__ void store(const HeavyArgs& a, int64_t pos, int32_t t0, int32_t t1,
                                      int32_t t2) {
  if (pos >= a.first && pos < a.first + a.count) {
    // the list is written once and never read back here: streaming stores
    // keep it from evicting the out-lists the probes re-read
    int32_t* o = a.out + 3 * (pos - a.first);
    __builtin_nontemporal_store(t0, o);
    __builtin_nontemporal_store(t1, o + 1);
    __builtin_nontemporal_store(t2, o + 2);
  }
}

// Per-item shared state; arrays a pass does not use shrink to one entry, so
// the write pass's static LDS leaves room for one more workgroup per CU.
template <bool kEmit, bool kDigest = false>
struct HeavyShared {
  int32_t nb_src[kItemSpan];          // start of N+(y) minus its probe prefix (int32: m <= INT32_MAX)
  int64_t nb_base[kEmit ? kItemSpan : 1];
  int32_t nb_pre[kItemSpan + 1];
  int32_t nb_e[kEmit && !kDigest ? 1 : kItemSpan];   // edge ids: count, and digest support
  int32_t nb_acc[kEmit ? 1 : kItemSpan];             // count: hits
  int32_t nb_first[kEmit ? 1 : kItemSpan];   // count: first hit, as a probe index of the item
  unsigned long long looks;                  // count: the block's write-pass probes
  int32_t nb_py[kEmit ? kItemSpan : 1];
  int32_t wave_k[kWavesPerBlock + 1];
  int64_t scan_tmp[kWavesPerBlock + 1];
  int32_t red[kWavesPerBlock + 1];
};

// Per-lane hits of one 64-probe window, reduced per neighbour segment (lanes
// hold non-decreasing neighbour indices k).  Returns, for each lane, the
// number of hits of its own segment in lanes below it; `seg_total` gets the
// segment's hit count in the window (valid on the segment's first lane,
// flagged by `first_lane`).
__device__ __forceinline__ int segment_rank(bool valid, int k, uint64_t hm, int* seg_total,
                                            bool* first_lane) {
  const int lane = lane_id();
  const int kprev = __shfl_up(k, 1, kWave);
  const bool start = valid && (lane == 0 || kprev != k);
  const uint64_t sm = ballot(start);
  const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  const uint64_t below_sm = sm & upto;
  const int s = below_sm ? 63 - __clzll((long long)below_sm) : 0;  // my segment's first lane
  const uint64_t lt = (1ull << lane) - 1ull;
  const uint64_t from_s = ~((1ull << s) - 1ull);
  const int rank = __popcll(hm & lt & from_s);
  const uint64_t above = lane < 63 ? (sm & ~((2ull << lane) - 1ull)) : 0ull;
  const int end = above ? __ffsll((long long)above) - 1 : 64;
  const uint64_t seg = (end == 64 ? ~0ull : ((1ull << end) - 1ull)) & ~lt;
  *seg_total = __popcll(hm & seg);
  *first_lane = start;
  return rank;
}

// The probes of kUnroll consecutive 64-probe windows starting at w0: each
// lane finds the neighbour of its probe with a cursor chained across the
// windows (usually one LDS read: the probe lies in the same out-list as the
// previous one) and issues the load of the probed id.  kk = -1 marks lanes
// at or past `end`.
template <int U>
struct Windows {
  int kk[U];
  int32_t wv[U];
};

template <int U>
__device__ __forceinline__ void load_windows(Windows<U>& W, const int32_t* pre, const int32_t* src,
                                             const int32_t* __restrict__ ocol, int& kc, int32_t& nxt,
                                             int kend, int32_t w0, int32_t end) {
  const int lane = lane_id();
  // nxt = pre[kc + 1], where the neighbour after kc starts, carried across
  // calls: it changes only when a probe crosses it (kc < kend while probes
  // remain)
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int32_t p = w0 + u * kWave + lane;
    const bool live = p < end;
    // search only when some lane's probe crosses into a later neighbour
    if (ballot(live && p >= nxt)) {
      if (live && p >= nxt) {
        kc = advance(pre, kc + 1, kend, p);
        nxt = pre[kc + 1];
      }
    }
    W.kk[u] = live ? kc : -1;
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    // every lane loads; a lane past the end reads ocol[0] and is ignored.  The
    // LDS read takes a valid slot on every lane, so the windows' reads issue
    // together instead of behind a branch each
    const int32_t p = w0 + u * kWave + lane;
    const int k = W.kk[u];
    const int32_t s0 = src[k < 0 ? 0 : k];
    const int32_t at = k >= 0 ? s0 + p : 0;
    W.wv[u] = ocol[at];
  }
}

// Count pass over one item's compacted neighbours (K of them, P probes):
// waves take interleaved runs of kUnroll windows.  A window
// inside one out-list adds the popcount of its hit ballot to a wave-uniform
// accumulator, flushed to LDS when the neighbour changes; a window across a
// boundary sums hits per neighbour segment.
template <int ARM>
__device__ int64_t probe_count(HeavyShared<false>& sh, const uint32_t* lds, const HeavyArgs& a,
                               const Index& ix, int K, int32_t P) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);   // same on every lane
  const int lane = lane_id();
  constexpr int32_t kStride = kBlock * kUnroll;
  int kc = 0;
  int32_t nxt = sh.nb_pre[1];
  int64_t hits_wave = 0;
  int acc_k = -1;     // wave-uniform: neighbour being accumulated
  int acc = 0;        // and its hits so far,
  int32_t acc_f = 0;  // and the first of them (a probe index)
  // adds the accumulated hits and first hit to their neighbour's slot
  auto flush = [&]() {
    if (acc_k >= 0 && lane == 0 && acc) {
      atomicAdd(&sh.nb_acc[acc_k], acc);
      atomicMin(&sh.nb_first[acc_k], acc_f);
    }
  };
  for (int32_t w0 = wave * kWave * kUnroll; w0 < P; w0 += kStride) {
    Windows<kUnroll> cur;
    load_windows(cur, sh.nb_pre, sh.nb_src, a.ocol, kc, nxt, K, w0, P);
    bool has[kUnroll];
    index_has_all<ARM>(ix, lds, cur.wv, has);
    uint64_t hms[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) hms[u] = ballot((cur.kk[u] >= 0) & has[u]);
    // a full run inside one out-list: one accumulator update for all windows
    const int ka = __builtin_amdgcn_readfirstlane(cur.kk[0]);
    const int kb = __builtin_amdgcn_readlane(cur.kk[kUnroll - 1], kWave - 1);
    if (w0 + kWave * kUnroll <= P && ka == kb) {
      int c = 0;
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) c += (int)__popcll(hms[u]);
      if (c) {
        hits_wave += c;
        if (ka == acc_k) {
          acc += c;
        } else {
          flush();
          acc_k = ka;
          acc = c;
          // the run's first hit: this wave's first for the neighbour
          int32_t f = w0 + kWave * kUnroll;
#pragma unroll
          for (int u = kUnroll - 1; u >= 0; --u)
            if (hms[u]) f = w0 + u * kWave + (int32_t)__builtin_ctzll(hms[u]);
          acc_f = f;
        }
      }
      continue;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const bool valid = cur.kk[u] >= 0;
      const uint64_t hm = hms[u];
      if (!hm) continue;
      const int c = (int)__popcll(hm);
      hits_wave += c;
      const uint64_t vm = ballot(valid);
      const int k0 = __builtin_amdgcn_readfirstlane(cur.kk[u]);
      const int k1 = __builtin_amdgcn_readlane(cur.kk[u], 63 - __clzll((long long)vm));
      if (k0 == k1) {
        if (k0 == acc_k) {
          acc += c;
        } else {
          flush();
          acc_k = k0;
          acc = c;
          acc_f = w0 + u * kWave + (int32_t)__builtin_ctzll(hm);
        }
      } else {
        flush();
        acc_k = -1;
        acc = 0;
        int tot;
        bool first;
        const int below = segment_rank(valid, cur.kk[u], hm, &tot, &first);
        if (first && tot) atomicAdd(&sh.nb_acc[cur.kk[u]], tot);
        // a segment's first hit (none of its hits below it)
        if (((hm >> lane) & 1ull) && below == 0)
          atomicMin(&sh.nb_first[cur.kk[u]], w0 + u * kWave + lane);
      }
    }
  }
  flush();
  return lane == 0 ? hits_wave : 0;
}

// Write pass over one item's compacted neighbours.  Each wave owns a run of
// whole neighbours holding about a quarter of the probes and walks it in
// order, so an edge's hits are
// ranked by probe order inside one wave, with the running count of the
// current edge in a wave-uniform register.  In a window inside one out-list
// a hit's rank is its count of hitting lanes below it; a window across a
// boundary ranks hits per segment.
template <int ARM, bool kDigest>
__device__ void probe_emit(HeavyShared<true, kDigest>& sh, const uint32_t* lds, const HeavyArgs& a,
                           const Index& ix, int K, int32_t P, int32_t pb, Digest& dg) {
  // the wave's bounds are the same on every lane: kept in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int k_lo = __builtin_amdgcn_readfirstlane(sh.wave_k[wave]);
  const int k_hi = __builtin_amdgcn_readfirstlane(sh.wave_k[wave + 1]);
  if (k_lo >= k_hi) return;
  const int32_t p_lo = __builtin_amdgcn_readfirstlane(sh.nb_pre[k_lo]);
  const int32_t p_hi = __builtin_amdgcn_readfirstlane(sh.nb_pre[k_hi]);
  const int32_t* __restrict__ perm = a.perm;
  constexpr int32_t kStride = kWave * kEmitUnroll;
  int kc = k_lo;
  int32_t nxt = sh.nb_pre[k_lo + 1];
  int run_k = -1;     // wave-uniform: edge whose hits are being ranked
  int run = 0;        // hits of run_k emitted so far
  for (int32_t w0 = p_lo; w0 < p_hi; w0 += kStride) {
    Windows<kEmitUnroll> cur;
    load_windows(cur, sh.nb_pre, sh.nb_src, a.ocol, kc, nxt, k_hi, w0, p_hi);
    bool hit[kEmitUnroll];
    int32_t third[kEmitUnroll];
    index_has_all<ARM>(ix, lds, cur.wv, hit);
#pragma unroll
    for (int u = 0; u < kEmitUnroll; ++u) {
      hit[u] = (cur.kk[u] >= 0) & hit[u];
      third[u] = perm[hit[u] ? cur.wv[u] : 0];      // gathers issued before any store
    }
    // a full run inside one out-list: one base and one neighbour for all windows
    const int ka = __builtin_amdgcn_readfirstlane(cur.kk[0]);
    const int kb = __builtin_amdgcn_readlane(cur.kk[kEmitUnroll - 1], kWave - 1);
    if (w0 + kStride <= p_hi && ka == kb) {
      if (ka != run_k) { run_k = ka; run = 0; }
      const int64_t base = sh.nb_base[ka] + run;
      const int32_t py = sh.nb_py[ka];
      const int32_t lo = min(pb, py), hi = max(pb, py);
      int before = 0;
#pragma unroll
      for (int u = 0; u < kEmitUnroll; ++u) {
        const uint64_t hm = ballot(hit[u]);
        if (hit[u]) {
          const int32_t t = third[u];
          if constexpr (kDigest) {
            // the edge {b, y} is the same for the whole run: its count is
            // added once below; here <y, w> (the probed entry) and <b, w>
            dg.add(min(lo, t), max(lo, min(hi, t)), max(hi, t));
            if (a.esup) {
              atomicAdd(&a.esup[sh.nb_src[ka] + w0 + u * kWave + lane_id()], 1u);
              atomicAdd(&a.esup[(ix.list - a.ocol) + lower_bound(ix.list, ix.len, cur.wv[u])],
                        1u);
            }
          } else {
            store(a, base + before + popc_below(hm), min(lo, t), max(lo, min(hi, t)),
                        max(hi, t));
          }
        }
        before += (int)__popcll(hm);
      }
      if constexpr (kDigest)
        if (a.esup && lane_id() == 0 && before) atomicAdd(&a.esup[sh.nb_e[ka]], (uint32_t)before);
      run += before;
      continue;
    }
#pragma unroll
    for (int u = 0; u < kEmitUnroll; ++u) {
      const bool valid = cur.kk[u] >= 0;
      const uint64_t hm = ballot(hit[u]);
      if (!hm) continue;
      const uint64_t vm = ballot(valid);
      const int k0 = __builtin_amdgcn_readfirstlane(cur.kk[u]);
      const int k1 = __builtin_amdgcn_readlane(cur.kk[u], 63 - __clzll((long long)vm));
      int64_t pos;
      int k;
      if (k0 == k1) {
        k = k0;
        if (k != run_k) { run_k = k; run = 0; }
        pos = sh.nb_base[k] + run + popc_below(hm);
        run += (int)__popcll(hm);
      } else {
        int tot;
        bool first;
        k = cur.kk[u];
        const int rank = segment_rank(valid, k, hm, &tot, &first);
        pos = sh.nb_base[k] + (k == run_k ? run : 0) + rank;
        const int last_hits = (int)__popcll(hm & ballot(valid && k == k1));
        run = (k1 == run_k ? run : 0) + last_hits;
        run_k = k1;
      }
      if (hit[u]) {
        const int32_t py = sh.nb_py[k];
        int32_t t0 = pb, t1 = py, t2 = third[u];
        sort3(t0, t1, t2);
        if constexpr (kDigest) {
          dg.add(t0, t1, t2);
          if (a.esup)
            add_support(a.esup, sh.nb_e[k], sh.nb_src[k] + w0 + u * kWave + lane_id(),
                        (ix.list - a.ocol) + lower_bound(ix.list, ix.len, cur.wv[u]));
        } else {
          store(a, pos, t0, t1, t2);
        }
      }
    }
  }
}

template <int ARM, bool kEmit, bool kDigest>
__device__ int64_t run_item(HeavyShared<kEmit, kDigest>& sh, uint32_t* lds, const HeavyArgs& a,
                            const int32_t* list, int32_t db, int K, int32_t P, int32_t pb,
                            Digest& dg) {
  const Index ix = build_index<ARM>(list, db, lds);   // ends with a barrier
  if constexpr (!kEmit) {
    return probe_count<ARM>(sh, lds, a, ix, K, P);
  } else {
    probe_emit<ARM, kDigest>(sh, lds, a, ix, K, P, pb, dg);
    return 0;
  }
}

// One work item: owner b and a window of up to kItemSpan of its neighbours
// (out-list, then in-list).  Ends with a barrier.
// Entries of the out-list ocol[oy, oy + dy) that the count pass may skip: no
// entry below lo, the smallest of the owner's out-neighbours, can be in its
// index.  The line samples give the last kLine-aligned position q * kLine in
// the list whose entry is still below lo; everything before it is below lo
// too, so the probes start there (up to kLine - 1 known misses remain, the
// price of reading one sample per line instead of searching the list).

__device__ __forceinline__ int32_t skip_below(const int32_t* __restrict__ lsamp, int64_t oy,
                                              int32_t dy, int32_t lo) {
  // line indices fit in int32: m <= INT32_MAX
  const int32_t y0 = (int32_t)oy;
  int32_t q = (y0 + kLine - 1) / kLine;                 // samples inside the list
  int32_t n = (y0 + dy - 1) / kLine - q + 1;
  if (n <= 0 || lsamp[q] >= lo) return 0;
  // last sample below lo: lsamp[q] < lo holds, narrow [q, q + n)
  while (n > 1) {
    const int32_t half = n >> 1;
    if (lsamp[q + half] < lo) { q += half; n -= half; } else { n = half; }
  }
  return q * kLine - y0;
}

// kArms: the index arms compiled in (bit per Arm).  A launch whose class can
// resolve to fewer arms takes a kernel with only those, which is smaller.
constexpr unsigned kAllArms = (1u << kNumArms) - 1u;

template <bool kEmit, bool kDigest, unsigned kArms = kAllArms>
__device__ void heavy_item(HeavyShared<kEmit, kDigest>& sh, uint32_t* lds, const HeavyArgs& a, int64_t it,
                           int64_t& tri_block, int64_t& look_block, Digest& dg) {
  const int tid = threadIdx.x;
  if constexpr (kEmit) {
    // an item whose owned edges hold no slot in the window is skipped whole
    if (a.item_e) {
      const int2 r = a.item_e[it];
      if (r.y < r.x) return;
      if constexpr (!kDigest) {
        const int64_t lo = a.tri_off[r.x], hi = a.tri_off[r.y + 1];
        if (hi <= a.first || lo >= a.first + a.count) return;
      }
    }
  }
  const int2 item = a.items[it];
  const int32_t b = item.x;
  const int64_t ob = a.orow[b];
  const int32_t db = (int32_t)(a.orow[b + 1] - ob);
  const int64_t ib = a.irow[b];
  const int32_t deg = db + (a.head ? 0 : (int32_t)(a.irow[b + 1] - ib));
  const int32_t j0 = item.y;
  const int32_t lo_b = kEmit ? 0 : a.ocol[ob];   // smallest entry of the index
  // the whole row, or one window of the out-list or of the in-list
  const int32_t j1 = deg <= kSplitAbove ? min(deg, j0 + kItemSpan)
                                        : min(j0 < db ? db : deg, j0 + kItemSpan);

  // owned neighbours of this window, compacted with a prefix of their probe counts
  constexpr int kPer = kItemSpan / kBlock;
  int32_t ny[kPer], ne[kPer], nd[kPer];
  int64_t noy[kPer], nbase[kPer];
  bool keep[kPer];
  int64_t packed = 0;
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int32_t j = j0 + tid + i * kBlock;
    keep[i] = false;
    nd[i] = 0;
    ny[i] = 0; ne[i] = 0; noy[i] = 0; nbase[i] = 0;
    bool near = j < j1;
    int32_t y = 0, e = 0;
    const bool out_edge = j < db;
    if (near) {
      if (out_edge) {
        e = (int32_t)(ob + j);
        // write pass: an edge outside the window's edge range is dropped before any load
        if constexpr (kEmit) near = e >= a.e_lo && e < a.e_hi;
        if (near) y = a.ocol[ob + j];
      } else {
        y = a.icol[ib + (j - db)];
        // an in-edge <y, b> lies in row y: rows outside the window's rows are dropped
        if constexpr (kEmit) near = y >= a.y_lo && y <= a.y_hi;
      }
    }
    if (near) {
      const int64_t oy = a.orow[y];
      const int32_t dy = (int32_t)(a.orow[y + 1] - oy);
      const bool owned = a.head ? out_edge : dy < db || (dy == db && y < b);
      // an owned in-edge <y, b>: its id is b's place in N+(y), the list probed
      // next; the count pass finds it and keeps it for the write pass
      if (owned && !out_edge) {
        int32_t* slot = a.ieid + ib + (j - db);
        if constexpr (!kEmit) {
          e = (int32_t)(oy + lower_bound(a.ocol + oy, dy, b));
          *slot = e;
        } else {
          e = *slot;
        }
      }
      ny[i] = y; ne[i] = e; noy[i] = oy; nd[i] = dy;
      if constexpr (!kEmit) {
        if (owned && dy == 0) a.cnt[e] = 0;
        keep[i] = owned && dy > 0;
        if (keep[i] && a.lsamp && dy >= kSkipMin) {
          const int32_t f = skip_below(a.lsamp, oy, dy, lo_b);
          noy[i] = oy + f;
          nd[i] = dy - f;
        }
      } else {
        if (owned) {
          const int64_t lo = a.tri_off[e], hi = a.tri_off[e + 1];
          nbase[i] = lo;
          keep[i] = hi > lo && (kDigest || (hi > a.first && lo < a.first + a.count));
          if (keep[i]) {
            // no hit lies before the first one the count pass found: the
            // write pass probes N+(y) from there on
            const int32_t f = (int32_t)(a.hfirst[e] - oy);
            noy[i] = oy + f;
            nd[i] = dy - f;
          }
        }
      }
    }
    if (keep[i]) packed += (int64_t(1) << 32) + nd[i];
  }
  if constexpr (!kEmit) {
    if (a.item_e) {
      int32_t lo = INT_MAX, hi = -1;
#pragma unroll
      for (int i = 0; i < kPer; ++i)
        if (keep[i]) { lo = min(lo, ne[i]); hi = max(hi, ne[i]); }
      lo = block_min(lo, sh.red);
      hi = block_max(hi, sh.red);
      if (tid == 0) a.item_e[it] = make_int2(lo, hi);
    }
  }
  int64_t total;
  int64_t at = block_exclusive_scan(packed, sh.scan_tmp, &total);
  const int K = (int)(total >> 32);
  const int32_t P = (int32_t)(total & 0xFFFFFFFF);
  if constexpr (!kEmit) {
    if (tid == 0) look_block += P;          // the probes this item makes
  }
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    if (keep[i]) {
      const int slot = (int)(at >> 32);
      sh.nb_src[slot] = (int32_t)(noy[i] - (at & 0xFFFFFFFF));
      sh.nb_pre[slot] = (int32_t)(at & 0xFFFFFFFF);
      if constexpr (!kEmit || kDigest) sh.nb_e[slot] = ne[i];
      if constexpr (!kEmit) sh.nb_acc[slot] = 0;
      if constexpr (!kEmit) sh.nb_first[slot] = INT_MAX;
      if constexpr (kEmit) {
        sh.nb_base[slot] = nbase[i];
        sh.nb_py[slot] = a.perm[ny[i]];
      }
      at += (int64_t(1) << 32) + nd[i];
    }
  }
  if (tid == 0) sh.nb_pre[K] = P;
  __syncthreads();
  if (K == 0) return;           // nothing owned in this window: no index needed
  if constexpr (kEmit) {
    // neighbour-aligned probe ranges of the four waves: wave w starts at the
    // first neighbour whose probes begin at or after w * P / 4
    if (tid <= kWavesPerBlock) {
      const int32_t target = (int32_t)(((int64_t)P * tid) / kWavesPerBlock);
      int lo = 0, hi = K;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (sh.nb_pre[mid] < target) lo = mid + 1; else hi = mid;
      }
      sh.wave_k[tid] = tid == kWavesPerBlock ? K : lo;
    }
  }
  const int32_t* list = a.ocol + ob;
  const int64_t span = (int64_t)list[db - 1] - list[0] + 1;
  const int arm = resolve_arm(a.arms[heavy_class(db)], db, span, a.idx_words);
  const int32_t pb = kEmit ? a.perm[b] : 0;
  int64_t t = 0;
  if constexpr (kArms == (1u << kArmBitmap)) {
    t = run_item<kArmBitmap, kEmit, kDigest>(sh, lds, a, list, db, K, P, pb, dg);
  } else if constexpr (kArms == (1u << kArmSorted)) {
    t = run_item<kArmSorted, kEmit, kDigest>(sh, lds, a, list, db, K, P, pb, dg);
  } else if constexpr (kArms == ((1u << kArmBitmap) | (1u << kArmSorted))) {
    if (arm == kArmBitmap) t = run_item<kArmBitmap, kEmit, kDigest>(sh, lds, a, list, db, K, P, pb, dg);
    else t = run_item<kArmSorted, kEmit, kDigest>(sh, lds, a, list, db, K, P, pb, dg);
  } else {
    static_assert(kArms == kAllArms, "arm subsets: bitmap, sorted, bitmap + sorted, all");
    switch (arm) {
      case kArmBitmap: t = run_item<kArmBitmap, kEmit, kDigest>(sh, lds, a, list, db, K, P, pb, dg); break;
      case kArmHash: t = run_item<kArmHash, kEmit, kDigest>(sh, lds, a, list, db, K, P, pb, dg); break;
      case kArmSorted: t = run_item<kArmSorted, kEmit, kDigest>(sh, lds, a, list, db, K, P, pb, dg); break;
      default: t = run_item<kArmGlobal, kEmit, kDigest>(sh, lds, a, list, db, K, P, pb, dg); break;
    }
  }
  if constexpr (!kEmit) tri_block += t;
  __syncthreads();
  if constexpr (!kEmit) {
    int32_t looks = 0;
    for (int s = tid; s < K; s += kBlock) {
      const int32_t hits = sh.nb_acc[s];
      a.cnt[sh.nb_e[s]] = hits;
      if (hits) {
        a.hfirst[sh.nb_e[s]] = sh.nb_src[s] + sh.nb_first[s];   // ocol index of the hit
        looks += sh.nb_pre[s + 1] - sh.nb_first[s];
      }
    }
    looks = wave_sum(looks);
    if (lane_id() == 0 && looks) atomicAdd(&sh.looks, (unsigned long long)looks);
  }
  __syncthreads();
}

template <bool kEmit, bool kDigest>
__device__ void heavy_finish(HeavyShared<kEmit, kDigest>& sh, const HeavyArgs& a, int64_t tri_block,
                             int64_t look_block, const Digest& dg) {
  if constexpr (!kEmit) {
    const int64_t t = block_sum(tri_block, sh.scan_tmp);
    if (a.tri_stat && threadIdx.x == 0 && t) atomicAdd(u64p(a.tri_stat), (unsigned long long)t);
    if (a.made_stat && threadIdx.x == 0 && look_block)
      atomicAdd(u64p(a.made_stat), (unsigned long long)look_block);
    if (a.look_stat && threadIdx.x == 0 && sh.looks) atomicAdd(u64p(a.look_stat), sh.looks);
  } else {
    if constexpr (kDigest) flush_digest(dg, a.digest);
  }
}

// A launch covers the work items of one heavy class; the LDS index lives in
// dynamic shared memory of a.idx_words words.
template <bool kEmit, bool kDigest = false, unsigned kArms = kAllArms>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kEmit ? 1 : 6)))
void k_heavy(HeavyArgs a) {
  __shared__ HeavyShared<kEmit, kDigest> sh;
  extern __shared__ uint32_t lds[];
  int64_t tri_block = 0, look_block = 0;
  Digest dg;
  if constexpr (!kEmit) {
    if (threadIdx.x == 0) sh.looks = 0;      // read after the last item's barriers
  }
  const int64_t n_items = a.item_list_n ? (int64_t)*a.item_list_n : a.item_count;
  for (int64_t it = blockIdx.x; it < n_items; it += gridDim.x)
    heavy_item<kEmit, kDigest, kArms>(sh, lds, a, a.item_list ? a.item_list[it] : a.item_base + it,
                                      tri_block, look_block, dg);
  heavy_finish<kEmit, kDigest>(sh, a, tri_block, look_block, dg);
}

// Persistent form: one launch drains the work items of every heavy class
// through an atomic cursor, heaviest class first (items are stored in class
// order).  The grid is sized to the resident workgroups, not to the work, so
// the launch needs nothing from the host.
template <bool kEmit>
__global__ __launch_bounds__(kBlock) void k_heavy_drain(HeavyArgs a,
                                                        const int64_t* __restrict__ stats,
                                                        unsigned long long* cursor) {
  __shared__ HeavyShared<kEmit> sh;
  __shared__ int64_t next;
  extern __shared__ uint32_t lds[];
  int64_t total = 0;
  for (int q = 0; q < kHeavyClasses; ++q) total += stats[(kHeavyBase + q) * kStats + kSItems];
  int64_t tri_block = 0, look_block = 0;
  Digest dg;
  if constexpr (!kEmit) {
    if (threadIdx.x == 0) sh.looks = 0;
  }
  while (true) {
    if (threadIdx.x == 0) next = (int64_t)atomicAdd(cursor, 1ull);
    __syncthreads();
    const int64_t t = next;
    __syncthreads();
    if (t >= total) break;
    heavy_item<kEmit, false>(sh, lds, a, total - 1 - t, tri_block, look_block, dg);
  }
  heavy_finish<kEmit, false>(sh, a, tri_block, look_block, dg);
}

// ---------------------------------------------------------------- light path

struct LightArgs {
  const int32_t* elist;
  const int64_t* orow;
  const int32_t* ocol;
  const int32_t* otail;
  int32_t* cnt;                 // count pass
  const int64_t* tri_off;       // write pass
  const int32_t* perm;
  int64_t first, count;
  int32_t* out;
  unsigned long long* digest;   // write pass in digest mode
  uint32_t* esup = nullptr;     // digest mode, optional: per-edge support
  int32_t head = 0;             // fixed orientation (edge_ends)
};

// One triangle of edge {pu, pv} with third vertex pw (original ids) at global
// index at: stored, or digested.
template <bool kDigest>
__device__ __forceinline__ void light_sink(const LightArgs& a, Digest& dg, int64_t at, int32_t pu,
                                           int32_t pv, int32_t pw) {
  int32_t t0 = pu, t1 = pv, t2 = pw;
  sort3(t0, t1, t2);
  if constexpr (kDigest) {
    dg.add(t0, t1, t2);
  } else if (at >= a.first && at < a.first + a.count) {
    int32_t* o = a.out + 3 * (at - a.first);      // streaming stores, as in store()
    __builtin_nontemporal_store(t0, o);
    __builtin_nontemporal_store(t1, o + 1);
    __builtin_nontemporal_store(t2, o + 2);
  }
}

// Binned light edges elist[t0 .. t1), G lanes per edge: each lane binary-
// searches N+(b) for its share of N+(s).
template <int G, bool kEmit, bool kDigest>
__device__ __forceinline__ void light_range(const LightArgs& a, int64_t t0, int64_t t1,
                                            int64_t& tri, Digest& dg) {
  constexpr int kGroups = kBlock / G;
  const int gi = threadIdx.x / G, li = threadIdx.x % G;
  for (int64_t t = t0 + gi; t < t1; t += kGroups) {
    const int32_t e = a.elist[t];
    const int32_t u = a.otail[e], v = a.ocol[e];
    const EdgeEnds x = edge_ends(a.orow, u, v, a.head != 0);
    const int64_t os = a.orow[x.s], ob = a.orow[x.b];
    const int32_t* ps = a.ocol + os;
    const int32_t* pb = a.ocol + ob;
    if constexpr (!kEmit) {
      int32_t hits = 0;
      for (int32_t q = li; q < x.c; q += G) hits += contains_sorted(pb, x.db, ps[q]);
      tri += hits;
      hits = group_sum<G>(hits);
      if (li == 0) a.cnt[e] = hits;
    } else {
      int64_t pos = a.tri_off[e];
      const int64_t end = a.tri_off[e + 1];
      if (pos == end || (!kDigest && (end <= a.first || pos >= a.first + a.count))) continue;
      const int32_t pu = a.perm[u], pv = a.perm[v];
      // digest mode: the edge's own triangles (other triangles add to it too)
      if constexpr (kDigest)
        if (a.esup && li == 0) atomicAdd(&a.esup[e], (uint32_t)(end - pos));
      for (int32_t q0 = 0; q0 < x.c; q0 += G) {
        const int32_t q = q0 + li;
        const int32_t w = q < x.c ? ps[q] : 0;
        const int64_t j = q < x.c ? lower_bound(pb, x.db, w) : x.db;
        const bool hit = j < x.db && pb[j] == w;
        const uint64_t mask = ballot(hit);
        const int64_t at = pos + popc_below_in_group<G>(mask);
        if (hit) {
          light_sink<kDigest>(a, dg, at, pu, pv, a.perm[w]);
          if constexpr (kDigest)
            if (a.esup) {
              atomicAdd(&a.esup[os + q], 1u);
              atomicAdd(&a.esup[ob + j], 1u);
            }
        }
        pos += __popcll(group_bits<G>(mask));
      }
    }
  }
}

// Algorithm 1's merge intersection of N+(u) and N+(v), G lanes per edge.
// Lane li takes a contiguous run of N+(u) and merges it with N+(v) from the
// first entry not below the run's first value, so the lanes together read
// both lists about once (plus one binary search per lane).  Hits come out in
// ascending order, lane after lane, as the other strategies emit them.
template <int G, bool kEmit, bool kDigest>
__device__ __forceinline__ void merge_range(const LightArgs& a, int64_t t0, int64_t t1,
                                            int64_t& tri, Digest& dg) {
  constexpr int kGroups = kBlock / G;
  const int gi = threadIdx.x / G, li = threadIdx.x % G;
  for (int64_t t = t0 + gi; t < t1; t += kGroups) {
    const int32_t e = a.elist[t];
    const int32_t u = a.otail[e], v = a.ocol[e];
    const int64_t ou = a.orow[u], ov = a.orow[v];
    const int32_t du = (int32_t)(a.orow[u + 1] - ou), dv = (int32_t)(a.orow[v + 1] - ov);
    const int32_t* A = a.ocol + ou;
    const int32_t* B = a.ocol + ov;
    int64_t pos = 0, end = 0;
    if constexpr (kEmit) {
      pos = a.tri_off[e];
      end = a.tri_off[e + 1];
      if (pos == end || (!kDigest && (end <= a.first || pos >= a.first + a.count))) continue;
    }
    const int32_t per = (du + G - 1) / G;
    const int32_t i0 = min(du, li * per), i1 = min(du, i0 + per);
    const int32_t j0 = i0 < i1 ? (int32_t)lower_bound(B, dv, A[i0]) : dv;
    int32_t hits = 0;
    for (int32_t i = i0, j = j0; i < i1 && j < dv;) {
      const int32_t x = A[i], y = B[j];
      hits += x == y;
      i += x <= y;
      j += y <= x;
    }
    if constexpr (!kEmit) {
      tri += hits;
      hits = group_sum<G>(hits);
      if (li == 0) a.cnt[e] = hits;
    } else {
      int64_t at = pos + group_exclusive_sum<G>(hits);
      const int32_t pu = a.perm[u], pv = a.perm[v];
      if constexpr (kDigest)
        if (a.esup && li == 0) atomicAdd(&a.esup[e], (uint32_t)(end - pos));
      for (int32_t i = i0, j = j0; i < i1 && j < dv;) {
        const int32_t x = A[i], y = B[j];
        if (x == y) {
          light_sink<kDigest>(a, dg, at++, pu, pv, a.perm[x]);
          if constexpr (kDigest)
            if (a.esup) {
              atomicAdd(&a.esup[ou + i], 1u);
              atomicAdd(&a.esup[ov + j], 1u);
            }
        }
        i += x <= y;
        j += y <= x;
      }
    }
  }
}

template <bool kEmit, bool kDigest>
__device__ void light_finish(const LightArgs& a, int64_t tri, const Digest& dg,
                             int64_t* tri_stat) {
  if constexpr (!kEmit) {
    __shared__ int64_t red[kWavesPerBlock];
    const int64_t s = block_sum(tri, red);
    if (tri_stat && threadIdx.x == 0 && s) atomicAdd(u64p(tri_stat), (unsigned long long)s);
  } else {
    if constexpr (kDigest) flush_digest(dg, a.digest);
  }
}

// A launch covers one light bin, elist[base .. base + total).
template <int G, bool kEmit, bool kDigest = false>
__global__ __launch_bounds__(kBlock) void k_light(LightArgs a, int64_t base, int64_t total,
                                                  int64_t* tri_stat) {
  constexpr int kGroups = kBlock / G;
  int64_t tri = 0;
  Digest dg;
  for (int64_t c = (int64_t)blockIdx.x * kGroups; c < total; c += (int64_t)gridDim.x * kGroups)
    light_range<G, kEmit, kDigest>(a, base + c, base + min(c + kGroups, total), tri, dg);
  light_finish<kEmit, kDigest>(a, tri, dg, tri_stat);
}

// The merge strategy's launch over one bin.
template <int G, bool kEmit, bool kDigest = false>
__global__ __launch_bounds__(kBlock) void k_merge(LightArgs a, int64_t base, int64_t total,
                                                  int64_t* tri_stat) {
  constexpr int kGroups = kBlock / G;
  int64_t tri = 0;
  Digest dg;
  for (int64_t c = (int64_t)blockIdx.x * kGroups; c < total; c += (int64_t)gridDim.x * kGroups)
    merge_range<G, kEmit, kDigest>(a, base + c, base + min(c + kGroups, total), tri, dg);
  light_finish<kEmit, kDigest>(a, tri, dg, tri_stat);
}

// Lanes per edge of every light bin and the group-rounds of one task.
struct LightPlan {
  int32_t tile[kLightBins];
  int32_t rounds;
};

// Persistent form: one launch drains every light bin through an atomic
// cursor.  A task is rounds * (kBlock / G) consecutive edges of one bin; bins
// of larger c (more probes per edge) come first.
template <bool kEmit>
__global__ __launch_bounds__(kBlock) void k_light_drain(LightArgs a, LightPlan p,
                                                        const int64_t* __restrict__ stats,
                                                        unsigned long long* cursor) {
  __shared__ int64_t tpre[kLightBins + 1], ebase[kLightBins], eper[kLightBins], ecnt[kLightBins];
  __shared__ int64_t next;
  if (threadIdx.x == 0) {
    int64_t base = 0;
    for (int k = 0; k < kLightBins; ++k) {
      ecnt[k] = stats[k * kStats + kSEdges];
      ebase[k] = base;
      base += ecnt[k];
      eper[k] = (int64_t)(kBlock / p.tile[k]) * p.rounds;
    }
    int64_t run = 0;
    for (int i = 0; i < kLightBins; ++i) {
      const int k = kLightBins - 1 - i;
      tpre[i] = run;
      run += (ecnt[k] + eper[k] - 1) / eper[k];
    }
    tpre[kLightBins] = run;
  }
  __syncthreads();
  int64_t tri = 0;
  Digest dg;
  while (true) {
    if (threadIdx.x == 0) next = (int64_t)atomicAdd(cursor, 1ull);
    __syncthreads();
    const int64_t t = next;
    __syncthreads();
    if (t >= tpre[kLightBins]) break;
    int i = 0;
    while (tpre[i + 1] <= t) ++i;
    const int k = kLightBins - 1 - i;
    const int64_t lo = (t - tpre[i]) * eper[k];
    const int64_t hi = min(lo + eper[k], ecnt[k]);
    const int64_t t0 = ebase[k] + lo, t1 = ebase[k] + hi;
    switch (p.tile[k]) {
      case 4: light_range<4, kEmit, false>(a, t0, t1, tri, dg); break;
      case 8: light_range<8, kEmit, false>(a, t0, t1, tri, dg); break;
      case 16: light_range<16, kEmit, false>(a, t0, t1, tri, dg); break;
      case 32: light_range<32, kEmit, false>(a, t0, t1, tri, dg); break;
      default: light_range<64, kEmit, false>(a, t0, t1, tri, dg); break;
    }
  }
  light_finish<kEmit, false>(a, tri, dg, nullptr);
}

// The part of the edge order a triangle window [first, first + count)
// touches, and each light bin's run of it: win[0..1] = [e_lo, e_hi), the
// edges whose slots can meet the window; win[2 + 2k .. 3 + 2k] = the elist
// indices of bin k's edges in [e_lo, e_hi) (bins are in edge order).
constexpr int kWinWords = 2 + 2 * kLightBins + 2;   // + tail ranks of e_lo and e_hi - 1

__global__ void k_window(int64_t m, const int64_t* __restrict__ tri_off, int64_t first,
                         int64_t count, const int64_t* __restrict__ stats,
                         const int32_t* __restrict__ elist, const int32_t* __restrict__ otail,
                         int32_t n, int64_t* __restrict__ win) {
  __shared__ int64_t range[2];
  if (threadIdx.x == 0) {
    int64_t lo = 0, hi = m;           // first e with tri_off[e + 1] > first
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (tri_off[mid + 1] > first) hi = mid; else lo = mid + 1;
    }
    range[0] = lo;
    const int64_t end = first + count;
    lo = 0; hi = m;                   // first e with tri_off[e] >= end (m if none)
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (tri_off[mid] >= end) hi = mid; else lo = mid + 1;
    }
    range[1] = lo;
    if (first <= 0 && end >= tri_off[m]) {   // the whole list: whole bins
      range[0] = 0;
      range[1] = m;
    }
    win[0] = range[0];
    win[1] = range[1];
    // the rows the window's edges come from (tails ascend with the edge id)
    const bool any = range[1] > range[0];
    win[kWinWords - 2] = any ? otail[range[0]] : n;
    win[kWinWords - 1] = any ? otail[range[1] - 1] : -1;
  }
  __syncthreads();
  if (threadIdx.x < kLightBins) {
    const int k = threadIdx.x;
    int64_t base = 0;
    for (int q = 0; q < k; ++q) base += stats[q * kStats + kSEdges];
    const int64_t len = stats[k * kStats + kSEdges];
    int64_t at[2];
    for (int z = 0; z < 2; ++z) {
      int64_t lo = 0, hi = len;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (elist[base + mid] < range[z]) lo = mid + 1; else hi = mid;
      }
      at[z] = base + lo;
    }
    win[2 + 2 * k] = at[0];
    win[3 + 2 * k] = at[1];
  }
}

// ---------------------------------------------------------------- host side

// Per-bucket choices: lanes per edge of each light bin, index arm of each
// heavy owner class.
struct Plan {
  int32_t light_tile[kLightBins];
  int32_t heavy_arm[kHeavyClasses];
};

// The plain rule: lanes per edge about the bin's c; heavy owners use the
// bitmap, held to 16 KiB per class (an owner whose window does not fit takes
// the sorted copy, then the global search).
Plan plain_plan() {
  Plan p;
  for (int k = 0; k < kLightBins; ++k)
    p.light_tile[k] = k <= 2 ? 4 : k == 3 ? 8 : k == 4 ? 16 : k == 5 ? 32 : 64;
  for (int h = 0; h < kHeavyClasses; ++h) p.heavy_arm[h] = kArmBitmap;
  return p;
}

bool valid_tile(int t) { return t == 4 || t == 8 || t == 16 || t == 32 || t == 64; }

// Table codes: entry k < kLightBins is tile << 8 (arm byte 0 = binary
// search); entry kHeavyBase + h is heavy class h's arm.
bool plan_from(const DispatchView& d, Plan* p) {
  *p = plain_plan();
  if (!d.table) return true;
  for (int k = 0; k < kLightBins; ++k) {
    const int code = d.table[k];
    const int tile = code >> 8;
    if ((code & 0xff) != 0 || !valid_tile(tile)) return false;
    p->light_tile[k] = tile;
  }
  for (int h = 0; h < kHeavyClasses; ++h) {
    const int arm = d.table[kHeavyBase + h];
    if (arm < 0 || arm >= kNumArms) return false;
    p->heavy_arm[h] = arm;
  }
  return true;
}

// Plan <-> table codes (the codes of aot_dispatch's table).
void plan_to_table(const Plan& p, int32_t* t) {
  for (int b = 0; b < kNumBuckets; ++b) t[b] = 0;
  for (int k = 0; k < kLightBins; ++k) t[k] = p.light_tile[k] << 8;
  for (int h = 0; h < kHeavyClasses; ++h) t[kHeavyBase + h] = p.heavy_arm[h];
}

constexpr int kLightTiles[5] = {4, 8, 16, 32, 64};

// The cost model's input for every bucket, from the per-bucket statistics.
void features_from_stats(const int64_t* hs, float* f, uint8_t* present) {
  for (int b = 0; b < kNumBuckets; ++b) {
    const int64_t* st = hs + b * kStats;
    const bool heavy = b >= kHeavyBase;
    const double e = (double)st[kSEdges];
    float* x = f + b * kFeatures;
    present[b] = st[kSEdges] > 0;
    const double safe = e > 0 ? e : 1.0;
    x[0] = heavy ? 1.f : 0.f;
    x[1] = (float)std::log2(1.0 + e);
    x[2] = (float)std::log2(1.0 + (double)st[kSProbes] / safe);
    x[3] = (float)std::log2(1.0 + (double)st[kSDb] / safe);
    x[4] = heavy ? (float)std::log2(1.0 + (double)st[kSSpan]) : 0.f;
    const double items = (double)st[kSItems];
    x[5] = heavy && items > 0 ? (float)std::log2(1.0 + (double)st[kSStaged] / items) : 0.f;
    x[6] = heavy ? (float)std::log2(1.0 + items) : 0.f;
    x[7] = (float)b / (float)kNumBuckets;
  }
}

// Argmin of the predicted cost per bucket over the bucket's options (light:
// outputs 0..4, heavy: 5..8).  False if any prediction of a present bucket is
// not finite.
bool plan_from_predictions(const float* pred, int stride, const uint8_t* present, Plan* p) {
  *p = plain_plan();
  for (int b = 0; b < kNumBuckets; ++b) {
    if (!present[b]) continue;
    const float* y = pred + b * stride;
    const bool heavy = b >= kHeavyBase;
    const int lo = heavy ? 5 : 0, hi = heavy ? 9 : 5;
    int best = lo;
    for (int o = lo; o < hi; ++o) {
      if (!std::isfinite(y[o])) return false;
      if (y[o] < y[best]) best = o;
    }
    if (heavy) p->heavy_arm[b - kHeavyBase] = best - 5;
    else if (b < kLightBins) p->light_tile[b] = kLightTiles[best];
  }
  return true;
}

// Work items: per heavy owner ceil(deg+/kItemSpan) + ceil(deg-/kItemSpan)
// <= (deg+ + deg-)/kItemSpan + 2, so at most 2n + 2m/kItemSpan in all.
int64_t max_items(int32_t n, int64_t m) { return 2 * (int64_t)n + cdiv(2 * m, kItemSpan) + 16; }

struct CountWs {
  int32_t* plan;
  float* feat;                       // [kNumBuckets][kFeatures], cost-model input
  float* pred;                       // [kNumBuckets][16], cost-model output
  unsigned long long* digest;
  int32_t* cnt;
  uint8_t* code;
  int32_t* elist;
  int2* items;
  int2* item_e;                      // per item: owned edge-id bounds
  int32_t* ieid;                     // [m] per in-list entry: owned in-edge id
  int32_t* hfirst;                   // [m] per heavy-owned edge: ocol index of its first hit
  int32_t* lsamp;                    // [m / kLine + 1] first entry of each line of ocol
  int32_t* witems;                   // [items] the items a write window visits
  int32_t* wcount;                   // [kHeavyClasses] their number per class
  int32_t* hist;                     // [kLightBins][chunks] light edges per chunk
  int64_t* hoff;                     // its exclusive scan
  int64_t* win;                      // window: edge range, then each bin's elist run
  int64_t* stats;
  unsigned long long* probes;
  void* scan_tmp;
};

CountWs carve_count(Carve& c, int32_t n, int64_t m) {
  CountWs w;
  w.plan = c.take<int32_t>(kPlanWords);
  w.feat = c.take<float>(kNumBuckets * kFeatures);
  w.pred = c.take<float>(kNumBuckets * 16);
  w.digest = c.take<unsigned long long>(4);
  w.cnt = c.take<int32_t>(m);
  w.code = c.take<uint8_t>(m);
  w.elist = c.take<int32_t>(m);
  w.items = c.take<int2>(max_items(n, m));
  w.item_e = c.take<int2>(max_items(n, m));
  w.ieid = c.take<int32_t>(m);
  w.hfirst = c.take<int32_t>(m);
  w.lsamp = c.take<int32_t>(cdiv(m, kLine) + 1);
  w.witems = c.take<int32_t>(max_items(n, m));
  w.wcount = c.take<int32_t>(kHeavyClasses);
  const int64_t cells = kLightBins * cdiv(m, kScatterChunk);
  w.hist = c.take<int32_t>(cells);
  w.hoff = c.take<int64_t>(cells + 1);
  w.win = c.take<int64_t>(kWinWords);
  w.stats = c.take<int64_t>(kStatWords);
  w.probes = c.take<unsigned long long>(8);   // [0] probes, [4..7] drain cursors
  w.scan_tmp = c.take<char>((int64_t)scan_workspace(m));
  return w;
}

#define AOT_TRY(x)                          \
  do {                                      \
    hipError_t e_ = (x);                    \
    if (e_ != hipSuccess) {                 \
      *err = hipGetErrorString(e_);         \
      return -5;                            \
    }                                       \
  } while (0)

template <bool kEmit, bool kDigest = false>
hipError_t launch_light(int tile, unsigned grid, const LightArgs& a, int64_t base, int64_t total,
                        int64_t* tri_stat, bool merge, hipStream_t s) {
#define L(G)                                                                     \
  if (merge) k_merge<G, kEmit, kDigest><<<grid, kBlock, 0, s>>>(a, base, total, tri_stat); \
  else k_light<G, kEmit, kDigest><<<grid, kBlock, 0, s>>>(a, base, total, tri_stat)
  switch (tile) {
    case 4: L(4); break;
    case 8: L(8); break;
    case 16: L(16); break;
    case 32: L(32); break;
    default: L(64); break;
  }
#undef L
  return hipGetLastError();
}

// The most LDS a bitmap class reserves when its widest window is larger:
// 16 KiB keeps six workgroups per CU (the probe kernels' register limit, with
// 10 KiB of static LDS).
constexpr int64_t kBitmapCapWords = 4096;

// LDS words a heavy class's launch reserves for its index: enough for the
// requested arm on every owner of the class (bitmap: the class's widest
// span; hash: a power-of-two table of twice deg+; sorted: deg+), capped at
// kMaxIndexWords, beyond which owners fall back to the next arm.  A bitmap
// class whose widest window exceeds kBitmapCapWords reserves that many words,
// or the sorted copy's deg+ if more: owners whose window fits keep the bitmap
// (one LDS read per probe), the others take the sorted copy (log2 deg+ reads),
// and the launch keeps its occupancy instead of holding a wide bitmap's words
// (a 38 KiB bitmap leaves three workgroups per CU) for every owner.
int index_words(int arm, int h, int64_t max_span) {
  const int64_t dmax = int64_t(1) << h;       // class h holds deg+ in (2^(h-1), 2^h]
  int64_t need = 0;
  if (arm == kArmBitmap) {
    need = (max_span + 31) / 32;
    if (need <= kBitmapCapWords) return (int)std::max<int64_t>(need, 1);
    return (int)std::min<int64_t>(std::max<int64_t>(dmax, kBitmapCapWords), kMaxIndexWords);
  }
  if (arm == kArmHash) {
    int64_t t = 2;
    while (t < 2 * dmax) t <<= 1;
    need = std::max(need, t);
  } else if (arm == kArmSorted) {
    need = dmax;
  }
  return (int)std::min<int64_t>(std::max<int64_t>(need, 1), kMaxIndexWords);
}

// The arms the owners of heavy class h can resolve to (resolve_arm) when the
// class requests `arm` with `words` LDS words and its widest list spans
// max_span ids.  Bitmap and sorted fail on independent monotone conditions
// (span, deg+), so the corners of the class's (deg+, span) box give every
// outcome; the hash arm and the open-ended last class take every arm.
unsigned class_arms(int arm, int h, int64_t max_span, int words) {
  if (arm == kArmHash || h >= kHeavyClasses - 1) return kAllArms;
  const int64_t dmin = (int64_t(1) << (h > 0 ? h - 1 : 0)) + (h > 0 ? 1 : 0);
  const int64_t dmax = int64_t(1) << h;
  unsigned m = 0;
  for (const int64_t d : {dmin, dmax})
    for (const int64_t sp : {int64_t(1), std::max<int64_t>(max_span, 1)})
      m |= 1u << resolve_arm(arm, d, sp, words);
  if (m == (1u << kArmBitmap) || m == (1u << kArmSorted) ||
      m == ((1u << kArmBitmap) | (1u << kArmSorted)))
    return m;
  return kAllArms;
}

hipError_t launch_heavy(bool emit, bool digest, unsigned arms, const HeavyArgs& a, unsigned grid,
                        size_t dyn, hipStream_t s) {
  constexpr unsigned B = 1u << kArmBitmap, S = 1u << kArmSorted;
  if (emit && digest) k_heavy<true, true><<<grid, kBlock, dyn, s>>>(a);
  else if (emit && arms == B) k_heavy<true, false, B><<<grid, kBlock, dyn, s>>>(a);
  else if (emit && arms == S) k_heavy<true, false, S><<<grid, kBlock, dyn, s>>>(a);
  else if (emit && arms == (B | S)) k_heavy<true, false, B | S><<<grid, kBlock, dyn, s>>>(a);
  else if (emit) k_heavy<true><<<grid, kBlock, dyn, s>>>(a);
  else if (arms == B) k_heavy<false, false, B><<<grid, kBlock, dyn, s>>>(a);
  else if (arms == S) k_heavy<false, false, S><<<grid, kBlock, dyn, s>>>(a);
  else if (arms == (B | S)) k_heavy<false, false, B | S><<<grid, kBlock, dyn, s>>>(a);
  else k_heavy<false><<<grid, kBlock, dyn, s>>>(a);
  return hipGetLastError();
}

unsigned grid_cap(int64_t work_units) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(kGrid * 4, work_units));
}

hipError_t bin_scatter(int64_t m, const CountWs& w, hipStream_t s) {
  const int64_t nchunks = cdiv(m, kScatterChunk);
  const unsigned g = grid_cap(std::min<int64_t>(nchunks, 4096));
  k_bin_hist<<<g, kBlock, 0, s>>>(m, w.code, nchunks, w.hist);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = exclusive_scan(w.hist, w.hoff, kLightBins * nchunks, w.scan_tmp, s);
  if (e != hipSuccess) return e;
  k_bin_place<<<g, kBlock, 0, s>>>(m, w.code, nchunks, w.hoff, w.elist);
  return hipGetLastError();
}

// The learned plan: features of every bucket -> cost model -> argmin.  A
// model of the wrong shape or with non-finite parameters or predictions
// leaves the plain rule in place (*learned = 0).
int learned_plan(const aot_mlp* net, const int64_t* hs, const CountWs& w, hipStream_t s,
                 Plan* plan, int32_t* learned) {
  *learned = 0;
  if (!net || !net->params || net->n_in != kFeatures || net->n_out != kOptions ||
      net->n_hidden < 1 || net->n_hidden > 64)
    return 0;
  int64_t np = 0;
  if (aot_mlp_param_count(net->n_in, net->n_hidden, net->n_out, &np) != AOT_OK) return 0;
  std::vector<float> params((size_t)np);
  if (hipMemcpyAsync(params.data(), net->params, sizeof(float) * np, hipMemcpyDeviceToHost, s) !=
      hipSuccess)
    return -5;
  float feat[kNumBuckets * kFeatures];
  uint8_t present[kNumBuckets];
  features_from_stats(hs, feat, present);
  if (hipMemcpyAsync(w.feat, feat, sizeof(feat), hipMemcpyHostToDevice, s) != hipSuccess) return -5;
  if (mlp_predict(net, w.feat, kNumBuckets, w.pred, s)) return -5;
  float pred[kNumBuckets * kOptions];
  if (hipMemcpyAsync(pred, w.pred, sizeof(pred), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return -5;
  for (float v : params)
    if (!std::isfinite(v)) return 0;
  Plan p;
  if (!plan_from_predictions(pred, kOptions, present, &p)) return 0;
  *plan = p;
  *learned = 1;
  return 0;
}

// Launches every non-empty bucket of one pass, recording each launch when
// the timing recorder is on.
int run_buckets(bool emit, const Plan& plan, const int64_t* hs, const CountWs& w,
                const int64_t* orow, const int32_t* ocol, const int32_t* otail,
                const int32_t* perm, const int64_t* irow, const int32_t* icol,
                const int64_t* tri_off, int64_t first, int64_t count, int32_t* out,
                unsigned long long* digest, uint32_t* esup,
                const int64_t* win, int strategy, hipStream_t s, const char** err) {
  const bool merge = strategy == kStratMerge;
  int64_t lbase = 0;
  for (int k = 0; k < kLightBins; ++k) {
    const int64_t* st = hs + k * kStats;
    const int64_t all = st[kSEdges];
    // a write window covers one run of the bin (bins are in edge order)
    const int64_t b0 = win ? win[2 + 2 * k] : lbase;
    const int64_t edges = win ? win[3 + 2 * k] - win[2 + 2 * k] : all;
    if (edges > 0) {
      const int tile = plan.light_tile[k];
      const unsigned grid = grid_cap(cdiv(edges, kBlock / tile));
      const int rec = timing_begin(emit ? 1 : 0, k, 0, tile, edges,
                                   edges == all ? st[kSProbes] : -1, 0,
                                   edges == all ? st[kSTriangles] : -1, s);
      LightArgs la;
      la.elist = w.elist; la.orow = orow; la.ocol = ocol; la.otail = otail;
      la.cnt = emit ? nullptr : w.cnt;
      la.tri_off = tri_off; la.perm = perm; la.first = first; la.count = count; la.out = out;
      la.digest = digest; la.esup = esup;
      la.head = strategy == kStratHead;
      const hipError_t e =
          emit ? (digest ? launch_light<true, true>(tile, grid, la, b0, edges, nullptr, merge, s)
                         : launch_light<true>(tile, grid, la, b0, edges, nullptr, merge, s))
               : launch_light<false>(tile, grid, la, b0, edges,
                                     w.stats + k * kStats + kSTriangles, merge, s);
      AOT_TRY(e);
      timing_end(rec, s);
    }
    lbase += all;
  }
  // a write window visits only the items whose triangles it holds
  const bool compact = emit && !digest && win;
  if (compact) AOT_TRY(fill_i32(w.wcount, kHeavyClasses, 0, s));
  for (int h = 0; h < kHeavyClasses; ++h) {
    const int64_t* st = hs + (kHeavyBase + h) * kStats;
    const int64_t items = st[kSItems];
    if (items <= 0) continue;
    HeavyArgs a;
    const int arm = plan.heavy_arm[h];
    for (int q = 0; q < kHeavyClasses; ++q) a.arms[q] = arm;
    a.idx_words = index_words(arm, h, st[kSSpan]);
    a.items = w.items;
    a.item_e = w.item_e;
    a.ieid = w.ieid;
    a.hfirst = w.hfirst;
    a.look_stat = emit ? nullptr : w.stats + (kHeavyBase + h) * kStats + kSLookups;
    a.made_stat = emit ? nullptr : w.stats + (kHeavyBase + h) * kStats + kSCountLooks;
    a.lsamp = emit ? nullptr : w.lsamp;
    a.item_base = st[kSItemBase];
    a.item_count = items;
    a.orow = orow; a.ocol = ocol; a.irow = irow; a.icol = icol;
    a.cnt = w.cnt;
    a.tri_stat = w.stats + (kHeavyBase + h) * kStats + kSTriangles;
    a.tri_off = tri_off;
    a.perm = perm;
    a.first = first;
    a.count = count;
    a.e_lo = win ? win[0] : 0;                         // no window: every edge
    a.e_hi = win ? win[1] : INT64_MAX;
    a.y_lo = win ? (int32_t)win[kWinWords - 2] : 0;
    a.y_hi = win ? (int32_t)win[kWinWords - 1] : INT32_MAX;
    a.out = out;
    a.digest = digest;
    a.esup = esup;
    a.head = strategy == kStratHead;
    // the write pass probes each owned list from its first hit on
    const int rec = timing_begin(emit ? 1 : 0, kHeavyBase + h, arm, kBlock, st[kSEdges],
                                 emit ? st[kSLookups] : st[kSProbes], st[kSStaged],
                                 st[kSTriangles], s);
    if (compact) {
      k_window_items<<<grid_cap(cdiv(items, kBlock)), kBlock, 0, s>>>(
          st[kSItemBase], items, w.item_e, tri_off, first, count, w.witems + st[kSItemBase],
          w.wcount + h);
      AOT_TRY(hipGetLastError());
      a.item_list = w.witems + st[kSItemBase];
      a.item_list_n = w.wcount + h;
    }
    const size_t dyn = sizeof(uint32_t) * (size_t)std::max(a.idx_words, 1);
    AOT_TRY(launch_heavy(emit, digest, class_arms(arm, h, st[kSSpan], a.idx_words), a,
                         grid_cap(items), dyn, s));
    timing_end(rec, s);
  }
  return 0;
}

}  // namespace

size_t count_workspace_bytes(int32_t n, int64_t m) {
  Carve c(nullptr, 0);
  carve_count(c, n, m);
  return c.used;
}

int count_run(int32_t n, int64_t m, const int64_t* orow, const int32_t* ocol, const int32_t* otail,
              const int64_t* irow, const int32_t* icol, const DispatchView& d, int64_t* tri_off, void* ws, size_t ws_bytes,
              uint64_t* result, hipStream_t s, const char** err) {
  Carve c(ws, ws_bytes);
  CountWs w = carve_count(c, n, m);
  if (!c.ok()) {
    *err = "count workspace too small";
    return -4;
  }
  const int strategy = d.strategy;
  // the merge and per-edge strategies keep no per-owner index: every edge is light
  const int32_t heavy_min = strategy == kStratMerge || strategy == kStratPerEdge ? INT32_MAX
                            : d.heavy_min > 0 ? d.heavy_min
                                              : kDefaultHeavyMin;
  const bool head = strategy == kStratHead;
  Plan plan;
  if (!plan_from(d, &plan)) {
    *err = "dispatch table holds an unknown arm or tile code";
    return -6;
  }
  int32_t learned = 0;
  AOT_TRY(fill_i64(w.stats, kStatWords, 0, s));
  AOT_TRY(fill_i64(reinterpret_cast<int64_t*>(w.probes), 8, 0, s));
  std::vector<int64_t> hs(kStatWords, 0);
  if (m > 0) {
    const unsigned ge = grid_cap(std::min<int64_t>(cdiv(m, kBlock), 2048));
    k_bin_count<<<ge, kBlock, 0, s>>>(m, orow, ocol, otail, heavy_min, strategy, w.cnt, w.code,
                                      w.stats, w.probes);
    AOT_TRY(hipGetLastError());
    AOT_TRY(bin_scatter(m, w, s));
    const unsigned gv = grid_cap(std::min<int64_t>(cdiv(n, kBlock), 1024));
    k_item_count<<<gv, kBlock, 0, s>>>(n, orow, ocol, irow, heavy_min, head, w.stats);
    AOT_TRY(hipGetLastError());
    k_item_scatter<<<gv, kBlock, 0, s>>>(n, orow, irow, heavy_min, head, w.stats, w.items);
    AOT_TRY(hipGetLastError());
    k_line_samples<<<grid_cap(cdiv(cdiv(m, kLine), kBlock)), kBlock, 0, s>>>(m, ocol, w.lsamp);
    AOT_TRY(hipGetLastError());
    AOT_TRY(hipMemcpyAsync(hs.data(), w.stats, sizeof(int64_t) * kStatWords,
                           hipMemcpyDeviceToHost, s));
    AOT_TRY(hipStreamSynchronize(s));
    if (d.model) {
      const int rc = learned_plan(d.model, hs.data(), w, s, &plan, &learned);
      if (rc) {
        *err = "cost model evaluation failed";
        return rc;
      }
    }
    const int rc = run_buckets(false, plan, hs.data(), w, orow, ocol, otail, nullptr, irow, icol,
                               nullptr, 0, 0, nullptr, nullptr, nullptr, nullptr, strategy, s,
                               err);
    if (rc) return rc;
  }
  {
    int32_t words[kPlanWords] = {0};
    plan_to_table(plan, words);
    words[kNumBuckets] = learned;
    words[kNumBuckets + 1] = 1;      // plan valid
    words[kNumBuckets + 2] = strategy;
    AOT_TRY(hipMemcpyAsync(w.plan, words, sizeof(words), hipMemcpyHostToDevice, s));
  }
  AOT_TRY(exclusive_scan(w.cnt, tri_off, m, w.scan_tmp, s));
  int64_t t = 0;
  unsigned long long pr = 0;
  AOT_TRY(hipMemcpyAsync(&t, tri_off + m, sizeof(t), hipMemcpyDeviceToHost, s));
  AOT_TRY(hipMemcpyAsync(&pr, w.probes, sizeof(pr), hipMemcpyDeviceToHost, s));
  AOT_TRY(hipMemcpyAsync(hs.data(), w.stats, sizeof(int64_t) * kStatWords, hipMemcpyDeviceToHost,
                         s));
  AOT_TRY(hipStreamSynchronize(s));
  result[0] = (uint64_t)t;
  result[1] = (uint64_t)pr;
  timing_fill_count(hs.data(), kStats, kSTriangles, kSCountLooks, kHeavyBase);
  return 0;
}

namespace {

struct PlanWords {
  int32_t w[kPlanWords];
};

__global__ void k_store_plan(PlanWords p, int32_t* __restrict__ plan) {
  for (int i = threadIdx.x; i < kPlanWords; i += blockDim.x) plan[i] = p.w[i];
}

// Per-graph triangle offsets of a batch: graph g's triangles are global
// indices [gtri[g], gtri[g+1]), its edges [orow[voff[g]], orow[voff[g+1]]).
__global__ void k_batch_totals(int32_t count, const int64_t* __restrict__ voff,
                               const int64_t* __restrict__ orow,
                               const int64_t* __restrict__ tri_off, int64_t* __restrict__ gtri) {
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g <= count;
       g += (int64_t)gridDim.x * blockDim.x)
    gtri[g] = tri_off[orow[voff[g]]];
}

// Resident workgroups of a kernel on the current device: the grid of a
// persistent launch.
template <typename K>
int resident_grid(K kernel, size_t dyn, unsigned* grid) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, kBlock, dyn) != hipSuccess)
    return -5;
  *grid = (unsigned)std::max(1, cus * std::max(per, 1));
  return 0;
}

}  // namespace

// The probe passes with no host synchronisation: binning, the count pass as
// two persistent drains (heavy owner items, then light edges), the scan, and
// the write pass of triangles [first, first + count) the same way.  Launch
// sizes depend only on n, m and the schedule, so the sequence can be
// captured in a HIP graph.  Stores the plan in the workspace like count_run,
// so list_run / digest_run work on it afterwards.
int drain_run(int32_t n, int64_t m, const int64_t* orow, const int32_t* ocol,
              const int32_t* otail, const int32_t* perm, const int64_t* irow,
              const int32_t* icol, const DrainSchedule& sc, int64_t* tri_off, void* ws,
              size_t ws_bytes, int64_t first, int64_t count, int32_t* out, hipStream_t s,
              const char** err) {
  Carve c(ws, ws_bytes);
  CountWs w = carve_count(c, n, m);
  if (!c.ok()) {
    *err = "count workspace too small";
    return -4;
  }
  Plan plan;
  DispatchView dv;
  dv.table = sc.table_given ? sc.table : nullptr;
  if (!plan_from(dv, &plan)) {
    *err = "schedule table holds an unknown arm or tile code";
    return -6;
  }
  const int32_t heavy_min = sc.heavy_min > 0 ? sc.heavy_min : kDefaultHeavyMin;
  LightPlan lp;
  for (int k = 0; k < kLightBins; ++k) lp.tile[k] = plan.light_tile[k];
  lp.rounds = sc.rounds > 0 ? sc.rounds : 4;
  const int64_t span_words = sc.max_span > 0 ? cdiv(sc.max_span, 32) : kMaxIndexWords;
  const int idx_words = (int)std::max<int64_t>(1, std::min<int64_t>(kMaxIndexWords, span_words));
  const size_t dyn = sizeof(uint32_t) * (size_t)idx_words;

  AOT_TRY(fill_i64(w.stats, kStatWords, 0, s));
  AOT_TRY(fill_i64(reinterpret_cast<int64_t*>(w.probes), 8, 0, s));
  {
    PlanWords pw;
    for (int i = 0; i < kPlanWords; ++i) pw.w[i] = 0;
    plan_to_table(plan, pw.w);
    pw.w[kNumBuckets] = 0;          // not learned
    pw.w[kNumBuckets + 1] = 1;      // plan valid
    k_store_plan<<<1, 64, 0, s>>>(pw, w.plan);
    AOT_TRY(hipGetLastError());
  }
  HeavyArgs ha;
  for (int h = 0; h < kHeavyClasses; ++h) ha.arms[h] = plan.heavy_arm[h];
  ha.idx_words = idx_words;
  ha.items = w.items;
  ha.item_e = w.item_e;
  ha.ieid = w.ieid;
  ha.hfirst = w.hfirst;
  ha.look_stat = nullptr;
  ha.lsamp = w.lsamp;
  ha.item_base = 0;
  ha.item_count = 0;
  ha.orow = orow; ha.ocol = ocol; ha.irow = irow; ha.icol = icol;
  ha.cnt = w.cnt;
  ha.tri_stat = nullptr;
  ha.tri_off = tri_off;
  ha.perm = perm;
  ha.first = first;
  ha.count = count;
  ha.e_lo = 0;
  ha.e_hi = INT64_MAX;
  ha.y_lo = 0;
  ha.y_hi = INT32_MAX;
  ha.out = out;
  ha.digest = nullptr;
  LightArgs la;
  la.elist = w.elist; la.orow = orow; la.ocol = ocol; la.otail = otail;
  la.cnt = w.cnt;
  la.tri_off = tri_off; la.perm = perm; la.first = first; la.count = count; la.out = out;
  la.digest = nullptr;
  unsigned gh0, gh1, gl0, gl1;
  if (resident_grid(k_heavy_drain<false>, dyn, &gh0) || resident_grid(k_heavy_drain<true>, dyn, &gh1) ||
      resident_grid(k_light_drain<false>, 0, &gl0) || resident_grid(k_light_drain<true>, 0, &gl1)) {
    *err = "occupancy query failed";
    return -5;
  }
  if (m > 0) {
    const unsigned ge = grid_cap(std::min<int64_t>(cdiv(m, kBlock), 2048));
    k_bin_count<<<ge, kBlock, 0, s>>>(m, orow, ocol, otail, heavy_min, kStratAdaptive, w.cnt,
                                      w.code, w.stats, w.probes);
    AOT_TRY(hipGetLastError());
    AOT_TRY(bin_scatter(m, w, s));
    const unsigned gv = grid_cap(std::min<int64_t>(cdiv(n, kBlock), 1024));
    k_item_count<<<gv, kBlock, 0, s>>>(n, orow, ocol, irow, heavy_min, false, w.stats);
    AOT_TRY(hipGetLastError());
    k_item_scatter<<<gv, kBlock, 0, s>>>(n, orow, irow, heavy_min, false, w.stats, w.items);
    AOT_TRY(hipGetLastError());
    k_line_samples<<<grid_cap(cdiv(cdiv(m, kLine), kBlock)), kBlock, 0, s>>>(m, ocol, w.lsamp);
    AOT_TRY(hipGetLastError());
    k_heavy_drain<false><<<gh0, kBlock, dyn, s>>>(ha, w.stats, w.probes + 4);
    AOT_TRY(hipGetLastError());
    k_light_drain<false><<<gl0, kBlock, 0, s>>>(la, lp, w.stats, w.probes + 5);
    AOT_TRY(hipGetLastError());
  }
  AOT_TRY(exclusive_scan(w.cnt, tri_off, m, w.scan_tmp, s));
  if (m > 0 && count > 0) {
    k_heavy_drain<true><<<gh1, kBlock, dyn, s>>>(ha, w.stats, w.probes + 6);
    AOT_TRY(hipGetLastError());
    k_light_drain<true><<<gl1, kBlock, 0, s>>>(la, lp, w.stats, w.probes + 7);
    AOT_TRY(hipGetLastError());
  }
  return 0;
}

int batch_totals(int32_t count, const int64_t* voff, const int64_t* orow, const int64_t* tri_off,
                 int64_t* gtri, hipStream_t s) {
  k_batch_totals<<<(unsigned)cdiv(count + 1, kBlock), kBlock, 0, s>>>(count, voff, orow, tri_off,
                                                                      gtri);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}

namespace {

// Per-vertex counts from per-edge support: each triangle through v has two
// of its edges at v, so t(v) is half the support summed over v's edges.
// Tail side: one wave per out-list, stored; head side: one atomic per edge.
__global__ __launch_bounds__(kBlock) void k_vertex_tail(int32_t n, const int64_t* __restrict__ orow,
                                                        const uint32_t* __restrict__ sup,
                                                        const int32_t* __restrict__ perm,
                                                        unsigned long long* __restrict__ vcount) {
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  for (int64_t r = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave; r < n; r += nwaves) {
    uint64_t acc = 0;
    for (int64_t e = orow[r] + lane_id(); e < orow[r + 1]; e += kWave) acc += sup[e];
    acc = wave_sum(acc);
    if (lane_id() == 0) vcount[perm[r]] = acc;
  }
}

__global__ __launch_bounds__(kBlock) void k_vertex_head(int64_t m, const int32_t* __restrict__ ocol,
                                                        const uint32_t* __restrict__ sup,
                                                        const int32_t* __restrict__ perm,
                                                        unsigned long long* __restrict__ vcount) {
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * kBlock) {
    const uint32_t c = sup[e];
    if (c) atomicAdd(&vcount[perm[ocol[e]]], (unsigned long long)c);
  }
}

__global__ __launch_bounds__(kBlock) void k_vertex_halve(int32_t n,
                                                         unsigned long long* __restrict__ vcount) {
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * kBlock)
    vcount[v] >>= 1;
}

int emit_run(int32_t n, int64_t m, const int64_t* orow, const int32_t* ocol, const int32_t* otail,
             const int32_t* perm, const int64_t* irow, const int32_t* icol, const DispatchView& d,
             const int64_t* tri_off, void* ws, size_t ws_bytes, int64_t first, int64_t count,
             int32_t* out, bool digest_mode, uint64_t* vcount, uint32_t* esup,
             uint64_t* digest_host, hipStream_t s, const char** err) {
  Carve c(ws, ws_bytes);
  CountWs w = carve_count(c, n, m);
  if (!c.ok()) {
    *err = "count workspace too small";
    return -4;
  }
  Plan plan;
  if (!plan_from(d, &plan)) {
    *err = "dispatch table holds an unknown arm or tile code";
    return -6;
  }
  // the plan the count resolved, unless a table is given: the plain rule's
  // heavy arms depend on the count's statistics, the learned plan on its model
  const bool stored = !d.given || !d.table;
  unsigned long long* dg = digest_mode ? w.digest : nullptr;
  unsigned long long* vc = reinterpret_cast<unsigned long long*>(vcount);
  // vertex counts come from edge support: the caller's array, or the count
  // pass's per-edge counts (no longer needed once tri_off is scanned)
  uint32_t* sup = esup ? esup : vc ? reinterpret_cast<uint32_t*>(w.cnt) : nullptr;
  if (digest_mode) {
    AOT_TRY(fill_i64(reinterpret_cast<int64_t*>(w.digest), 4, 0, s));
    if (sup) AOT_TRY(fill_i32(reinterpret_cast<int32_t*>(sup), m, 0, s));
  }
  if (m > 0 && (digest_mode || count > 0)) {
    std::vector<int64_t> hs(kStatWords, 0);
    int32_t words[kPlanWords];
    int64_t win[kWinWords];
    if (!digest_mode) {
      k_window<<<1, 64, 0, s>>>(m, tri_off, first, count, w.stats, w.elist, otail, n, w.win);
      AOT_TRY(hipGetLastError());
      AOT_TRY(hipMemcpyAsync(win, w.win, sizeof(win), hipMemcpyDeviceToHost, s));
    }
    AOT_TRY(hipMemcpyAsync(hs.data(), w.stats, sizeof(int64_t) * kStatWords,
                           hipMemcpyDeviceToHost, s));
    AOT_TRY(hipMemcpyAsync(words, w.plan, sizeof(words), hipMemcpyDeviceToHost, s));
    AOT_TRY(hipStreamSynchronize(s));
    if (stored && words[kNumBuckets + 1] == 1) {
      DispatchView t;
      t.table = words;
      if (!plan_from(t, &plan)) plan = plain_plan();
    }
    // the bins and work items are the count's, so is the strategy
    const int32_t strategy = words[kNumBuckets + 1] == 1 ? words[kNumBuckets + 2] : 0;
    if (strategy < 0 || strategy >= kNumStrategies) {
      *err = "the workspace holds no valid count";
      return -4;
    }
    const int rc = run_buckets(true, plan, hs.data(), w, orow, ocol, otail, perm, irow, icol,
                               tri_off, first, count, out, dg, sup,
                               digest_mode ? nullptr : win, strategy, s, err);
    if (rc) return rc;
  }
  if (digest_mode && vc && n > 0) {
    k_vertex_tail<<<grid_cap(cdiv(n, kWavesPerBlock)), kBlock, 0, s>>>(n, orow, sup, perm, vc);
    AOT_TRY(hipGetLastError());
    if (m > 0) {
      k_vertex_head<<<grid_cap(cdiv(m, kBlock)), kBlock, 0, s>>>(m, ocol, sup, perm, vc);
      AOT_TRY(hipGetLastError());
    }
    k_vertex_halve<<<grid_cap(cdiv(n, kBlock)), kBlock, 0, s>>>(n, vc);
    AOT_TRY(hipGetLastError());
  }
  if (digest_mode) {
    unsigned long long h[4];
    AOT_TRY(hipMemcpyAsync(h, w.digest, sizeof(h), hipMemcpyDeviceToHost, s));
    AOT_TRY(hipStreamSynchronize(s));
    if (digest_host) {
      digest_host[0] = h[0];
      digest_host[1] = h[1];
      digest_host[2] = h[2];
    }
  }
  return 0;
}

}  // namespace

int list_run(int32_t n, int64_t m, const int64_t* orow, const int32_t* ocol, const int32_t* otail,
             const int32_t* perm, const int64_t* irow, const int32_t* icol, const DispatchView& d,
             const int64_t* tri_off, void* ws, size_t ws_bytes, int64_t first, int64_t count,
             int32_t* out, hipStream_t s, const char** err) {
  return emit_run(n, m, orow, ocol, otail, perm, irow, icol, d, tri_off, ws, ws_bytes, first,
                  count, out, false, nullptr, nullptr, nullptr, s, err);
}

int digest_run(int32_t n, int64_t m, const int64_t* orow, const int32_t* ocol,
               const int32_t* otail, const int32_t* perm, const int64_t* irow,
               const int32_t* icol, const DispatchView& d, const int64_t* tri_off, void* ws,
               size_t ws_bytes, uint64_t* vcount, uint64_t* digest, hipStream_t s,
               const char** err) {
  return emit_run(n, m, orow, ocol, otail, perm, irow, icol, d, tri_off, ws, ws_bytes, 0, 0,
                  nullptr, true, vcount, nullptr, digest, s, err);
}

int support_run(int32_t n, int64_t m, const int64_t* orow, const int32_t* ocol,
                const int32_t* otail, const int32_t* perm, const int64_t* irow,
                const int32_t* icol, const DispatchView& d, const int64_t* tri_off, void* ws,
                size_t ws_bytes, uint32_t* esup, uint64_t* vcount, uint64_t* digest,
                hipStream_t s, const char** err) {
  return emit_run(n, m, orow, ocol, otail, perm, irow, icol, d, tri_off, ws, ws_bytes, 0, 0,
                  nullptr, true, vcount, esup, digest, s, err);
}

int count_plan(const void* ws, size_t ws_bytes, int32_t n, int64_t m, int32_t* table,
               int32_t* learned) {
  Carve c(const_cast<void*>(ws), ws_bytes);
  CountWs w = carve_count(c, n, m);
  int32_t words[kPlanWords];
  if (hipMemcpy(words, w.plan, sizeof(words), hipMemcpyDeviceToHost) != hipSuccess) return -5;
  if (words[kNumBuckets + 1] != 1) plan_to_table(plain_plan(), words);
  for (int b = 0; b < kNumBuckets; ++b) table[b] = words[b];
  *learned = words[kNumBuckets + 1] == 1 ? words[kNumBuckets] : 0;
  return 0;
}

int count_features(const void* ws, size_t ws_bytes, int32_t n, int64_t m, float* features,
                   uint8_t* present) {
  Carve c(const_cast<void*>(ws), ws_bytes);
  CountWs w = carve_count(c, n, m);
  std::vector<int64_t> hs(kStatWords, 0);
  if (hipMemcpy(hs.data(), w.stats, sizeof(int64_t) * kStatWords, hipMemcpyDeviceToHost) !=
      hipSuccess)
    return -5;
  features_from_stats(hs.data(), features, present);
  return 0;
}

}  // namespace aot
