// Orientation (Section 2.2, "Orientation technique"; first step of Algorithm
// 3): rank vertices by (degree, id) ascending, keep <u,v> iff rank(u) <
// rank(v), relabel to rank space and sort every out-list ascending; the
// in-lists Algorithm 3's second loop walks are the rest of each row.
//
// After the radix sort, rank order is degree order, so consecutive ranks have
// similar row lengths: rows are processed in rank ranges with a row-group
// width G matched to the degree range (4, 16 or 64 lanes, or a whole
// workgroup for rows longer than 64).  Out-list lengths are not monotone in
// rank, so the sort step first bins rows by length.  On request, in-lists are
// sorted the same way into ascending rank, which is the order of their edges'
// ids (this makes windows of a huge triangle list cheap; see aot_list).
//
// Labels by id (AOT-randomOrder of Section 4.2): the order still directs every
// edge, but vertices keep their original ids as labels, so an out-list is in
// ascending id instead of the degree local order of Section 3.2; with
// randomly permuted ids that is a random local order.  Rows are then written
// at their id, and perm/rank are the identity.
#include <algorithm>
#include <climits>

#include "kernels.hpp"

namespace aot {

namespace {

// counters[] layout (int32, device)
enum : int {
  kCMaxDeg = 0,
  kCDeg0 = 1,   // #vertices with degree 0
  kCDeg4 = 2,   // #vertices with degree <= 4
  kCDeg16 = 3,  // <= 16
  kCDeg512 = 4, // <= 512 (one wave per row up to here)
  kCError = 5,
  kCSortCount = 8,    // [8..12] rows per sort class
  kCSortCursor = 13,  // [13..17]
  kCRowCount = 18,    // [18..22] rows per degree class (row-list mode; 4 used)
  kCRowCursor = 23,   // [23..27]
  kCInCount = 28,     // [28..32] in-lists per sort class
  kCInCursor = 33,    // [33..37]
  // core order, two slots each (sub-round parity): the least current degree
  // left before the sub-round (INT32_MAX: none), its level, the vertices it
  // removes; then the vertices not yet removed and the sub-rounds so far
  kCCoreMin = 38,     // [38..39]
  kCCoreLevel = 40,   // [40..41]
  kCCoreFront = 42,   // [42..43]
  kCCoreLeft = 44,
  kCCoreRound = 45,
  kCCoreList = 46,    // entries appended by the compaction
  kCCoreBig = 47,     // [47..48] removed vertices with rows longer than kBigRow
  kCounters = 49,
};

constexpr int kSortClasses = 5;     // len <= 16, <= 64, <= 256, <= 4096, longer
constexpr int kBitmapWords = 8192;  // 32 KiB window for the long-list sort
constexpr int kGrid = 4096;         // grid of the grid-stride kernels
constexpr int kRowUnroll = 4;       // chunks of kBlock entries per step on a workgroup's row
constexpr int64_t kBigRow = 1024;   // core peel: rows updated by more than one wave,
constexpr int32_t kBigShared = 8;   // by the whole grid when a sub-round has this few

enum : int {
  kErrRowptr = 1, kErrRange = 2, kErrLoop = 4, kErrOrder = 8, kErrAsym = 16,
};

__global__ __launch_bounds__(kBlock) void k_validate_rowptr(int32_t n, int64_t nnz,
                                                            const int64_t* __restrict__ rowptr,
                                                            int32_t* __restrict__ counters) {
  int bad = 0;
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v <= n;
       v += (int64_t)gridDim.x * kBlock) {
    const int64_t a = rowptr[v];
    if (v == 0 && a != 0) bad = 1;
    if (v == n && a != nnz) bad = 1;
    if (v < n && (rowptr[v + 1] < a)) bad = 1;
    if (a < 0 || a > nnz) bad = 1;
  }
  if (bad) atomicOr(&counters[kCError], kErrRowptr);
}

// One wave per row (grid-stride over rows).
__global__ __launch_bounds__(kBlock) void k_validate_rows(int32_t n,
                                                          const int64_t* __restrict__ rowptr,
                                                          const int32_t* __restrict__ col,
                                                          int32_t* __restrict__ counters) {
  int bad = 0;
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  for (int64_t u = wave; u < n; u += nwaves) {
    const int64_t beg = rowptr[u], end = rowptr[u + 1];
    for (int64_t k = beg + lane_id(); k < end; k += kWave) {
      const int32_t v = col[k];
      if (v < 0 || v >= n) { bad |= kErrRange; continue; }
      if (v == u) bad |= kErrLoop;
      if (k > beg && col[k - 1] >= v) bad |= kErrOrder;
      const int64_t vb = rowptr[v], ve = rowptr[v + 1];
      if (!contains_sorted(col + vb, ve - vb, (int32_t)u)) bad |= kErrAsym;
    }
  }
  if (bad) atomicOr(&counters[kCError], bad);
}

// deg(v), the (key, value) pairs for the rank sort, and the degree-class sizes.
__global__ __launch_bounds__(kBlock) void k_degree(int32_t n, const int64_t* __restrict__ rowptr,
                                                   int32_t* __restrict__ keys,
                                                   int32_t* __restrict__ vals,
                                                   int32_t* __restrict__ counters) {
  __shared__ int32_t red[kWavesPerBlock];
  int32_t mx = 0, c0 = 0, c4 = 0, c16 = 0, c512 = 0;
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * kBlock) {
    const int32_t d = (int32_t)(rowptr[v + 1] - rowptr[v]);
    keys[v] = d;
    vals[v] = (int32_t)v;
    mx = d > mx ? d : mx;
    c0 += d == 0;
    c4 += d <= 4;
    c16 += d <= 16;
    c512 += d <= 512;
  }
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const int32_t y = __shfl_xor(mx, o, kWave);
    mx = y > mx ? y : mx;
  }
  if (lane_id() == 0) red[threadIdx.x / kWave] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t b = 0;
    for (int q = 0; q < kWavesPerBlock; ++q) b = red[q] > b ? red[q] : b;
    atomicMax(&counters[kCMaxDeg], b);
  }
  __syncthreads();
  c0 = block_sum(c0, red);
  c4 = block_sum(c4, red);
  c16 = block_sum(c16, red);
  c512 = block_sum(c512, red);
  if (threadIdx.x == 0) {
    atomicAdd(&counters[kCDeg0], c0);
    atomicAdd(&counters[kCDeg4], c4);
    atomicAdd(&counters[kCDeg16], c16);
    atomicAdd(&counters[kCDeg512], c512);
  }
}

// ---------------------------------------------------------------- core order
// kClist orients by the core (degeneracy) order (Section 2.3); here it is
// taken as synchronous peeling.  Sub-round r raises the level to the least
// current degree left if that is larger, removes every remaining vertex whose
// current degree is at most the level (round[v] = r) and takes one off the
// current degree of each remaining neighbour per removed neighbour.  Sorting
// by (round, id) then gives every vertex at most `level` out-neighbours.
//
// A sub-round is two launches.  The least degree the next sub-round starts
// from is gathered on the way: k_core_mark takes the minimum over the vertices
// it leaves, k_core_update over the decremented degrees atomicSub returns.
// Counters alternate between two slots by sub-round parity, so no launch
// resets a slot another launch of the same sub-round uses.  Sub-rounds after
// the last vertex do nothing, so the host checks progress every few.

// Lowers *slot to the least x over the workgroup: one atomic per workgroup,
// and none when the slot already holds no more (most workgroups see the same
// least degree, and same-address atomics serialise).
__device__ __forceinline__ void block_min_into(int32_t x, int32_t* slot) {
  __shared__ int32_t red[kWavesPerBlock];
  for (int o = kWave / 2; o > 0; o >>= 1) x = min(x, __shfl_xor(x, o, kWave));
  if (lane_id() == 0) red[threadIdx.x / kWave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < kWavesPerBlock; ++q) x = min(x, red[q]);
    if (x != INT32_MAX && x < __atomic_load_n(slot, __ATOMIC_RELAXED)) atomicMin(slot, x);
  }
}

__global__ __launch_bounds__(kBlock) void k_core_init(int32_t n, const int64_t* __restrict__ rowptr,
                                                      int32_t* __restrict__ cur,
                                                      int32_t* __restrict__ round,
                                                      int32_t* __restrict__ vals,
                                                      int32_t* __restrict__ counters) {
  if (blockIdx.x == 0 && threadIdx.x == 0) counters[kCCoreLeft] = n;
  int32_t lo = INT32_MAX;
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * kBlock) {
    const int32_t d = (int32_t)(rowptr[v + 1] - rowptr[v]);
    cur[v] = d;
    round[v] = -1;
    vals[v] = (int32_t)v;
    lo = min(lo, d);
  }
  block_min_into(lo, &counters[kCCoreMin]);
}

// Scans the remaining vertices: list[0 .. len), or every vertex 0 .. len
// when list is null.
// Removed vertices go to front[0 ..) when their rows are short, and to
// front[n - 1], front[n - 2], ... when longer than kBigRow (the two never
// meet: together they hold at most the n vertices).
__global__ __launch_bounds__(kBlock) void k_core_mark(int32_t n, int32_t len,
                                                      const int32_t* __restrict__ list,
                                                      const int64_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ cur,
                                                      int32_t* __restrict__ round,
                                                      int32_t* __restrict__ front,
                                                      int32_t* __restrict__ counters, int32_t r) {
  const int p = r & 1;
  const int32_t lo = counters[kCCoreMin + p];
  const int32_t prev = counters[kCCoreLevel + (p ^ 1)];
  const int32_t level = lo == INT32_MAX ? prev : max(prev, lo);
  if (blockIdx.x == 0 && threadIdx.x == 0) counters[kCCoreLevel + p] = level;
  if (lo == INT32_MAX) return;                      // nothing left
  int32_t next = INT32_MAX;                         // least degree among those left
  for (int64_t b0 = (int64_t)blockIdx.x * kBlock; b0 < len; b0 += (int64_t)gridDim.x * kBlock) {
    const int64_t i = b0 + threadIdx.x;
    const int64_t v = i < len ? (list ? list[i] : i) : 0;
    const bool alive = i < len && round[v] < 0;
    const int32_t d = alive ? cur[v] : 0;
    const bool take = alive && d <= level;
    if (alive && !take) next = min(next, d);
    if (!ballot(take)) continue;
    const bool big = take && rowptr[v + 1] - rowptr[v] > kBigRow;
    const uint64_t ms = ballot(take && !big), mb = ballot(big);
    int32_t as = 0, ab = 0;
    if (lane_id() == 0) {
      if (ms) as = atomicAdd(&counters[kCCoreFront + p], (int32_t)__popcll(ms));
      if (mb) ab = atomicAdd(&counters[kCCoreBig + p], (int32_t)__popcll(mb));
    }
    as = __shfl(as, 0, kWave);
    ab = __shfl(ab, 0, kWave);
    if (take) {
      round[v] = r;
      if (big) front[n - 1 - (ab + popc_below(mb))] = (int32_t)v;
      else front[as + popc_below(ms)] = (int32_t)v;
    }
  }
  block_min_into(next, &counters[kCCoreMin + (p ^ 1)]);
}

// The remaining vertices of list[0 .. len) (every vertex when list is null)
// appended to out, in no particular order (the peel does not depend on it).
__global__ __launch_bounds__(kBlock) void k_core_compact(int32_t len,
                                                         const int32_t* __restrict__ list,
                                                         const int32_t* __restrict__ round,
                                                         int32_t* __restrict__ out,
                                                         int32_t* __restrict__ counters) {
  for (int64_t b0 = (int64_t)blockIdx.x * kBlock; b0 < len; b0 += (int64_t)gridDim.x * kBlock) {
    const int64_t i = b0 + threadIdx.x;
    const int32_t v = i < len ? (list ? list[i] : (int32_t)i) : 0;
    const bool keep = i < len && round[v] < 0;
    const uint64_t mask = ballot(keep);
    if (!mask) continue;
    const int leader = __ffsll((long long)mask) - 1;
    int32_t at = 0;
    if (lane_id() == leader) at = atomicAdd(&counters[kCCoreList], (int32_t)__popcll(mask));
    at = __shfl(at, leader, kWave);
    if (keep) out[at + popc_below(mask)] = v;
  }
}

// One wave per removed vertex.
// One wave per removed vertex with a short row; long rows get a workgroup
// each, or the whole grid each when there are only a few (a hub removed late
// would otherwise hold one wave for its whole row).
__global__ __launch_bounds__(kBlock) void k_core_update(int32_t n,
                                                        const int64_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ col,
                                                        const int32_t* __restrict__ front,
                                                        const int32_t* __restrict__ round,
                                                        int32_t* __restrict__ cur,
                                                        int32_t* __restrict__ counters,
                                                        int32_t r) {
  const int p = r & 1;
  const int32_t k = counters[kCCoreFront + p];
  const int32_t kb = counters[kCCoreBig + p];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    counters[kCCoreMin + p] = INT32_MAX;      // read by this sub-round's mark only
    counters[kCCoreFront + (p ^ 1)] = 0;      // the next sub-round's frontiers
    counters[kCCoreBig + (p ^ 1)] = 0;
    counters[kCCoreLeft] -= k + kb;
    if (k + kb > 0) counters[kCCoreRound] = r + 1;
  }
  int32_t next = INT32_MAX;
  const int64_t nwaves = (int64_t)gridDim.x * kWavesPerBlock;
  for (int64_t i = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave; i < k; i += nwaves) {
    const int32_t v = front[i];
    for (int64_t e = rowptr[v] + lane_id(); e < rowptr[v + 1]; e += kWave) {
      const int32_t x = col[e];
      if (round[x] < 0) next = min(next, atomicSub(&cur[x], 1) - 1);
    }
  }
  if (kb <= kBigShared) {
    // a few long rows (hubs, late in the peel): the whole grid on each
    const int64_t nthreads = (int64_t)gridDim.x * kBlock;
    for (int32_t j = 0; j < kb; ++j) {
      const int32_t v = front[n - 1 - j];
      for (int64_t e = rowptr[v] + (int64_t)blockIdx.x * kBlock + threadIdx.x; e < rowptr[v + 1];
           e += nthreads) {
        const int32_t x = col[e];
        if (round[x] < 0) next = min(next, atomicSub(&cur[x], 1) - 1);
      }
    }
  } else {
    // many: one workgroup per row
    for (int32_t j = blockIdx.x; j < kb; j += gridDim.x) {
      const int32_t v = front[n - 1 - j];
      for (int64_t e = rowptr[v] + threadIdx.x; e < rowptr[v + 1]; e += kBlock) {
        const int32_t x = col[e];
        if (round[x] < 0) next = min(next, atomicSub(&cur[x], 1) - 1);
      }
    }
  }
  block_min_into(next, &counters[kCCoreMin + (p ^ 1)]);
}

__global__ __launch_bounds__(kBlock) void k_perm_rank(int32_t n, const int32_t* __restrict__ sorted_ids,
                                                      int32_t* __restrict__ perm,
                                                      int32_t* __restrict__ rank) {
  for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * kBlock) {
    const int32_t v = sorted_ids[r];
    perm[r] = v;
    rank[v] = (int32_t)r;
  }
}

// perm and rank when labels stay original ids: both the identity.
__global__ __launch_bounds__(kBlock) void k_identity(int32_t n, int32_t* __restrict__ perm,
                                                     int32_t* __restrict__ rank) {
  for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * kBlock) {
    perm[r] = (int32_t)r;
    rank[r] = (int32_t)r;
  }
}

// Sort keys of a batch of graphs held as one block-diagonal CSR: vertex v of
// graph g (voff[g] <= v < voff[g+1]) gets key (g << dbits) | deg(v), so the
// stable sort ranks graph by graph and, inside a graph, by (degree, id).
__global__ __launch_bounds__(kBlock) void k_batch_keys(int32_t n, const int64_t* __restrict__ voff,
                                                       int32_t count, int dbits,
                                                       const int64_t* __restrict__ rowptr,
                                                       int32_t* __restrict__ keys,
                                                       int32_t* __restrict__ vals) {
  for (int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * kBlock) {
    int lo = 0, hi = count;               // last g with voff[g] <= v
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (voff[mid] <= v) lo = mid; else hi = mid;
    }
    keys[v] = (int32_t)(((int64_t)lo << dbits) | (rowptr[v + 1] - rowptr[v]));
    vals[v] = (int32_t)v;
  }
}

// The rows a launch covers: ranks [r0, r1), or (row-list mode, rows !=
// nullptr) the entries of degree class `cls` in `rows`, whose size the
// device counters hold.
struct RowSet {
  int32_t r0, r1;
  const int32_t* rows;
  const int32_t* counters;
  int cls;
  __device__ __forceinline__ void bounds(int64_t* total, int64_t* base) const {
    if (!rows) {
      *total = r1 - r0;
      *base = r0;
      return;
    }
    int64_t b = 0;
    for (int q = 0; q < cls; ++q) b += counters[kCRowCount + q];
    *total = counters[kCRowCount + cls];
    *base = b;
  }
  __device__ __forceinline__ int64_t at(int64_t base, int64_t t) const {
    return rows ? (int64_t)rows[base + t] : base + t;
  }
};

// deg+(r) and deg-(r) for the rows of a RowSet; G lanes per row (G = kBlock:
// one row per workgroup).
template <int G>
__global__ __launch_bounds__(kBlock) void k_orient_count(RowSet rs,
                                                         const int64_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ col,
                                                         const int32_t* __restrict__ perm,
                                                         const int32_t* __restrict__ rank,
                                                         bool by_id,
                                                         int32_t* __restrict__ dplus,
                                                         int32_t* __restrict__ dminus,
                                                         int32_t* __restrict__ rcol) {
  constexpr int kGroups = kBlock / G;
  __shared__ int32_t red[kWavesPerBlock];
  const int gi = threadIdx.x / G, li = threadIdx.x % G;
  int64_t total, base;
  rs.bounds(&total, &base);
  for (int64_t tb = (int64_t)blockIdx.x * kGroups; tb < total;
       tb += (int64_t)gridDim.x * kGroups) {
    const bool live = tb + gi < total;
    const int64_t r = live ? rs.at(base, tb + gi) : 0;
    int32_t cnt = 0;
    int64_t deg = 0, o = 0;
    if (live) {
      const int32_t u = perm[r];
      o = by_id ? (int64_t)u : r;        // the row's label
      const int64_t beg = rowptr[u];
      deg = rowptr[u + 1] - beg;
      if constexpr (G == kBlock) {
        // a workgroup per (long) row: kRowUnroll chunks per step, so their
        // loads and rank gathers are in flight together (a hub row of tens
        // of thousands of entries otherwise waits out one gather per chunk)
        for (int64_t j0 = li; j0 < deg; j0 += (int64_t)G * kRowUnroll) {
          bool ok[kRowUnroll];
          int32_t c[kRowUnroll];
#pragma unroll
          for (int q = 0; q < kRowUnroll; ++q) {
            const int64_t j = j0 + q * G;
            ok[q] = j < deg;
            c[q] = col[beg + (ok[q] ? j : 0)];
          }
#pragma unroll
          for (int q = 0; q < kRowUnroll; ++q) {
            const int32_t x = rank[c[q]];
            cnt += ok[q] & (x > r);
            if (ok[q]) rcol[beg + j0 + q * G] = x;     // the write pass reads it back
          }
        }
      } else {
        for (int64_t j = li; j < deg; j += G) {
          const int32_t x = rank[col[beg + j]];
          cnt += x > r;
          rcol[beg + j] = x;
        }
      }
    }
    if constexpr (G <= kWave) {
      cnt = group_sum<G>(cnt);
      if (li == 0 && live) {
        dplus[o] = cnt;
        dminus[o] = (int32_t)(deg - cnt);
      }
    } else {
      cnt = block_sum(cnt, red);
      if (threadIdx.x == 0) {
        dplus[o] = cnt;
        dminus[o] = (int32_t)(deg - cnt);
      }
    }
  }
}

// Splits every row into its out-part (unsorted, original order) and in-part
// (original order), and records each out-edge's tail.  r is the row's rank,
// o its label: the rank itself, or with labels by id the original id, in
// which case entries are written as original ids too.
// Rows of one workgroup (G == kBlock): kRowUnroll chunks of kBlock entries
// per step, ranked with one pair of barriers per step.
template <int G>
__device__ __forceinline__ void orient_write_long(int64_t r, int64_t o, bool by_id, int64_t beg,
                                                  int64_t deg, int64_t op, int64_t ip,
                                                  const int32_t* __restrict__ col,
                                                  const int32_t* __restrict__ rcol,
                                                  int32_t* __restrict__ unsorted,
                                                  int32_t* __restrict__ otail,
                                                  int32_t* __restrict__ icol) {
  __shared__ int32_t so[kRowUnroll][kWavesPerBlock], si[kRowUnroll][kWavesPerBlock];
  const int w = threadIdx.x / kWave;
  for (int64_t j0 = 0; j0 < deg; j0 += (int64_t)kBlock * kRowUnroll) {
    int32_t rv[kRowUnroll], xs[kRowUnroll];
    bool out[kRowUnroll], in[kRowUnroll];
    uint64_t bo[kRowUnroll], bi[kRowUnroll];
#pragma unroll
    for (int q = 0; q < kRowUnroll; ++q) {
      const int64_t j = j0 + q * kBlock + threadIdx.x;
      out[q] = j < deg;                   // valid, for now
      const int64_t at = beg + (out[q] ? j : 0);
      xs[q] = rcol[at];                   // the ranks the count pass gathered
      rv[q] = by_id ? col[at] : xs[q];
    }
#pragma unroll
    for (int q = 0; q < kRowUnroll; ++q) {
      const bool valid = out[q];
      const int32_t x = xs[q];
      out[q] = valid && x > r;
      in[q] = valid && x < r;
      bo[q] = ballot(out[q]);
      bi[q] = ballot(in[q]);
      if (lane_id() == 0) { so[q][w] = (int32_t)__popcll(bo[q]); si[q][w] = (int32_t)__popcll(bi[q]); }
    }
    __syncthreads();
    // chunk q of this step starts after chunks 0..q-1; inside a chunk, wave
    // w after waves 0..w-1
    int32_t ao = 0, ai = 0;
#pragma unroll
    for (int q = 0; q < kRowUnroll; ++q) {
      int32_t wo = 0, wi = 0, to = 0, ti = 0;
      for (int x = 0; x < kWavesPerBlock; ++x) {
        if (x < w) { wo += so[q][x]; wi += si[q][x]; }
        to += so[q][x]; ti += si[q][x];
      }
      if (out[q]) {
        const int64_t at = op + ao + wo + popc_below(bo[q]);
        unsorted[at] = rv[q];
        otail[at] = (int32_t)o;
      }
      if (in[q]) icol[ip + ai + wi + popc_below(bi[q])] = rv[q];
      ao += to;
      ai += ti;
    }
    op += ao;
    ip += ai;
    __syncthreads();
  }
}

template <int G>
__global__ __launch_bounds__(kBlock) void k_orient_write(
    RowSet rs, const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const int32_t* __restrict__ perm, const int32_t* __restrict__ rank, bool by_id,
    const int64_t* __restrict__ orow, const int64_t* __restrict__ irow,
    int32_t* __restrict__ unsorted, int32_t* __restrict__ otail, int32_t* __restrict__ icol,
    const int32_t* __restrict__ rcol) {
  constexpr int kGroups = kBlock / G;
  __shared__ int32_t so[kWavesPerBlock], si[kWavesPerBlock];
  const int gi = threadIdx.x / G, li = threadIdx.x % G;
  const int w = threadIdx.x / kWave;
  int64_t total, base;
  rs.bounds(&total, &base);
  for (int64_t tb = (int64_t)blockIdx.x * kGroups; tb < total;
       tb += (int64_t)gridDim.x * kGroups) {
    const bool live = tb + gi < total;
    const int64_t r = live ? rs.at(base, tb + gi) : 0;
    int64_t beg = 0, deg = 0, op = 0, ip = 0, o = 0;
    if (live) {
      const int32_t u = perm[r];
      o = by_id ? (int64_t)u : r;
      beg = rowptr[u];
      deg = rowptr[u + 1] - beg;
      op = orow[o];
      ip = irow[o];
    }
    if constexpr (G == kBlock) {
      orient_write_long<G>(r, o, by_id, beg, deg, op, ip, col, rcol, unsorted, otail, icol);
      continue;
    }
    for (int64_t j0 = 0; j0 < deg; j0 += G) {
      const int64_t j = j0 + li;
      const bool valid = j < deg;
      const int32_t x = valid ? rcol[beg + j] : 0;    // gathered by the count pass
      const int32_t rv = by_id ? (valid ? col[beg + j] : 0) : x;
      const bool out = valid && x > r;
      const bool in = valid && x < r;
      const uint64_t bo = ballot(out), bi = ballot(in);
      int32_t po, pi, to, ti;
      if constexpr (G <= kWave) {
        po = popc_below_in_group<G>(bo);
        pi = popc_below_in_group<G>(bi);
        to = __popcll(group_bits<G>(bo));
        ti = __popcll(group_bits<G>(bi));
      } else {
        if (lane_id() == 0) { so[w] = __popcll(bo); si[w] = __popcll(bi); }
        __syncthreads();
        int32_t ao = 0, ai = 0;
        to = 0; ti = 0;
        for (int q = 0; q < kWavesPerBlock; ++q) {
          if (q < w) { ao += so[q]; ai += si[q]; }
          to += so[q]; ti += si[q];
        }
        po = ao + popc_below(bo);
        pi = ai + popc_below(bi);
        __syncthreads();
      }
      if (out) {
        unsorted[op + po] = rv;
        otail[op + po] = (int32_t)o;
      }
      if (in) icol[ip + pi] = rv;
      op += to;
      ip += ti;
    }
  }
}

__device__ __forceinline__ int sort_class(int64_t len) {
  return len <= 16 ? 0 : len <= 64 ? 1 : len <= 256 ? 2 : len <= 4096 ? 3 : 4;
}

__global__ __launch_bounds__(kBlock) void k_copy(const int32_t* __restrict__ src, int64_t n,
                                                 int32_t* __restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock)
    dst[i] = src[i];
}

// What a class pass bins: the out-lists (by length, for sorting), the full
// rows (by degree, the orientation's row-group widths 4, 16, 64, kBlock), or
// the in-lists (by length, for sorting).
enum ClassMode : int { kOutLists = 0, kRowsByDegree = 1, kInLists = 2 };

template <int kMode>
struct ClassSlots {
  static constexpr int count = kMode == kOutLists ? kCSortCount
                               : kMode == kRowsByDegree ? kCRowCount : kCInCount;
  static constexpr int cursor = kMode == kOutLists ? kCSortCursor
                                : kMode == kRowsByDegree ? kCRowCursor : kCInCursor;
};

// Class of rank r's row, or -1 for an empty one.  len: deg+ (out-lists) or
// deg- (in-lists) per rank.
template <int kMode>
__device__ __forceinline__ int row_class(int64_t r, const int32_t* __restrict__ len,
                                         const int32_t* __restrict__ perm,
                                         const int64_t* __restrict__ rowptr) {
  if constexpr (kMode == kRowsByDegree) {
    const int32_t u = perm[r];
    const int64_t d = rowptr[u + 1] - rowptr[u];
    return d == 0 ? -1 : d <= 4 ? 0 : d <= 16 ? 1 : d <= 512 ? 2 : 3;
  } else {
    const int32_t l = len[r];
    return l > 0 ? sort_class(l) : -1;
  }
}

template <int kMode>
__global__ __launch_bounds__(kBlock) void k_count_classes(int32_t n,
                                                          const int32_t* __restrict__ len,
                                                          const int32_t* __restrict__ perm,
                                                          const int64_t* __restrict__ rowptr,
                                                          int32_t* __restrict__ counters) {
  constexpr int kOff = ClassSlots<kMode>::count;
  int32_t h[kSortClasses] = {0, 0, 0, 0, 0};
  for (int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * kBlock) {
    const int c = row_class<kMode>(r, len, perm, rowptr);
#pragma unroll
    for (int q = 0; q < kSortClasses; ++q) h[q] += c == q;
  }
  __shared__ int32_t red[kWavesPerBlock];
#pragma unroll
  for (int q = 0; q < kSortClasses; ++q) {
    const int32_t t = block_sum(h[q], red);
    if (threadIdx.x == 0 && t) atomicAdd(&counters[kOff + q], t);
  }
}

// Rows into their classes.  A workgroup takes kClassChunk rows at a time:
// it counts them per class, reserves their slots with one global atomic per
// class, then places them through LDS cursors (the order inside a class is
// free: each row is then processed on its own).  One atomic per wave and
// class, on five addresses, serialised badly on millions of rows.
constexpr int kClassChunk = 16 * kBlock;

template <int kMode>
__global__ __launch_bounds__(kBlock) void k_scatter_classes(int32_t n,
                                                            const int32_t* __restrict__ len,
                                                            const int32_t* __restrict__ perm,
                                                            const int64_t* __restrict__ rowptr,
                                                            int32_t* __restrict__ counters,
                                                            int32_t* __restrict__ rows) {
  constexpr int kOff = ClassSlots<kMode>::count;
  constexpr int kCur = ClassSlots<kMode>::cursor;
  __shared__ int32_t base[kSortClasses], cnt[kSortClasses], at[kSortClasses];
  if (threadIdx.x == 0) {
    int32_t run = 0;
    for (int q = 0; q < kSortClasses; ++q) { base[q] = run; run += counters[kOff + q]; }
  }
  for (int64_t c0 = (int64_t)blockIdx.x * kClassChunk; c0 < n;
       c0 += (int64_t)gridDim.x * kClassChunk) {
    const int64_t c1 = min((int64_t)n, c0 + kClassChunk);
    if (threadIdx.x < kSortClasses) cnt[threadIdx.x] = 0;
    __syncthreads();
    for (int64_t r0 = c0; r0 < c1; r0 += kBlock) {
      const int64_t r = r0 + threadIdx.x;
      const int c = r < c1 ? row_class<kMode>(r, len, perm, rowptr) : -1;
      for (int q = 0; q < kSortClasses; ++q) {
        const uint64_t mask = ballot(c == q);
        if (mask && lane_id() == 0) atomicAdd(&cnt[q], (int32_t)__popcll(mask));
      }
    }
    __syncthreads();
    if (threadIdx.x < kSortClasses) {
      const int q = threadIdx.x;
      at[q] = base[q] + (cnt[q] ? atomicAdd(&counters[kCur + q], cnt[q]) : 0);
    }
    __syncthreads();
    for (int64_t r0 = c0; r0 < c1; r0 += kBlock) {
      const int64_t r = r0 + threadIdx.x;
      const int c = r < c1 ? row_class<kMode>(r, len, perm, rowptr) : -1;
      for (int q = 0; q < kSortClasses; ++q) {
        const uint64_t mask = ballot(c == q);
        if (!mask) continue;
        int32_t slot = 0;
        if (lane_id() == 0) slot = atomicAdd(&at[q], (int32_t)__popcll(mask));
        slot = __shfl(slot, 0, kWave);
        if (c == q) rows[slot + popc_below(mask)] = (int32_t)r;
      }
    }
    __syncthreads();
  }
}

// Bitonic sort of one row per G-lane group, one element per lane.
template <int G>
__global__ __launch_bounds__(kBlock) void k_sort_lanes(int cbase, int cls, const int32_t* __restrict__ counters,
                                                       const int32_t* __restrict__ rows,
                                                       const int64_t* __restrict__ orow,
                                                       const int32_t* __restrict__ src,
                                                       int32_t* __restrict__ dst) {
  constexpr int kGroups = kBlock / G;
  int32_t base = 0;
  for (int q = 0; q < cls; ++q) base += counters[cbase + q];
  const int32_t count = counters[cbase + cls];
  const int gi = threadIdx.x / G, li = threadIdx.x % G;
  for (int64_t t = (int64_t)blockIdx.x * kGroups + gi; t < count;
       t += (int64_t)gridDim.x * kGroups) {
    const int32_t r = rows[base + t];
    const int64_t beg = orow[r];
    const int64_t len = orow[r + 1] - beg;
    int32_t x = li < len ? src[beg + li] : INT_MAX;
#pragma unroll
    for (int k = 2; k <= G; k <<= 1) {
#pragma unroll
      for (int j = k >> 1; j > 0; j >>= 1) {
        const int32_t y = __shfl_xor(x, j, G);
        const bool up = (li & k) == 0;
        const bool lower = (li & j) == 0;
        x = (lower == up) ? min(x, y) : max(x, y);
      }
    }
    if (li < len) dst[beg + li] = x;
  }
}

// Bitonic sort of one row (64 < len <= 64 * K) per wave, K elements per lane
// in registers: element i = lane * K + k; partners within a lane swap in
// registers, partners across lanes exchange with a shuffle.  No LDS, no
// barrier.
template <int K>
__global__ __launch_bounds__(kBlock) void k_sort_wave(int cbase, int cls,
                                                      const int32_t* __restrict__ counters,
                                                      const int32_t* __restrict__ rows,
                                                      const int64_t* __restrict__ orow,
                                                      const int32_t* __restrict__ src,
                                                      int32_t* __restrict__ dst) {
  constexpr int N = kWave * K;
  int32_t base = 0;
  for (int q = 0; q < cls; ++q) base += counters[cbase + q];
  const int32_t count = counters[cbase + cls];
  const int lane = lane_id();
  for (int64_t t = (int64_t)blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; t < count;
       t += (int64_t)gridDim.x * kWavesPerBlock) {
    const int32_t r = rows[base + t];
    const int64_t beg = orow[r];
    const int32_t len = (int32_t)(orow[r + 1] - beg);
    int32_t x[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = lane * K + k;
      x[k] = i < len ? src[beg + i] : INT_MAX;
    }
#pragma unroll
    for (int sz = 2; sz <= N; sz <<= 1) {
#pragma unroll
      for (int j = sz >> 1; j > 0; j >>= 1) {
        if (j < K) {
#pragma unroll
          for (int k = 0; k < K; ++k) {
            if ((k & j) == 0) {
              const int i = lane * K + k;
              const bool up = (i & sz) == 0;
              const int32_t a = x[k], b = x[k | j];
              const bool swap = (a > b) == up;
              x[k] = swap ? b : a;
              x[k | j] = swap ? a : b;
            }
          }
        } else {
          const int lj = j / K;
          const bool lower = (lane & lj) == 0;
#pragma unroll
          for (int k = 0; k < K; ++k) {
            const int i = lane * K + k;
            const bool up = (i & sz) == 0;
            const int32_t y = __shfl_xor(x[k], lj, kWave);
            x[k] = (lower == up) ? min(x[k], y) : max(x[k], y);
          }
        }
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = lane * K + k;
      if (i < len) dst[beg + i] = x[k];
    }
  }
}

// Bitonic sort in LDS, one row (256 < len <= 4096) per workgroup.
__global__ __launch_bounds__(kBlock) void k_sort_block(int cbase, int cls, const int32_t* __restrict__ counters,
                                                       const int32_t* __restrict__ rows,
                                                       const int64_t* __restrict__ orow,
                                                       const int32_t* __restrict__ src,
                                                       int32_t* __restrict__ dst) {
  __shared__ int32_t s[4096];
  int32_t base = 0;
  for (int q = 0; q < cls; ++q) base += counters[cbase + q];
  const int32_t count = counters[cbase + cls];
  for (int64_t t = blockIdx.x; t < count; t += gridDim.x) {
    const int32_t r = rows[base + t];
    const int64_t beg = orow[r];
    const int32_t len = (int32_t)(orow[r + 1] - beg);
    int N = 1;
    while (N < len) N <<= 1;
    for (int i = threadIdx.x; i < N; i += kBlock) s[i] = i < len ? src[beg + i] : INT_MAX;
    __syncthreads();
    for (int k = 2; k <= N; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int idx = threadIdx.x; idx < N / 2; idx += kBlock) {
          const int i = (idx / j) * 2 * j + (idx % j);
          const int p = i + j;
          const bool up = (i & k) == 0;
          const int32_t a = s[i], b = s[p];
          if ((a > b) == up) { s[i] = b; s[p] = a; }
        }
        __syncthreads();
      }
    }
    for (int i = threadIdx.x; i < len; i += kBlock) dst[beg + i] = s[i];
    __syncthreads();
  }
}

// Long rows: values are distinct labels, so a bitmap in LDS sorts them, one
// window of kBits ids at a time.  A row whose [min, max] fits one window is
// set into the bitmap straight from src.  A wider row is first partitioned by
// window into its place in dst (a histogram of windows, its prefix sum, and
// a scatter whose lanes with the same window take consecutive slots with one
// LDS atomic per group); then each window's bucket is read back, set into the
// bitmap and written over itself in ascending order.  Every entry is read
// four times and written twice however wide the row's range is.
constexpr int64_t kBits = (int64_t)kBitmapWords * 32;
constexpr int kMaxWindows = 8192;   // (INT32_MAX + 1) / kBits: every id range

// Windows a row of labels in [0, label_range) can span, and the dynamic LDS
// of k_sort_bitmap: the bitmap, then the window offsets.  Labels are ranks
// or ids below n, so with n = 2^26 the offsets take 1 KiB and four
// workgroups share a CU.
inline int sort_windows(int64_t label_range) {
  return (int)std::min<int64_t>(kMaxWindows, (std::max<int64_t>(label_range, 1) - 1) / kBits + 1);
}
inline size_t sort_bitmap_lds(int64_t label_range) {
  return sizeof(uint32_t) * (size_t)(kBitmapWords + sort_windows(label_range) + 1);
}

// Lanes (among the active ones) whose window w equals this lane's; w < 2^nbits.
__device__ __forceinline__ uint64_t match_window(int w, int nbits, bool active) {
  uint64_t peers = ballot(active);
  for (int b = 0; b < nbits; ++b) {
    const bool bit = (w >> b) & 1;
    const uint64_t m = ballot(bit);
    peers &= bit ? m : ~m;
  }
  return peers;
}

// Writes the set bits of bm (ids w0 + bit index) to out[0..) in ascending
// order; `tmp` holds kWavesPerBlock + 1 entries.  Ends with a barrier.
__device__ __forceinline__ int64_t emit_bitmap(const uint32_t* bm, int64_t w0, int32_t* out,
                                               int64_t* tmp) {
  constexpr int kWordsPerThread = kBitmapWords / kBlock;
  const int wbeg = threadIdx.x * kWordsPerThread;
  int64_t c = 0;
  for (int q = 0; q < kWordsPerThread; ++q) c += __popc(bm[wbeg + q]);
  int64_t total;
  int64_t pos = block_exclusive_scan(c, tmp, &total);
  for (int q = 0; q < kWordsPerThread; ++q) {
    uint32_t bits = bm[wbeg + q];
    while (bits) {
      const int b = __ffs(bits) - 1;
      out[pos++] = (int32_t)(w0 + (int64_t)(wbeg + q) * 32 + b);
      bits &= bits - 1;
    }
  }
  __syncthreads();
  return total;
}

// One workgroup per row; every pass over a row keeps kSortUnroll loads per
// thread in flight.
constexpr int kSortUnroll = 8;
constexpr int32_t kRankSortMax = 512;    // buckets up to this size are ranked in LDS

__global__ __launch_bounds__(kBlock) void k_sort_bitmap(int cbase, int cls, const int32_t* __restrict__ counters,
                                                        const int32_t* __restrict__ rows,
                                                        const int64_t* __restrict__ orow,
                                                        const int32_t* __restrict__ src,
                                                        int32_t* __restrict__ dst,
                                                        int max_windows) {
  constexpr int U = kSortUnroll;
  extern __shared__ uint32_t sort_lds[];
  uint32_t* bm = sort_lds;                                            // kBitmapWords
  int32_t* woff = reinterpret_cast<int32_t*>(sort_lds + kBitmapWords);  // max_windows + 1
  __shared__ int64_t tmp[kWavesPerBlock + 1];
  __shared__ int32_t red[2][kWavesPerBlock];
  __shared__ int32_t stmp[kWavesPerBlock + 1];
  int32_t* cursor = reinterpret_cast<int32_t*>(bm);   // during the scatter only
  int32_t base = 0;
  for (int q = 0; q < cls; ++q) base += counters[cbase + q];
  const int32_t count = counters[cbase + cls];
  for (int64_t t = blockIdx.x; t < count; t += gridDim.x) {
    const int32_t r = rows[base + t];
    const int64_t beg = orow[r];
    const int64_t len = orow[r + 1] - beg;
    int32_t lo = INT_MAX, hi = INT_MIN;
    for (int64_t i0 = threadIdx.x; i0 < len; i0 += (int64_t)kBlock * U) {
      int32_t v[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int64_t i = i0 + q * kBlock;
        v[q] = src[beg + (i < len ? i : 0)];
      }
#pragma unroll
      for (int q = 0; q < U; ++q)
        if (i0 + q * kBlock < len) { lo = min(lo, v[q]); hi = max(hi, v[q]); }
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {
      lo = min(lo, __shfl_xor(lo, o, kWave));
      hi = max(hi, __shfl_xor(hi, o, kWave));
    }
    if (lane_id() == 0) { red[0][threadIdx.x / kWave] = lo; red[1][threadIdx.x / kWave] = hi; }
    __syncthreads();
    lo = red[0][0]; hi = red[1][0];
    for (int q = 1; q < kWavesPerBlock; ++q) { lo = min(lo, red[0][q]); hi = max(hi, red[1][q]); }
    __syncthreads();
    const int nwin = (int)(((int64_t)hi - lo) / kBits) + 1;   // <= max_windows
    if (nwin == 1) {
      for (int i = threadIdx.x; i < kBitmapWords; i += kBlock) bm[i] = 0u;
      __syncthreads();
      for (int64_t i0 = threadIdx.x; i0 < len; i0 += (int64_t)kBlock * U) {
        int32_t v[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
          const int64_t i = i0 + q * kBlock;
          v[q] = src[beg + (i < len ? i : 0)];
        }
#pragma unroll
        for (int q = 0; q < U; ++q)
          if (i0 + q * kBlock < len) {
            const int64_t off = (int64_t)v[q] - lo;
            atomicOr(&bm[off >> 5], 1u << (off & 31));
          }
      }
      __syncthreads();
      emit_bitmap(bm, lo, dst + beg, tmp);
      continue;
    }
    // histogram of windows
    const int nbits = ceil_log2(nwin);
    for (int i = threadIdx.x; i < nwin; i += kBlock) woff[i] = 0;
    __syncthreads();
    for (int64_t i0 = 0; i0 < len; i0 += (int64_t)kBlock * U) {
      int32_t v[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int64_t i = i0 + q * kBlock + threadIdx.x;
        v[q] = src[beg + (i < len ? i : 0)];
      }
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const bool live = i0 + q * kBlock + threadIdx.x < len;
        const int w = live ? (int)(((int64_t)v[q] - lo) / kBits) : 0;
        const uint64_t peers = match_window(w, nbits, live);
        if (live && popc_below(peers) == 0) atomicAdd(&woff[w], (int32_t)__popcll(peers));
      }
    }
    __syncthreads();
    // exclusive prefix over the windows: each thread a run of consecutive ones
    {
      const int kPer = (max_windows + kBlock - 1) / kBlock;
      const int w0 = threadIdx.x * kPer;
      int32_t run = 0;
      for (int q = 0; q < kPer; ++q)
        if (w0 + q < nwin) run += woff[w0 + q];
      int32_t total;
      int32_t at = block_exclusive_scan(run, stmp, &total);
      for (int q = 0; q < kPer; ++q)
        if (w0 + q < nwin) {
          const int32_t c = woff[w0 + q];
          woff[w0 + q] = at;
          at += c;
        }
      if (threadIdx.x == 0) woff[nwin] = total;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nwin; i += kBlock) cursor[i] = woff[i];
    __syncthreads();
    // scatter into the row's place in dst, bucketed by window
    for (int64_t i0 = 0; i0 < len; i0 += (int64_t)kBlock * U) {
      int32_t v[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int64_t i = i0 + q * kBlock + threadIdx.x;
        v[q] = src[beg + (i < len ? i : 0)];
      }
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const bool live = i0 + q * kBlock + threadIdx.x < len;
        const int w = live ? (int)(((int64_t)v[q] - lo) / kBits) : 0;
        const uint64_t peers = match_window(w, nbits, live);
        const int leader = peers ? __ffsll((long long)peers) - 1 : 0;
        int32_t at = 0;
        if (live && lane_id() == leader) at = atomicAdd(&cursor[w], (int32_t)__popcll(peers));
        at = __shfl(at, leader, kWave);
        if (live) dst[beg + at + popc_below(peers)] = v[q];
      }
    }
    __syncthreads();
    // each window's bucket written over itself in order: a sparse bucket by
    // ranks counted in LDS (each entry's rank is the number of smaller ones;
    // entries are distinct), a denser one through the bitmap, whose clearing
    // and scan cost the same however few entries it holds
    for (int w = 0; w < nwin; ++w) {
      const int32_t b0 = woff[w], b1 = woff[w + 1];
      if (b1 == b0) continue;
      if (b1 - b0 <= kRankSortMax) {
        const int32_t nb = b1 - b0;
        int32_t* vals = reinterpret_cast<int32_t*>(bm);
        for (int32_t i = threadIdx.x; i < nb; i += kBlock) vals[i] = dst[beg + b0 + i];
        __syncthreads();
        for (int32_t i = threadIdx.x; i < nb; i += kBlock) {
          const int32_t v = vals[i];
          int32_t r = 0;
          for (int32_t j = 0; j < nb; ++j) r += vals[j] < v;
          dst[beg + b0 + r] = v;
        }
        __syncthreads();
        continue;
      }
      const int64_t w0 = (int64_t)lo + (int64_t)w * kBits;
      for (int i = threadIdx.x; i < kBitmapWords; i += kBlock) bm[i] = 0u;
      __syncthreads();
      for (int32_t i0 = b0 + threadIdx.x; i0 < b1; i0 += kBlock * U) {
        int32_t v[U];
#pragma unroll
        for (int q = 0; q < U; ++q) {
          const int32_t i = i0 + q * kBlock;
          v[q] = dst[beg + (i < b1 ? i : b0)];
        }
#pragma unroll
        for (int q = 0; q < U; ++q)
          if (i0 + q * kBlock < b1) {
            const int64_t off = (int64_t)v[q] - w0;
            atomicOr(&bm[off >> 5], 1u << (off & 31));
          }
      }
      __syncthreads();
      emit_bitmap(bm, w0, dst + beg + b0, tmp);
    }
  }
}

unsigned grid_for(int64_t items, int per_block) {
  int64_t b = cdiv(items, per_block);
  if (b < 1) b = 1;
  if (b > kGrid * 4) b = kGrid * 4;
  return (unsigned)b;
}

template <int G, typename F>
hipError_t launch_rows(const RowSet& rs, int64_t bound, hipStream_t s, F f) {
  if (bound <= 0) return hipSuccess;
  f(rs, grid_for(bound, kBlock / G), s);
  return hipGetLastError();
}

#define AOT_TRY(x)                          \
  do {                                      \
    hipError_t e_ = (x);                    \
    if (e_ != hipSuccess) {                 \
      *err = hipGetErrorString(e_);         \
      return -5;                            \
    }                                       \
  } while (0)

}  // namespace

size_t orient_workspace_bytes(int32_t n, int64_t nnz) {
  Carve c(nullptr, 0);
  const int64_t m = nnz / 2;
  for (int i = 0; i < 4; ++i) c.take<int32_t>(n);  // key/val a/b
  c.take<int32_t>(n);                               // dplus
  c.take<int32_t>(n);                               // dminus
  c.take<int32_t>(m);                               // unsorted
  c.take<int32_t>(nnz);                             // rcol
  c.take<int32_t>(n);                               // rows_by_len
  c.take<int32_t>(kCounters);
  c.take<char>((int64_t)scan_workspace(n));
  c.take<char>((int64_t)radix_workspace(n));
  return c.used;
}

namespace {

// Sorts every list of (offsets, src) into dst by its length class; cbase:
// the counter slots holding the class sizes.
hipError_t sort_lists(int cbase, unsigned g_small, const int32_t* counters, const int32_t* rows,
                      const int64_t* offsets, const int32_t* src, int32_t* dst,
                      int64_t label_range, hipStream_t s) {
  k_sort_lanes<16><<<g_small, kBlock, 0, s>>>(cbase, 0, counters, rows, offsets, src, dst);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_sort_lanes<64><<<g_small, kBlock, 0, s>>>(cbase, 1, counters, rows, offsets, src, dst);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_sort_wave<4><<<g_small, kBlock, 0, s>>>(cbase, 2, counters, rows, offsets, src, dst);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_sort_block<<<kGrid, kBlock, 0, s>>>(cbase, 3, counters, rows, offsets, src, dst);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  k_sort_bitmap<<<1024, kBlock, sort_bitmap_lds(label_range), s>>>(
      cbase, 4, counters, rows, offsets, src, dst, sort_windows(label_range));
  return hipGetLastError();
}

// Batch mode: sort keys (graph, degree) with `bits` key bits, and row lists
// instead of rank ranges, so that nothing is read back to the host.
struct BatchKeys {
  const int64_t* voff;   // device [count+1]
  int32_t count;
  int dbits, bits;
};

constexpr int kCoreBatch = 16;      // sub-rounds launched between progress checks
constexpr unsigned kCoreGrid = 256;  // workgroups of the per-sub-round launches

// round[v] of the core order into keys, ids into vals; *rounds = sub-rounds.
// cur, front, la and lb are n-entry scratch arrays (la, lb: lists of the
// remaining vertices, compacted whenever fewer than half of a list remain).
int core_order(int32_t n, const int64_t* rowptr, const int32_t* col, int32_t* keys, int32_t* vals,
               int32_t* cur, int32_t* front, int32_t* la, int32_t* lb, int32_t* counters,
               int32_t* rounds, hipStream_t s, const char** err) {
  const unsigned gv = std::min(grid_for(n, kBlock), 1024u);
  AOT_TRY(fill_i32(counters + kCCoreMin, 2, INT32_MAX, s));
  AOT_TRY(fill_i32(counters + kCCoreLevel, kCounters - kCCoreLevel, 0, s));
  k_core_init<<<gv, kBlock, 0, s>>>(n, rowptr, cur, keys, vals, counters);
  AOT_TRY(hipGetLastError());
  int32_t left = n;
  int32_t r = 0;
  const int32_t* list = nullptr;      // null: every vertex
  int32_t len = n;
  while (left > 0) {
    const unsigned gm = std::min(grid_for(len, kBlock), kCoreGrid);
    for (int b = 0; b < kCoreBatch; ++b, ++r) {
      k_core_mark<<<gm, kBlock, 0, s>>>(n, len, list, rowptr, cur, keys, front, counters, r);
      k_core_update<<<kCoreGrid, kBlock, 0, s>>>(n, rowptr, col, front, keys, cur, counters, r);
      AOT_TRY(hipGetLastError());
    }
    int32_t hc[2];
    AOT_TRY(hipMemcpyAsync(hc, counters + kCCoreLeft, sizeof(hc), hipMemcpyDeviceToHost, s));
    AOT_TRY(hipStreamSynchronize(s));
    // every sub-round with vertices left removes at least the one of least degree
    if (hc[0] >= left) {
      *err = "core peeling made no progress";
      return -5;
    }
    left = hc[0];
    *rounds = hc[1];
    if (left > 0 && left < len / 2) {
      int32_t* out = list == la ? lb : la;
      AOT_TRY(fill_i32(counters + kCCoreList, 1, 0, s));
      k_core_compact<<<std::min(grid_for(len, kBlock), 1024u), kBlock, 0, s>>>(len, list, keys,
                                                                             out, counters);
      AOT_TRY(hipGetLastError());
      list = out;
      len = left;                    // exactly the vertices not yet removed
    }
  }
  return 0;
}

int orient_impl(int32_t n, int64_t nnz, const int64_t* rowptr, const int32_t* col, bool validate,
                bool in_by_rank, bool core, bool by_id, const BatchKeys* bk, int64_t* orow,
                int32_t* ocol,
                int32_t* otail,
                int32_t* perm, int32_t* rank, int64_t* irow, int32_t* icol, void* ws,
                size_t ws_bytes, hipStream_t s, const char** err) {
  const int64_t m = nnz / 2;
  Carve c(ws, ws_bytes);
  int32_t* key_a = c.take<int32_t>(n);
  int32_t* val_a = c.take<int32_t>(n);
  int32_t* key_b = c.take<int32_t>(n);
  int32_t* val_b = c.take<int32_t>(n);
  int32_t* dplus = c.take<int32_t>(n);
  int32_t* dminus = c.take<int32_t>(n);
  int32_t* unsorted = c.take<int32_t>(m);
  int32_t* rcol = c.take<int32_t>(nnz);   // rank of every symmetric entry, by input position
  int32_t* rows = c.take<int32_t>(n);
  int32_t* counters = c.take<int32_t>(kCounters);
  void* scan_tmp = c.take<char>((int64_t)scan_workspace(n));
  void* radix_tmp = c.take<char>((int64_t)radix_workspace(n));
  if (!c.ok()) {
    *err = "orientation workspace too small";
    return -4;
  }
  AOT_TRY(fill_i32(counters, kCounters, 0, s));
  if (validate) {
    k_validate_rowptr<<<grid_for(n + 1, kBlock), kBlock, 0, s>>>(n, nnz, rowptr, counters);
    AOT_TRY(hipGetLastError());
    int32_t flag = 0;
    AOT_TRY(hipMemcpyAsync(&flag, counters + kCError, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    AOT_TRY(hipStreamSynchronize(s));
    if (flag) {
      *err = "row offsets are not a valid CSR (rowptr[0] != 0, decreasing, or end != nnz)";
      return -2;
    }
    k_validate_rows<<<grid_for((int64_t)n * kWave, kBlock), kBlock, 0, s>>>(n, rowptr, col,
                                                                             counters);
    AOT_TRY(hipGetLastError());
    AOT_TRY(hipMemcpyAsync(&flag, counters + kCError, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    AOT_TRY(hipStreamSynchronize(s));
    if (flag) {
      *err = (flag & kErrRange)  ? "column id out of range"
             : (flag & kErrLoop) ? "self-loop"
             : (flag & kErrOrder) ? "row not strictly ascending (unsorted or duplicate)"
                                  : "graph is not symmetric";
      return -2;
    }
  }
  if (n == 0) {
    AOT_TRY(fill_i64(orow, 1, 0, s));
    AOT_TRY(fill_i64(irow, 1, 0, s));
    return 0;
  }
  int bits;
  int32_t c0 = 0, c4 = 0, c16 = 0, c512 = 0;
  // rank order is degree order only for the plain single-graph case; the
  // others process rows from lists built on the device
  const bool lists = bk || core;
  if (core) {
    int32_t rounds = 0;
    const int rc = core_order(n, rowptr, col, key_a, val_a, dplus, dminus, key_b, val_b, counters,
                              &rounds, s, err);
    if (rc) return rc;
    bits = ceil_log2((int64_t)rounds + 1);
  } else if (!bk) {
    k_degree<<<std::min(grid_for(n, kBlock), 1024u), kBlock, 0, s>>>(n, rowptr, key_a, val_a,
                                                                     counters);
    AOT_TRY(hipGetLastError());
    int32_t hc[kCounters];
    AOT_TRY(hipMemcpyAsync(hc, counters, sizeof(hc), hipMemcpyDeviceToHost, s));
    AOT_TRY(hipStreamSynchronize(s));
    bits = ceil_log2((int64_t)hc[kCMaxDeg] + 1);
    c0 = hc[kCDeg0]; c4 = hc[kCDeg4]; c16 = hc[kCDeg16]; c512 = hc[kCDeg512];
  } else {
    k_batch_keys<<<grid_for(n, kBlock), kBlock, 0, s>>>(n, bk->voff, bk->count, bk->dbits,
                                                         rowptr, key_a, val_a);
    AOT_TRY(hipGetLastError());
    bits = bk->bits;
  }
  int32_t *sk, *sv;
  AOT_TRY(radix_sort_pairs(key_a, val_a, key_b, val_b, n, bits, radix_tmp, s, &sk, &sv));
  // With labels by id, the order eta (rank -> id, id -> rank) only directs
  // the edges: it goes to the two key buffers, free once the sorted ids sv
  // (a value buffer) are read, and perm/rank become the identity.
  int32_t* eperm = by_id ? key_a : perm;
  int32_t* erank = by_id ? key_b : rank;
  k_perm_rank<<<grid_for(n, kBlock), kBlock, 0, s>>>(n, sv, eperm, erank);
  AOT_TRY(hipGetLastError());
  if (by_id) {
    k_identity<<<grid_for(n, kBlock), kBlock, 0, s>>>(n, perm, rank);
    AOT_TRY(hipGetLastError());
  }

  // Row sets of the four row-group widths.  Single graph: rank order is
  // degree order, so each is a rank range.  Batch: ranks go graph by graph,
  // so each is a list built on the device.
  RowSet sets[4];
  int64_t bound[4];
  const int32_t cuts[5] = {c0, c4, c16, c512, n};
  for (int q = 0; q < 4; ++q) {
    sets[q].r0 = cuts[q];
    sets[q].r1 = cuts[q + 1];
    sets[q].rows = lists ? rows : nullptr;
    sets[q].counters = counters;
    sets[q].cls = q;
    bound[q] = lists ? (int64_t)n : (int64_t)cuts[q + 1] - cuts[q];
  }
  if (lists) {
    AOT_TRY(fill_i32(dplus, n, 0, s));
    AOT_TRY(fill_i32(dminus, n, 0, s));
    k_count_classes<kRowsByDegree><<<std::min(grid_for(n, kBlock), 1024u), kBlock, 0, s>>>(
        n, dplus, eperm, rowptr, counters);
    AOT_TRY(hipGetLastError());
    k_scatter_classes<kRowsByDegree><<<grid_for(n, kClassChunk), kBlock, 0, s>>>(n, dplus, eperm, rowptr,
                                                                   counters, rows);
    AOT_TRY(hipGetLastError());
  } else {
    // rows of degree 0 are not visited: the first c0 ranks, or with labels
    // by id anywhere
    AOT_TRY(fill_i32(dplus, by_id ? n : c0, 0, s));
    AOT_TRY(fill_i32(dminus, by_id ? n : c0, 0, s));
  }
#define ROWS(q, G, KERNEL, ...)                                                          \
  AOT_TRY(launch_rows<G>(sets[q], bound[q], s,                                          \
                         [&](const RowSet& rs, unsigned grid, hipStream_t st) {          \
                           KERNEL<G><<<grid, kBlock, 0, st>>>(rs, __VA_ARGS__);          \
                         }))
  ROWS(0, 4, k_orient_count, rowptr, col, eperm, erank, by_id, dplus, dminus, rcol);
  ROWS(1, 16, k_orient_count, rowptr, col, eperm, erank, by_id, dplus, dminus, rcol);
  ROWS(2, 64, k_orient_count, rowptr, col, eperm, erank, by_id, dplus, dminus, rcol);
  ROWS(3, 256, k_orient_count, rowptr, col, eperm, erank, by_id, dplus, dminus, rcol);
  AOT_TRY(exclusive_scan(dplus, orow, n, scan_tmp, s));
  AOT_TRY(exclusive_scan(dminus, irow, n, scan_tmp, s));
  ROWS(0, 4, k_orient_write, rowptr, col, eperm, erank, by_id, orow, irow, unsorted, otail, icol, rcol);
  ROWS(1, 16, k_orient_write, rowptr, col, eperm, erank, by_id, orow, irow, unsorted, otail, icol, rcol);
  ROWS(2, 64, k_orient_write, rowptr, col, eperm, erank, by_id, orow, irow, unsorted, otail, icol, rcol);
  ROWS(3, 256, k_orient_write, rowptr, col, eperm, erank, by_id, orow, irow, unsorted, otail, icol, rcol);
#undef ROWS

  // sort each out-list into ocol (with labels by id, rows of a valid CSR
  // are already ascending; the sort still guarantees it for the probe
  // kernels' windows and searches)
  k_count_classes<kOutLists><<<std::min(grid_for(n, kBlock), 1024u), kBlock, 0, s>>>(
      n, dplus, perm, rowptr, counters);
  AOT_TRY(hipGetLastError());
  k_scatter_classes<kOutLists><<<grid_for(n, kClassChunk), kBlock, 0, s>>>(n, dplus, perm, rowptr,
                                                                  counters, rows);
  AOT_TRY(hipGetLastError());
  const unsigned g_small = (unsigned)std::min<int64_t>(kGrid, cdiv(n, kBlock / 16) + 1);
  AOT_TRY(sort_lists(kCSortCount, g_small, counters, rows, orow, unsorted, ocol, n, s));

  if (!in_by_rank) return 0;
  // sort each in-list into ascending rank (= edge order of the in-edges): the
  // in-lists were written to icol; move them to the now free scratch first
  AOT_TRY(fill_i32(counters + kCInCount, 2 * kSortClasses, 0, s));
  k_copy<<<grid_for(m, kBlock), kBlock, 0, s>>>(icol, m, unsorted);
  AOT_TRY(hipGetLastError());
  k_count_classes<kInLists><<<std::min(grid_for(n, kBlock), 1024u), kBlock, 0, s>>>(
      n, dminus, perm, rowptr, counters);
  AOT_TRY(hipGetLastError());
  k_scatter_classes<kInLists><<<grid_for(n, kClassChunk), kBlock, 0, s>>>(n, dminus, perm, rowptr,
                                                                     counters, rows);
  AOT_TRY(hipGetLastError());
  AOT_TRY(sort_lists(kCInCount, g_small, counters, rows, irow, unsorted, icol, n, s));
  return 0;
}

}  // namespace

int orient_run(int32_t n, int64_t nnz, const int64_t* rowptr, const int32_t* col, bool validate,
               bool in_by_rank, bool core, bool by_id, int64_t* orow, int32_t* ocol, int32_t* otail,
               int32_t* perm, int32_t* rank, int64_t* irow, int32_t* icol, void* ws,
               size_t ws_bytes, hipStream_t s, const char** err) {
  return orient_impl(n, nnz, rowptr, col, validate, in_by_rank, core, by_id, nullptr, orow, ocol,
                     otail, perm, rank, irow, icol, ws, ws_bytes, s, err);
}

int orient_batch_run(int32_t n, int64_t nnz, const int64_t* rowptr, const int32_t* col,
                     const int64_t* voff, int32_t count, int dbits, int gbits, int64_t* orow,
                     int32_t* ocol, int32_t* otail, int32_t* perm, int32_t* rank, int64_t* irow,
                     int32_t* icol, void* ws, size_t ws_bytes, hipStream_t s, const char** err) {
  BatchKeys bk{voff, count, dbits, dbits + gbits};
  return orient_impl(n, nnz, rowptr, col, false, false, false, false, &bk, orow, ocol, otail, perm, rank,
                     irow,
                     icol,
                     ws, ws_bytes, s, err);
}

}  // namespace aot
