// Adaptive-orientation probe passes (Algorithm 3's two loops; Section 3.1,
// "The main idea"; Section 3.2, Correctness, Time Complexity).
//
// Every directed edge e = <u,v> of the oriented graph is charged to its owner
// b, the endpoint with the larger (deg+, rank) (ties by id, the footnote of
// Section 3.2); the other endpoint s is probed: each w in N+(s) is looked up
// in an index of N+(b), so edge e costs min(deg+(u), deg+(v)) look-ups.
//
// Two paths, by the owner's out-degree:
//  * heavy owners (deg+(b) >= heavy_min): owner-grouped, as in Algorithm 3,
//    where each pivot builds its index once (Section 3.2, the remark on the
//    bitmap).  A workgroup takes one work item = an owner and a window of up
//    to kItemSpan of its neighbours (out-list then in-list), stages N+(b) in
//    LDS as a bitmap over [min N+(b), max N+(b)] or as an open-addressing
//    hash, then each wave probes one owned neighbour's out-list at a time.
//  * light owners: edge-centric.  Edges are binned by c = min(deg+) so that
//    a bin's edges get G lanes each with G close to c, and every lane
//    binary-searches its w in the (short, cache-resident) sorted N+(b).
// The count pass writes cnt[e]; an exclusive scan gives each edge's slot in
// the global triangle list; the write pass repeats the probes and stores the
// hits in ascending w at those slots.
#include <algorithm>
#include <climits>

#include "kernels.hpp"

namespace aot {

namespace {

constexpr int kLightBins = 8;       // c in {1}, {2}, (2,4], (4,8], ..., (64,128]
constexpr int kItemSpan = 1024;     // neighbours of one owner per work item
constexpr int kIndexWords = 8192;   // LDS index: 32 KiB
constexpr int kGrid = 4096;
constexpr int kDefaultHeavyMin = 32;

enum : int {
  kCBinCount = 0,                   // [0..7]
  kCBinCursor = 8,                  // [8..15]
  kCItems = 16,
  kCounters32 = 32,
};

// Index arms of the heavy (owner-grouped) path; the numbers are the codes
// of a dispatch table's heavy entries.
enum Arm : int { kArmBitmap = 0, kArmHash = 1, kArmGlobal = 2, kArmSorted = 3, kNumArms = 4 };
constexpr int kHeavyClasses = 16;   // owner classes by ceil(log2 deg+(b))

// Per-bucket choices: lanes per edge of each light bin, index arm of each
// heavy owner class.
struct Plan {
  int32_t light_tile[kLightBins];
  int32_t heavy_arm[kHeavyClasses];
};

__device__ __forceinline__ int light_bin(int32_t c) {
  const int k = c <= 1 ? 0 : ceil_log2(c);
  return k < kLightBins ? k : kLightBins - 1;   // last bin takes everything longer
}

struct EdgeEnds {
  int32_t s, b;      // probe side, owner
  int32_t c, db;     // deg+(s), deg+(b)
};

__device__ __forceinline__ EdgeEnds edge_ends(const int64_t* __restrict__ orow, int32_t u,
                                              int32_t v) {
  const int32_t du = (int32_t)(orow[u + 1] - orow[u]);
  const int32_t dv = (int32_t)(orow[v + 1] - orow[v]);
  // u < v in rank, so on a tie u has the smaller (deg+, id) and is probed
  EdgeEnds r;
  if (du <= dv) { r.s = u; r.b = v; r.c = du; r.db = dv; }
  else { r.s = v; r.b = u; r.c = dv; r.db = du; }
  return r;
}

// ---------------------------------------------------------------- binning

__global__ __launch_bounds__(kBlock) void k_bin_count(int64_t m, const int64_t* __restrict__ orow,
                                                      const int32_t* __restrict__ ocol,
                                                      const int32_t* __restrict__ otail,
                                                      int32_t heavy_min,
                                                      int32_t* __restrict__ cnt,
                                                      int32_t* __restrict__ counters,
                                                      unsigned long long* __restrict__ probes) {
  __shared__ int32_t h[kLightBins];
  __shared__ unsigned long long red[kWavesPerBlock];
  if (threadIdx.x < kLightBins) h[threadIdx.x] = 0;
  __syncthreads();
  unsigned long long sum = 0;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * kBlock) {
    const EdgeEnds x = edge_ends(orow, otail[e], ocol[e]);
    sum += (unsigned long long)x.c;
    if (x.db >= heavy_min) continue;             // the owner's work item counts it
    if (x.c == 0) { cnt[e] = 0; continue; }
    atomicAdd(&h[light_bin(x.c)], 1);
  }
  sum = wave_sum(sum);
  if (lane_id() == 0) red[threadIdx.x / kWave] = sum;
  __syncthreads();
  if (threadIdx.x < kLightBins) atomicAdd(&counters[kCBinCount + threadIdx.x], h[threadIdx.x]);
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int q = 0; q < kWavesPerBlock; ++q) t += red[q];
    atomicAdd(probes, t);
  }
}

__global__ __launch_bounds__(kBlock) void k_bin_scatter(int64_t m, const int64_t* __restrict__ orow,
                                                        const int32_t* __restrict__ ocol,
                                                        const int32_t* __restrict__ otail,
                                                        int32_t heavy_min,
                                                        int32_t* __restrict__ counters,
                                                        int32_t* __restrict__ elist) {
  __shared__ int32_t base[kLightBins];
  if (threadIdx.x == 0) {
    int32_t run = 0;
    for (int q = 0; q < kLightBins; ++q) { base[q] = run; run += counters[kCBinCount + q]; }
  }
  __syncthreads();
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < m;
       e += (int64_t)gridDim.x * kBlock) {
    const EdgeEnds x = edge_ends(orow, otail[e], ocol[e]);
    if (x.db >= heavy_min || x.c == 0) continue;
    const int k = light_bin(x.c);
    elist[base[k] + atomicAdd(&counters[kCBinCursor + k], 1)] = (int32_t)e;
  }
}

// Work items of the heavy owners: (owner, first neighbour index).
__global__ __launch_bounds__(kBlock) void k_make_items(int32_t n, const int64_t* __restrict__ orow,
                                                       const int64_t* __restrict__ irow,
                                                       int32_t heavy_min,
                                                       int32_t* __restrict__ counters,
                                                       int2* __restrict__ items) {
  for (int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x; b < n;
       b += (int64_t)gridDim.x * kBlock) {
    const int64_t db = orow[b + 1] - orow[b];
    if (db < heavy_min) continue;
    const int64_t deg = db + irow[b + 1] - irow[b];
    const int32_t k = (int32_t)((deg + kItemSpan - 1) / kItemSpan);
    const int32_t at = atomicAdd(&counters[kCItems], k);
    for (int32_t q = 0; q < k; ++q) items[at + q] = make_int2((int32_t)b, q * kItemSpan);
  }
}

// ---------------------------------------------------------------- LDS index

struct Index {
  int arm;
  int32_t lo, span;   // bitmap window
  int32_t mask;       // hash table size - 1
  int shift;          // hash: 32 - log2(size)
  const int32_t* list;
  int32_t len;
};

__device__ __forceinline__ uint32_t hash_slot(int32_t w) {
  return (uint32_t)w * 0x9E3779B1u;
}

// Builds the index of N+(b) (sorted list `a` of length db) in `lds` with the
// requested arm, falling back (bitmap -> hash -> sorted -> global) when the
// owner does not fit the arm's LDS budget.
__device__ Index build_index(const int32_t* __restrict__ a, int32_t db, uint32_t* lds, int arm) {
  Index ix;
  ix.list = a;
  ix.len = db;
  ix.lo = a[0];
  const int32_t hi = a[db - 1];
  ix.span = hi - ix.lo + 1;
  const bool bitmap_fits = (int64_t)ix.span <= (int64_t)kIndexWords * 32;
  const bool hash_fits = 2 * (int64_t)db <= kIndexWords;
  const bool sorted_fits = (int64_t)db <= kIndexWords;
  if (arm == kArmBitmap && !bitmap_fits) arm = kArmHash;
  if (arm == kArmHash && !hash_fits) arm = kArmSorted;
  if (arm == kArmSorted && !sorted_fits) arm = kArmGlobal;
  ix.arm = arm;
  if (arm == kArmBitmap) {
    const int words = (ix.span + 31) >> 5;
    for (int i = threadIdx.x; i < words; i += kBlock) lds[i] = 0u;
    __syncthreads();
    for (int i = threadIdx.x; i < db; i += kBlock) {
      const int32_t off = a[i] - ix.lo;
      atomicOr(&lds[off >> 5], 1u << (off & 31));
    }
  } else if (arm == kArmHash) {
    int size = 1;
    while (size < 2 * db) size <<= 1;
    ix.mask = size - 1;
    ix.shift = 32 - ceil_log2(size);
    for (int i = threadIdx.x; i < size; i += kBlock) lds[i] = 0xFFFFFFFFu;
    __syncthreads();
    for (int i = threadIdx.x; i < db; i += kBlock) {
      const uint32_t w = (uint32_t)a[i];
      uint32_t h = hash_slot((int32_t)w) >> ix.shift;
      while (atomicCAS(&lds[h], 0xFFFFFFFFu, w) != 0xFFFFFFFFu) h = (h + 1) & (uint32_t)ix.mask;
    }
  } else if (arm == kArmSorted) {
    for (int i = threadIdx.x; i < db; i += kBlock) lds[i] = (uint32_t)a[i];
  }
  __syncthreads();
  return ix;
}

__device__ __forceinline__ bool index_has(const Index& ix, const uint32_t* lds, int32_t w) {
  if (ix.arm == kArmBitmap) {
    const uint32_t off = (uint32_t)(w - ix.lo);
    if (off >= (uint32_t)ix.span) return false;
    return (lds[off >> 5] >> (off & 31)) & 1u;
  }
  if (ix.arm == kArmHash) {
    uint32_t h = hash_slot(w) >> ix.shift;
    while (true) {
      const uint32_t k = lds[h];
      if (k == (uint32_t)w) return true;
      if (k == 0xFFFFFFFFu) return false;
      h = (h + 1) & (uint32_t)ix.mask;
    }
  }
  if (ix.arm == kArmSorted) {
    const int32_t* l = reinterpret_cast<const int32_t*>(lds);
    int lo = 0, hi = ix.len;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (l[mid] < w) lo = mid + 1; else hi = mid;
    }
    return lo < ix.len && l[lo] == w;
  }
  return contains_sorted(ix.list, ix.len, w);
}

// ---------------------------------------------------------------- heavy path

// kEmit = false: count pass (writes cnt); true: write pass (emits triangles
// whose global index falls in [first, first + count)).
template <bool kEmit>
__global__ __launch_bounds__(kBlock) void k_heavy(Plan plan, const int32_t* __restrict__ counters,
                                                  const int2* __restrict__ items,
                                                  const int64_t* __restrict__ orow,
                                                  const int32_t* __restrict__ ocol,
                                                  const int64_t* __restrict__ irow,
                                                  const int32_t* __restrict__ icol,
                                                  const int32_t* __restrict__ ieid,
                                                  int32_t* __restrict__ cnt,
                                                  const int64_t* __restrict__ tri_off,
                                                  const int32_t* __restrict__ perm,
                                                  int64_t first, int64_t count,
                                                  int32_t* __restrict__ out) {
  __shared__ uint32_t lds[kIndexWords];
  const int32_t nitems = counters[kCItems];
  const int w_id = threadIdx.x / kWave;
  const int lane = lane_id();
  for (int64_t it = blockIdx.x; it < nitems; it += gridDim.x) {
    const int2 item = items[it];
    const int32_t b = item.x;
    const int64_t ob = orow[b];
    const int32_t db = (int32_t)(orow[b + 1] - ob);
    const int64_t ib = irow[b];
    const int32_t deg = db + (int32_t)(irow[b + 1] - ib);
    const int32_t j1 = min(deg, item.y + kItemSpan);
    const int cls = min(kHeavyClasses - 1, ceil_log2(db));
    const Index ix = build_index(ocol + ob, db, lds, plan.heavy_arm[cls]);
    for (int32_t j = item.y + w_id; j < j1; j += kWavesPerBlock) {
      int32_t y, e;
      if (j < db) { y = ocol[ob + j]; e = (int32_t)(ob + j); }
      else { y = icol[ib + (j - db)]; e = ieid[ib + (j - db)]; }
      const int64_t oy = orow[y];
      const int32_t dy = (int32_t)(orow[y + 1] - oy);
      const bool owned = dy < db || (dy == db && y < b);
      if (!owned) continue;
      if constexpr (!kEmit) {
        int32_t hits = 0;
        for (int32_t q = lane; q < dy; q += kWave) hits += index_has(ix, lds, ocol[oy + q]);
        hits = wave_sum(hits);
        if (lane == 0) cnt[e] = hits;
      } else {
        int64_t pos = tri_off[e];
        const int64_t end = tri_off[e + 1];
        if (end <= first || pos >= first + count || pos == end) continue;
        const int32_t pb = perm[b], py = perm[y];
        for (int32_t q0 = 0; q0 < dy; q0 += kWave) {
          const int32_t q = q0 + lane;
          const int32_t w = q < dy ? ocol[oy + q] : 0;
          const bool hit = q < dy && index_has(ix, lds, w);
          const uint64_t mask = ballot(hit);
          const int64_t at = pos + popc_below(mask);
          if (hit && at >= first && at < first + count) {
            int32_t t0 = pb, t1 = py, t2 = perm[w];
            sort3(t0, t1, t2);
            int32_t* o = out + 3 * (at - first);
            o[0] = t0; o[1] = t1; o[2] = t2;
          }
          pos += __popcll(mask);
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- light path

template <int G, bool kEmit>
__global__ __launch_bounds__(kBlock) void k_light(int bin, const int32_t* __restrict__ counters,
                                                  const int32_t* __restrict__ elist,
                                                  const int64_t* __restrict__ orow,
                                                  const int32_t* __restrict__ ocol,
                                                  const int32_t* __restrict__ otail,
                                                  int32_t* __restrict__ cnt,
                                                  const int64_t* __restrict__ tri_off,
                                                  const int32_t* __restrict__ perm,
                                                  int64_t first, int64_t count,
                                                  int32_t* __restrict__ out) {
  constexpr int kGroups = kBlock / G;
  int32_t base = 0;
  for (int q = 0; q < bin; ++q) base += counters[kCBinCount + q];
  const int32_t total = counters[kCBinCount + bin];
  const int gi = threadIdx.x / G, li = threadIdx.x % G;
  for (int64_t t = (int64_t)blockIdx.x * kGroups + gi; t < total;
       t += (int64_t)gridDim.x * kGroups) {
    const int32_t e = elist[base + t];
    const int32_t u = otail[e], v = ocol[e];
    const EdgeEnds x = edge_ends(orow, u, v);
    const int32_t* ps = ocol + orow[x.s];
    const int32_t* pb = ocol + orow[x.b];
    if constexpr (!kEmit) {
      int32_t hits = 0;
      for (int32_t q = li; q < x.c; q += G) hits += contains_sorted(pb, x.db, ps[q]);
      hits = group_sum<G>(hits);
      if (li == 0) cnt[e] = hits;
    } else {
      int64_t pos = tri_off[e];
      const int64_t end = tri_off[e + 1];
      if (end <= first || pos >= first + count || pos == end) continue;
      const int32_t pu = perm[u], pv = perm[v];
      for (int32_t q0 = 0; q0 < x.c; q0 += G) {
        const int32_t q = q0 + li;
        const int32_t w = q < x.c ? ps[q] : 0;
        const bool hit = q < x.c && contains_sorted(pb, x.db, w);
        const uint64_t mask = ballot(hit);
        const int64_t at = pos + popc_below_in_group<G>(mask);
        if (hit && at >= first && at < first + count) {
          int32_t t0 = pu, t1 = pv, t2 = perm[w];
          sort3(t0, t1, t2);
          int32_t* o = out + 3 * (at - first);
          o[0] = t0; o[1] = t1; o[2] = t2;
        }
        pos += __popcll(group_bits<G>(mask));
      }
    }
  }
}

template <bool kEmit>
hipError_t launch_light(int bin, int tile, const int32_t* counters, const int32_t* elist,
                        const int64_t* orow, const int32_t* ocol, const int32_t* otail,
                        int32_t* cnt, const int64_t* tri_off, const int32_t* perm,
                        int64_t first, int64_t count, int32_t* out, int64_t m, hipStream_t s) {
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(kGrid * 4, cdiv(m, kBlock / tile)));
#define L(G) k_light<G, kEmit><<<grid, kBlock, 0, s>>>(bin, counters, elist, orow, ocol, otail, \
                                                     cnt, tri_off, perm, first, count, out)
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

// The plain rule: lanes per edge about the bin's c; for heavy owners the
// bitmap (falling back to hash / sorted / global by size).
Plan plain_plan() {
  Plan p;
  for (int k = 0; k < kLightBins; ++k)
    p.light_tile[k] = k <= 2 ? 4 : k == 3 ? 8 : k == 4 ? 16 : k == 5 ? 32 : 64;
  for (int h = 0; h < kHeavyClasses; ++h) p.heavy_arm[h] = kArmBitmap;
  return p;
}

bool valid_tile(int t) { return t == 4 || t == 8 || t == 16 || t == 32 || t == 64; }

// Table codes: entry k < kLightBins is the light bin's tile << 8 (arm byte 0,
// binary search); entry 16 + h is heavy class h's arm.  Returns false on a
// code outside those sets.
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
    const int arm = d.table[16 + h];
    if (arm < 0 || arm >= kNumArms) return false;
    p->heavy_arm[h] = arm;
  }
  return true;
}

struct CountWs {
  int32_t* cnt;
  int32_t* elist;
  int2* items;
  int32_t* counters;
  unsigned long long* probes;
  void* scan_tmp;
};

int64_t max_items(int32_t n, int64_t m) { return (int64_t)n + cdiv(2 * m, kItemSpan) + 16; }

CountWs carve_count(Carve& c, int32_t n, int64_t m) {
  CountWs w;
  w.cnt = c.take<int32_t>(m);
  w.elist = c.take<int32_t>(m);
  w.items = c.take<int2>(max_items(n, m));
  w.counters = c.take<int32_t>(kCounters32);
  w.probes = c.take<unsigned long long>(4);
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

}  // namespace

size_t count_workspace_bytes(int32_t n, int64_t m) {
  Carve c(nullptr, 0);
  carve_count(c, n, m);
  return c.used;
}

int count_run(int32_t n, int64_t m, const int64_t* orow, const int32_t* ocol, const int32_t* otail,
              const int64_t* irow, const int32_t* icol, const int32_t* ieid,
              const DispatchView& d, int64_t* tri_off, void* ws, size_t ws_bytes,
              uint64_t* result, hipStream_t s, const char** err) {
  Carve c(ws, ws_bytes);
  CountWs w = carve_count(c, n, m);
  if (!c.ok()) {
    *err = "count workspace too small";
    return -4;
  }
  const int32_t heavy_min = d.heavy_min > 0 ? d.heavy_min : kDefaultHeavyMin;
  Plan plan;
  if (!plan_from(d, &plan)) {
    *err = "dispatch table holds an unknown arm or tile code";
    return -6;
  }
  AOT_TRY(fill_i32(w.counters, kCounters32, 0, s));
  AOT_TRY(fill_i64(reinterpret_cast<int64_t*>(w.probes), 4, 0, s));
  if (m > 0) {
    const unsigned ge = (unsigned)std::min<int64_t>(kGrid * 4, cdiv(m, kBlock));
    k_bin_count<<<ge, kBlock, 0, s>>>(m, orow, ocol, otail, heavy_min, w.cnt, w.counters, w.probes);
    AOT_TRY(hipGetLastError());
    k_bin_scatter<<<ge, kBlock, 0, s>>>(m, orow, ocol, otail, heavy_min, w.counters, w.elist);
    AOT_TRY(hipGetLastError());
    const unsigned gv = (unsigned)std::max<int64_t>(1, std::min<int64_t>(kGrid * 4, cdiv(n, kBlock)));
    k_make_items<<<gv, kBlock, 0, s>>>(n, orow, irow, heavy_min, w.counters, w.items);
    AOT_TRY(hipGetLastError());
    for (int bin = 0; bin < kLightBins; ++bin)
      AOT_TRY(launch_light<false>(bin, plan.light_tile[bin], w.counters, w.elist, orow, ocol,
                                  otail, w.cnt, nullptr, nullptr, 0, 0, nullptr, m, s));
    k_heavy<false><<<kGrid, kBlock, 0, s>>>(plan, w.counters, w.items, orow, ocol, irow, icol,
                                             ieid, w.cnt, nullptr, nullptr, 0, 0, nullptr);
    AOT_TRY(hipGetLastError());
  }
  AOT_TRY(exclusive_scan(w.cnt, tri_off, m, w.scan_tmp, s));
  int64_t t = 0;
  unsigned long long pr = 0;
  AOT_TRY(hipMemcpyAsync(&t, tri_off + m, sizeof(t), hipMemcpyDeviceToHost, s));
  AOT_TRY(hipMemcpyAsync(&pr, w.probes, sizeof(pr), hipMemcpyDeviceToHost, s));
  AOT_TRY(hipStreamSynchronize(s));
  result[0] = (uint64_t)t;
  result[1] = (uint64_t)pr;
  return 0;
}

int list_run(int32_t n, int64_t m, const int64_t* orow, const int32_t* ocol, const int32_t* otail,
             const int32_t* perm, const int64_t* irow, const int32_t* icol, const int32_t* ieid,
             const DispatchView& d, const int64_t* tri_off, void* ws, size_t ws_bytes,
             int64_t first, int64_t count, int32_t* out, hipStream_t s, const char** err) {
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
  if (m == 0 || count <= 0) return 0;
  for (int bin = 0; bin < kLightBins; ++bin)
    AOT_TRY(launch_light<true>(bin, plan.light_tile[bin], w.counters, w.elist, orow, ocol, otail,
                               nullptr, tri_off, perm, first, count, out, m, s));
  k_heavy<true><<<kGrid, kBlock, 0, s>>>(plan, w.counters, w.items, orow, ocol, irow, icol, ieid,
                                          nullptr, tri_off, perm, first, count, out);
  AOT_TRY(hipGetLastError());
  return 0;
}

}  // namespace aot
