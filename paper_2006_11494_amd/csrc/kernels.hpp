// Internal interface between the C ABI (abi.cpp) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "aot.h"
#include "common.hpp"

namespace aot {

inline int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }
inline int64_t cdiv(int64_t x, int64_t a) { return (x + a - 1) / a; }

// Carves aligned sub-buffers out of one workspace allocation.
struct Carve {
  char* base;
  size_t used = 0;
  size_t cap;
  Carve(void* p, size_t c) : base(static_cast<char*>(p)), cap(c) {}
  template <typename T>
  T* take(int64_t count) {
    size_t bytes = (size_t)align_up((int64_t)(sizeof(T) * (size_t)(count > 0 ? count : 1)), 256);
    T* p = reinterpret_cast<T*>(base ? base + used : nullptr);
    used += bytes;
    return p;
  }
  bool ok() const { return used <= cap; }
};

// ---- fill.hip
hipError_t fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t s);

// ---- scan.hip: out[0..n] = exclusive prefix sums of in[0..n), out[n] = total.
size_t scan_workspace(int64_t n);
hipError_t exclusive_scan(const int32_t* in, int64_t* out, int64_t n, void* tmp, hipStream_t s);
hipError_t exclusive_scan(const int64_t* in, int64_t* out, int64_t n, void* tmp, hipStream_t s);

// ---- radix.hip: stable LSD sort of (key, value) pairs by the low `bits` bits
// of non-negative int32 keys.  Result lands in (keys_out, vals_out); the
// other pair of buffers is clobbered.
size_t radix_workspace(int64_t n);
hipError_t radix_sort_pairs(int32_t* keys, int32_t* vals, int32_t* keys_alt, int32_t* vals_alt,
                            int64_t n, int bits, void* tmp, hipStream_t s,
                            int32_t** keys_out, int32_t** vals_out);

// ---- orient.hip
size_t orient_workspace_bytes(int32_t n, int64_t nnz);
// One graph.  in_by_rank: sort each in-list by label; core: rank by the core
// order instead of degree; by_id: keep original ids as labels (the order
// still directs the edges; perm and rank come out as the identity).
int orient_run(int32_t n, int64_t nnz, const int64_t* rowptr, const int32_t* col, bool validate,
               bool in_by_rank, bool core, bool by_id, int64_t* orow, int32_t* ocol, int32_t* otail,
               int32_t* perm,
               int32_t* rank, int64_t* irow, int32_t* icol, void* ws, size_t ws_bytes,
               hipStream_t s, const char** err);
// Orientation of a batch held as one block-diagonal CSR (graph g owns
// vertices [voff[g], voff[g+1])): ranks go graph by graph, (degree, id)
// inside a graph; every launch is sized from n and nnz only (no host reads).
// dbits / gbits: key bits of a degree / of a graph index.
int orient_batch_run(int32_t n, int64_t nnz, const int64_t* rowptr, const int32_t* col,
                     const int64_t* voff, int32_t count, int dbits, int gbits, int64_t* orow,
                     int32_t* ocol, int32_t* otail, int32_t* perm, int32_t* rank, int64_t* irow,
                     int32_t* icol, void* ws, size_t ws_bytes, hipStream_t s, const char** err);

// ---- timing.cpp: the per-launch recorder of the probe passes.  A record is
// opened just before a bucket's kernel launch and closed right after it,
// with HIP events on the launch stream; disabled, both calls do nothing.
constexpr int kNumBuckets = 32;
int timing_begin(int pass, int bucket, int arm, int tile, int64_t edges, int64_t probes,
                 int64_t staged, int64_t triangles, hipStream_t s);
void timing_end(int rec, hipStream_t s);
// Fills the triangle totals of the count-pass records still missing them,
// and the look-ups the heavy ones made.
void timing_fill_count(const int64_t* stats, int stride, int tri_offset, int look_offset,
                       int heavy_base);

// ---- count.hip
size_t count_workspace_bytes(int32_t n, int64_t m);
struct DispatchView {
  bool given = false;              // a dispatch was passed (else: the stored plan / plain rule)
  int32_t heavy_min = 0;
  int32_t strategy = 0;            // AOT_STRATEGY_*
  const int32_t* table = nullptr;  // host, kNumBuckets codes or nullptr
  const aot_mlp* model = nullptr;  // learned dispatch
};
// Cost-model forward (mlp.hip).
int mlp_predict(const aot_mlp* net, const float* x_dev, int32_t batch, float* y_dev, hipStream_t s);
// The plan and bucket features of the last count on a workspace (count.hip).
int count_plan(const void* ws, size_t ws_bytes, int32_t n, int64_t m, int32_t* table,
               int32_t* learned);
int count_features(const void* ws, size_t ws_bytes, int32_t n, int64_t m, float* features,
                   uint8_t* present);
int count_run(int32_t n, int64_t m, const int64_t* orow, const int32_t* ocol, const int32_t* otail,
              const int64_t* irow, const int32_t* icol, const DispatchView& d, int64_t* tri_off, void* ws, size_t ws_bytes,
              uint64_t* result, hipStream_t s, const char** err);
int list_run(int32_t n, int64_t m, const int64_t* orow, const int32_t* ocol, const int32_t* otail,
             const int32_t* perm, const int64_t* irow, const int32_t* icol, const DispatchView& d, const int64_t* tri_off, void* ws, size_t ws_bytes,
             int64_t first, int64_t count, int32_t* out, hipStream_t s, const char** err);

// Schedule of the persistent probe passes (the autotuner's choices).
struct DrainSchedule {
  int32_t heavy_min = 0;             // 0 = library default
  bool table_given = false;
  int32_t table[kNumBuckets] = {0};  // codes as in aot_dispatch's table
  int32_t rounds = 0;                // group-rounds per light task, 0 = default
  int64_t max_span = 0;              // bound on an out-list's id span, 0 = unknown
};
int drain_run(int32_t n, int64_t m, const int64_t* orow, const int32_t* ocol,
              const int32_t* otail, const int32_t* perm, const int64_t* irow,
              const int32_t* icol, const DrainSchedule& sc, int64_t* tri_off, void* ws,
              size_t ws_bytes, int64_t first, int64_t count, int32_t* out, hipStream_t s,
              const char** err);
int batch_totals(int32_t count, const int64_t* voff, const int64_t* orow, const int64_t* tri_off,
                 int64_t* gtri, hipStream_t s);

// The write pass in digest mode: nothing stored; digest = {T, hash sum, hash
// xor} (host), vcount (device, optional) = triangles per original vertex id.
int digest_run(int32_t n, int64_t m, const int64_t* orow, const int32_t* ocol,
               const int32_t* otail, const int32_t* perm, const int64_t* irow,
               const int32_t* icol, const DispatchView& d, const int64_t* tri_off, void* ws,
               size_t ws_bytes, uint64_t* vcount, uint64_t* digest, hipStream_t s,
               const char** err);
// The digest pass with per-edge support (and optional vertex counts / digest).
int support_run(int32_t n, int64_t m, const int64_t* orow, const int32_t* ocol,
                const int32_t* otail, const int32_t* perm, const int64_t* irow,
                const int32_t* icol, const DispatchView& d, const int64_t* tri_off, void* ws,
                size_t ws_bytes, uint32_t* esup, uint64_t* vcount, uint64_t* digest,
                hipStream_t s, const char** err);

}  // namespace aot
