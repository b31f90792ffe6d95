// The C ABI (include/aot.h): argument checks, workspace sizing, status codes.
#include <algorithm>
#include <climits>
#include <cstring>
#include <mutex>
#include <string>

#include "aot.h"
#include "kernels.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int ok() {
  g_err.clear();
  return AOT_OK;
}

int check_graph_sizes(int32_t n, int64_t nnz) {
  if (n < 0) return fail(AOT_E_ARG, "n < 0");
  if (nnz < 0) return fail(AOT_E_ARG, "nnz < 0");
  if (nnz % 2) return fail(AOT_E_GRAPH, "nnz is odd, so the CSR cannot be symmetric");
  if (nnz / 2 > INT32_MAX) return fail(AOT_E_OVERFLOW, "m = nnz/2 exceeds INT32_MAX edge ids");
  return AOT_OK;
}

int check_oriented(const aot_oriented* g) {
  if (!g) return fail(AOT_E_ARG, "oriented graph is NULL");
  if (g->n < 0 || g->m < 0) return fail(AOT_E_ARG, "negative n or m");
  if (g->m > INT32_MAX) return fail(AOT_E_OVERFLOW, "m exceeds INT32_MAX edge ids");
  if (!g->rowptr || !g->in_rowptr) return fail(AOT_E_ARG, "rowptr / in_rowptr is NULL");
  if (g->m > 0 && (!g->col || !g->tail || !g->in_col))
    return fail(AOT_E_ARG, "an edge array of the oriented graph is NULL");
  if (g->n > 0 && (!g->perm || !g->rank)) return fail(AOT_E_ARG, "perm / rank is NULL");
  return AOT_OK;
}

int check_dispatch(const aot_dispatch* d, aot::DispatchView* v) {
  *v = aot::DispatchView();
  if (!d) return AOT_OK;
  if (d->mode != AOT_DISPATCH_PLAIN && d->mode != AOT_DISPATCH_TABLE &&
      d->mode != AOT_DISPATCH_LEARNED)
    return fail(AOT_E_ARG, "unknown dispatch mode");
  if (d->heavy_min < 0) return fail(AOT_E_ARG, "heavy_min < 0");
  if (d->strategy < AOT_STRATEGY_ADAPTIVE || d->strategy > AOT_STRATEGY_PER_EDGE)
    return fail(AOT_E_ARG, "unknown strategy");
  if (d->strategy != AOT_STRATEGY_ADAPTIVE && d->mode == AOT_DISPATCH_LEARNED)
    return fail(AOT_E_ARG, "the cost model chooses for the adaptive strategy only");
  v->given = true;
  v->heavy_min = d->heavy_min;
  v->strategy = d->strategy;
  if (d->mode == AOT_DISPATCH_TABLE) {
    if (!d->table) return fail(AOT_E_MODEL, "table dispatch without a table");
    v->table = d->table;
  }
  if (d->mode == AOT_DISPATCH_LEARNED) v->model = d->model;   // checked (and fallen back) later
  return AOT_OK;
}

int hip_status(int rc, const char* err) {
  if (rc == 0) return ok();
  switch (rc) {
    case -2: return fail(AOT_E_GRAPH, err ? err : "malformed graph");
    case -4: return fail(AOT_E_WORKSPACE, err ? err : "workspace too small");
    case -6: return fail(AOT_E_MODEL, err ? err : "invalid dispatch table");
    default: return fail(AOT_E_HIP, err ? err : "HIP error");
  }
}

// A batch's offsets and the bits its (graph, degree) sort key needs.
int check_batch(const aot_batch* b, int* dbits, int* gbits, int64_t* max_n) {
  if (!b) return fail(AOT_E_ARG, "batch is NULL");
  if (b->count < 1) return fail(AOT_E_ARG, "batch count < 1");
  if (!b->voff_host || !b->voff) return fail(AOT_E_ARG, "batch offsets are NULL");
  int rc = check_graph_sizes(b->arena.n, b->arena.nnz);
  if (rc) return rc;
  if (!b->arena.rowptr) return fail(AOT_E_ARG, "arena rowptr is NULL");
  if (b->arena.nnz > 0 && !b->arena.col) return fail(AOT_E_ARG, "arena col is NULL");
  const int64_t* v = b->voff_host;
  if (v[0] != 0 || v[b->count] != b->arena.n)
    return fail(AOT_E_ARG, "voff[0] must be 0 and voff[count] the arena's n");
  int64_t mx = 0;
  for (int32_t g = 0; g < b->count; ++g) {
    if (v[g + 1] < v[g]) return fail(AOT_E_ARG, "voff is decreasing");
    mx = std::max<int64_t>(mx, v[g + 1] - v[g]);
  }
  *max_n = mx;
  *dbits = aot::ceil_log2(mx);
  *gbits = aot::ceil_log2((int64_t)b->count);
  if (*dbits + *gbits > 31)
    return fail(AOT_E_OVERFLOW, "(graph, degree) sort key needs more than 31 bits");
  return AOT_OK;
}

size_t batch_ws_bytes(int32_t n, int64_t nnz) {
  // orientation scratch and count workspace alias: the first is dead before
  // the second is first written (same stream)
  return std::max(aot::orient_workspace_bytes(n, nnz), aot::count_workspace_bytes(n, nnz / 2));
}

int batch_enqueue(const aot_batch* b, const aot_schedule* sc, aot_oriented* out, int64_t* tri_off,
                  int64_t* graph_tri, int32_t* tri, int64_t cap, void* ws, size_t ws_bytes,
                  hipStream_t s) {
  int dbits = 0, gbits = 0;
  int64_t max_n = 0;
  int rc = check_batch(b, &dbits, &gbits, &max_n);
  if (rc) return rc;
  const int32_t n = b->arena.n;
  const int64_t m = b->arena.nnz / 2;
  if (!out || !tri_off || !graph_tri) return fail(AOT_E_ARG, "output is NULL");
  if (!out->rowptr || !out->in_rowptr) return fail(AOT_E_ARG, "output rowptr is NULL");
  if (n > 0 && (!out->perm || !out->rank)) return fail(AOT_E_ARG, "output perm/rank is NULL");
  if (m > 0 && (!out->col || !out->tail || !out->in_col))
    return fail(AOT_E_ARG, "an output edge array is NULL");
  if (cap < 0) return fail(AOT_E_ARG, "cap < 0");
  if (cap > 0 && !tri) return fail(AOT_E_ARG, "tri is NULL");
  if (cap > INT64_MAX / 3) return fail(AOT_E_CAPACITY, "cap too large");
  aot::DrainSchedule ds;
  if (sc) {
    if (sc->heavy_min < 0 || sc->light_rounds < 0) return fail(AOT_E_ARG, "negative schedule entry");
    if (sc->light_rounds > 1024) return fail(AOT_E_ARG, "light_rounds > 1024");
    ds.heavy_min = sc->heavy_min;
    ds.rounds = sc->light_rounds;
    ds.table_given = sc->use_table != 0;
    for (int k = 0; k < AOT_NUM_BUCKETS; ++k) ds.table[k] = sc->table[k];
  }
  ds.max_span = max_n;
  if (ws_bytes < batch_ws_bytes(n, b->arena.nnz) || !ws)
    return fail(AOT_E_WORKSPACE, "workspace smaller than aot_batch_workspace()");
  out->n = n;
  out->m = m;
  const char* err = nullptr;
  rc = aot::orient_batch_run(n, b->arena.nnz, b->arena.rowptr, b->arena.col, b->voff, b->count,
                             dbits, gbits, out->rowptr, out->col, out->tail, out->perm,
                             out->rank, out->in_rowptr, out->in_col, ws, ws_bytes, s, &err);
  if (rc) return hip_status(rc, err);
  rc = aot::drain_run(n, m, out->rowptr, out->col, out->tail, out->perm, out->in_rowptr,
                      out->in_col, ds, tri_off, ws, ws_bytes, 0, cap, tri, s, &err);
  if (rc) return hip_status(rc, err);
  if (aot::batch_totals(b->count, b->voff, out->rowptr, tri_off, graph_tri, s))
    return fail(AOT_E_HIP, "batch totals launch failed");
  return ok();
}

// Fixed scratch of aot_count_noalloc: the count workspace of callers that
// cannot allocate device memory.  Each device holds its own copy from the
// time the library's code object is loaded there until the process ends.
// The array's name is a host-side stand-in; kernels get the device address
// that hipGetSymbolAddress returns, looked up once per device.
__device__ __align__(256) unsigned char scratch[AOT_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxScratchDevices] = {};

int scratch_of_current_device(void** ptr) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(AOT_E_HIP, "hipGetDevice failed");
  if (dev < 0 || dev >= kMaxScratchDevices)
    return fail(AOT_E_ARG, "device index beyond the fixed scratch table (64 devices)");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
      return fail(AOT_E_HIP, "hipGetSymbolAddress of the fixed scratch failed");
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return AOT_OK;
}

}  // namespace

struct aot_batch_graph {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

extern "C" {

const char* aot_status_str(int status) {
  switch (status) {
    case AOT_OK: return "ok";
    case AOT_E_ARG: return "invalid argument";
    case AOT_E_GRAPH: return "malformed graph";
    case AOT_E_OVERFLOW: return "size overflow";
    case AOT_E_WORKSPACE: return "workspace too small";
    case AOT_E_HIP: return "HIP runtime error";
    case AOT_E_MODEL: return "cost model missing or invalid";
    case AOT_E_CAPACITY: return "output capacity too small";
    default: return "unknown status";
  }
}

const char* aot_last_error(void) { return g_err.c_str(); }

int aot_version(void) { return 3; }

int aot_orient_workspace(int32_t n, int64_t nnz, size_t* bytes) {
  if (!bytes) return fail(AOT_E_ARG, "bytes is NULL");
  int rc = check_graph_sizes(n, nnz);
  if (rc) return rc;
  *bytes = aot::orient_workspace_bytes(n, nnz);
  return ok();
}

int aot_orient(const aot_graph* g, uint32_t flags, aot_oriented* out, void* ws, size_t ws_bytes,
               void* stream) {
  if (!g || !out) return fail(AOT_E_ARG, "graph or output is NULL");
  if (flags & ~(AOT_VALIDATE | AOT_IN_LISTS_BY_RANK | AOT_ORDER_CORE | AOT_LOCAL_BY_ID))
    return fail(AOT_E_ARG, "unknown flag");
  int rc = check_graph_sizes(g->n, g->nnz);
  if (rc) return rc;
  if (!g->rowptr) return fail(AOT_E_ARG, "rowptr is NULL");
  if (g->nnz > 0 && !g->col) return fail(AOT_E_ARG, "col is NULL");
  const int64_t m = g->nnz / 2;
  if (!out->rowptr || !out->in_rowptr) return fail(AOT_E_ARG, "output rowptr is NULL");
  if (g->n > 0 && (!out->perm || !out->rank)) return fail(AOT_E_ARG, "output perm/rank is NULL");
  if (m > 0 && (!out->col || !out->tail || !out->in_col))
    return fail(AOT_E_ARG, "an output edge array is NULL");
  const size_t need = aot::orient_workspace_bytes(g->n, g->nnz);
  if (ws_bytes < need || (!ws && need > 0))
    return fail(AOT_E_WORKSPACE, "orientation workspace smaller than aot_orient_workspace()");
  out->n = g->n;
  out->m = m;
  const char* err = nullptr;
  rc = aot::orient_run(g->n, g->nnz, g->rowptr, g->col, (flags & AOT_VALIDATE) != 0,
                       (flags & AOT_IN_LISTS_BY_RANK) != 0, (flags & AOT_ORDER_CORE) != 0,
                       (flags & AOT_LOCAL_BY_ID) != 0, out->rowptr,
                       out->col, out->tail, out->perm, out->rank, out->in_rowptr, out->in_col,
                       ws, ws_bytes, static_cast<hipStream_t>(stream), &err);
  return hip_status(rc, err);
}

int aot_count_workspace(int32_t n, int64_t m, size_t* bytes) {
  if (!bytes) return fail(AOT_E_ARG, "bytes is NULL");
  if (n < 0 || m < 0) return fail(AOT_E_ARG, "negative n or m");
  if (m > INT32_MAX) return fail(AOT_E_OVERFLOW, "m exceeds INT32_MAX edge ids");
  *bytes = aot::count_workspace_bytes(n, m);
  return ok();
}

int aot_count(const aot_oriented* g, const aot_dispatch* d, int64_t* tri_off, void* ws,
              size_t ws_bytes, uint64_t* result, void* stream) {
  int rc = check_oriented(g);
  if (rc) return rc;
  if (!tri_off || !result) return fail(AOT_E_ARG, "tri_off or result is NULL");
  aot::DispatchView dv;
  rc = check_dispatch(d, &dv);
  if (rc) return rc;
  const size_t need = aot::count_workspace_bytes(g->n, g->m);
  if (ws_bytes < need || !ws) return fail(AOT_E_WORKSPACE, "count workspace smaller than aot_count_workspace()");
  const char* err = nullptr;
  rc = aot::count_run(g->n, g->m, g->rowptr, g->col, g->tail, g->in_rowptr, g->in_col, dv,
                      tri_off, ws, ws_bytes, result, static_cast<hipStream_t>(stream), &err);
  return hip_status(rc, err);
}

int aot_count_noalloc(const aot_oriented* g, const aot_dispatch* d, int64_t* tri_off,
                      uint64_t* result, void* stream) {
  int rc = check_oriented(g);
  if (rc) return rc;
  if (!tri_off || !result) return fail(AOT_E_ARG, "tri_off or result is NULL");
  aot::DispatchView dv;
  rc = check_dispatch(d, &dv);
  if (rc) return rc;
  const size_t need = aot::count_workspace_bytes(g->n, g->m);
  if (need > (size_t)AOT_NOALLOC_SCRATCH_BYTES)
    return fail(AOT_E_CAPACITY, "graph too large for the fixed scratch of aot_count_noalloc: needs " +
                                    std::to_string(need) + " bytes, the scratch holds " +
                                    std::to_string((size_t)AOT_NOALLOC_SCRATCH_BYTES));
  void* ws = nullptr;
  rc = scratch_of_current_device(&ws);
  if (rc) return rc;
  const char* err = nullptr;
  rc = aot::count_run(g->n, g->m, g->rowptr, g->col, g->tail, g->in_rowptr, g->in_col, dv,
                      tri_off, ws, (size_t)AOT_NOALLOC_SCRATCH_BYTES, result,
                      static_cast<hipStream_t>(stream), &err);
  return hip_status(rc, err);
}

int aot_list(const aot_oriented* g, const aot_dispatch* d, const int64_t* tri_off, void* ws,
             size_t ws_bytes, int64_t first, int64_t count, int32_t* out, int64_t* written,
             void* stream) {
  int rc = check_oriented(g);
  if (rc) return rc;
  if (!tri_off) return fail(AOT_E_ARG, "tri_off is NULL");
  if (first < 0 || count < 0) return fail(AOT_E_ARG, "negative window");
  if (count > 0 && !out) return fail(AOT_E_ARG, "out is NULL");
  if (count > INT64_MAX / 3) return fail(AOT_E_CAPACITY, "window too large");
  aot::DispatchView dv;
  rc = check_dispatch(d, &dv);
  if (rc) return rc;
  const size_t need = aot::count_workspace_bytes(g->n, g->m);
  if (ws_bytes < need || !ws) return fail(AOT_E_WORKSPACE, "count workspace smaller than aot_count_workspace()");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const char* err = nullptr;
  rc = aot::list_run(g->n, g->m, g->rowptr, g->col, g->tail, g->perm, g->in_rowptr, g->in_col,
                     dv, tri_off, ws, ws_bytes, first, count, out, s, &err);
  if (rc) return hip_status(rc, err);
  if (written) {
    int64_t t = 0;
    if (hipMemcpyAsync(&t, tri_off + g->m, sizeof(t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(AOT_E_HIP, "reading the triangle count back failed");
    int64_t w = t - first;
    *written = w < 0 ? 0 : (w > count ? count : w);
  }
  return ok();
}

int aot_digest(const aot_oriented* g, const aot_dispatch* d, const int64_t* tri_off, void* ws,
               size_t ws_bytes, uint64_t* vertex_counts, uint64_t* digest, void* stream) {
  int rc = check_oriented(g);
  if (rc) return rc;
  if (!tri_off || !digest) return fail(AOT_E_ARG, "tri_off or digest is NULL");
  aot::DispatchView dv;
  rc = check_dispatch(d, &dv);
  if (rc) return rc;
  const size_t need = aot::count_workspace_bytes(g->n, g->m);
  if (ws_bytes < need || !ws) return fail(AOT_E_WORKSPACE, "count workspace smaller than aot_count_workspace()");
  const char* err = nullptr;
  rc = aot::digest_run(g->n, g->m, g->rowptr, g->col, g->tail, g->perm, g->in_rowptr, g->in_col,
                       dv, tri_off, ws, ws_bytes, vertex_counts, digest,
                       static_cast<hipStream_t>(stream), &err);
  return hip_status(rc, err);
}

int aot_support(const aot_oriented* g, const aot_dispatch* d, const int64_t* tri_off, void* ws,
                size_t ws_bytes, uint32_t* edge_support, uint64_t* vertex_counts,
                uint64_t* digest, void* stream) {
  int rc = check_oriented(g);
  if (rc) return rc;
  if (!tri_off) return fail(AOT_E_ARG, "tri_off is NULL");
  if (g->m > 0 && !edge_support) return fail(AOT_E_ARG, "edge_support is NULL");
  aot::DispatchView dv;
  rc = check_dispatch(d, &dv);
  if (rc) return rc;
  const size_t need = aot::count_workspace_bytes(g->n, g->m);
  if (ws_bytes < need || !ws) return fail(AOT_E_WORKSPACE, "count workspace smaller than aot_count_workspace()");
  const char* err = nullptr;
  rc = aot::support_run(g->n, g->m, g->rowptr, g->col, g->tail, g->perm, g->in_rowptr, g->in_col,
                        dv, tri_off, ws, ws_bytes, edge_support, vertex_counts, digest,
                        static_cast<hipStream_t>(stream), &err);
  return hip_status(rc, err);
}

int aot_count_plan(const void* ws, size_t ws_bytes, int32_t n, int64_t m, int32_t* table,
                   int32_t* learned) {
  if (!ws || !table || !learned || n < 0 || m < 0) return fail(AOT_E_ARG, "bad argument");
  if (ws_bytes < aot::count_workspace_bytes(n, m)) return fail(AOT_E_WORKSPACE, "workspace too small");
  return aot::count_plan(ws, ws_bytes, n, m, table, learned) ? fail(AOT_E_HIP, "copy failed") : ok();
}

int aot_bucket_features(const void* ws, size_t ws_bytes, int32_t n, int64_t m, float* features,
                        uint8_t* present) {
  if (!ws || !features || !present || n < 0 || m < 0) return fail(AOT_E_ARG, "bad argument");
  if (ws_bytes < aot::count_workspace_bytes(n, m)) return fail(AOT_E_WORKSPACE, "workspace too small");
  return aot::count_features(ws, ws_bytes, n, m, features, present) ? fail(AOT_E_HIP, "copy failed")
                                                                     : ok();
}

int aot_batch_workspace(const aot_batch* b, size_t* bytes) {
  if (!bytes) return fail(AOT_E_ARG, "bytes is NULL");
  int dbits = 0, gbits = 0;
  int64_t max_n = 0;
  int rc = check_batch(b, &dbits, &gbits, &max_n);
  if (rc) return rc;
  *bytes = batch_ws_bytes(b->arena.n, b->arena.nnz);
  return ok();
}

int aot_batch_run(const aot_batch* b, const aot_schedule* sc, aot_oriented* out,
                  int64_t* tri_off, int64_t* graph_tri, int32_t* tri, int64_t cap, void* ws,
                  size_t ws_bytes, void* stream) {
  return batch_enqueue(b, sc, out, tri_off, graph_tri, tri, cap, ws, ws_bytes,
                       static_cast<hipStream_t>(stream));
}

int aot_batch_capture(const aot_batch* b, const aot_schedule* sc, aot_oriented* out,
                      int64_t* tri_off, int64_t* graph_tri, int32_t* tri, int64_t cap, void* ws,
                      size_t ws_bytes, aot_batch_graph** graph) {
  if (!graph) return fail(AOT_E_ARG, "graph is NULL");
  *graph = nullptr;
  int dbits = 0, gbits = 0;
  int64_t max_n = 0;
  int rc = check_batch(b, &dbits, &gbits, &max_n);   // fail before opening a capture
  if (rc) return rc;
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
    return fail(AOT_E_HIP, "stream creation failed");
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess) {
    hipStreamDestroy(cs);
    return fail(AOT_E_HIP, "hipStreamBeginCapture failed");
  }
  rc = batch_enqueue(b, sc, out, tri_off, graph_tri, tri, cap, ws, ws_bytes, cs);
  const std::string detail = g_err;
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(cs, &g);
  hipStreamDestroy(cs);
  if (rc) {
    if (g) hipGraphDestroy(g);
    return fail(rc, detail);
  }
  if (e != hipSuccess || !g) return fail(AOT_E_HIP, "stream capture failed");
  hipGraphExec_t x = nullptr;
  if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
    hipGraphDestroy(g);
    return fail(AOT_E_HIP, "hipGraphInstantiate failed");
  }
  *graph = new aot_batch_graph{g, x};
  return ok();
}

int aot_batch_launch(const aot_batch_graph* graph, void* stream) {
  if (!graph) return fail(AOT_E_ARG, "graph is NULL");
  if (hipGraphLaunch(graph->exec, static_cast<hipStream_t>(stream)) != hipSuccess)
    return fail(AOT_E_HIP, "hipGraphLaunch failed");
  return ok();
}

int aot_batch_destroy(aot_batch_graph* graph) {
  if (!graph) return ok();
  hipGraphExecDestroy(graph->exec);
  hipGraphDestroy(graph->graph);
  delete graph;
  return ok();
}

}  // extern "C"
