// The C ABI (include/aot.h): argument checks, workspace sizing, status codes.
#include <climits>
#include <cstring>
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
  v->given = true;
  v->heavy_min = d->heavy_min;
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

}  // namespace

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

int aot_version(void) { return 1; }

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
  if (flags & ~AOT_VALIDATE) return fail(AOT_E_ARG, "unknown flag");
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
  rc = aot::orient_run(g->n, g->nnz, g->rowptr, g->col, (flags & AOT_VALIDATE) != 0, out->rowptr,
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

}  // extern "C"
