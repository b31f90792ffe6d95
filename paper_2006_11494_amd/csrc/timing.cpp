// Per-launch timing recorder of the probe passes (one record per bucket
// launch): the data the cost model of the dispatch is trained on, and the
// live launch times the benchmark's roofline uses.  Thread-local: a thread
// records only its own calls.
#include <vector>

#include "aot.h"
#include "kernels.hpp"

namespace aot {

namespace {

struct Rec {
  aot_timing t;
  hipEvent_t a = nullptr, b = nullptr;
};

struct Recorder {
  bool on = false;
  std::vector<Rec> recs;
};

thread_local Recorder g_rec;

void drop_events() {
  for (Rec& r : g_rec.recs) {
    if (r.a) (void)hipEventDestroy(r.a);
    if (r.b) (void)hipEventDestroy(r.b);
  }
  g_rec.recs.clear();
}

}  // namespace

int timing_begin(int pass, int bucket, int arm, int tile, int64_t edges, int64_t probes,
                 int64_t staged, int64_t triangles, hipStream_t s) {
  if (!g_rec.on) return -1;
  Rec r;
  r.t.pass = pass;
  r.t.bucket = bucket;
  r.t.arm = arm;
  r.t.tile = tile;
  r.t.edges = edges;
  r.t.probes = probes;
  r.t.staged = staged;
  r.t.triangles = pass == 0 ? -1 : triangles;
  r.t.lookups = probes;             // heavy count launches: filled in after the pass
  r.t.ms = 0.0;
  if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess ||
      hipEventRecord(r.a, s) != hipSuccess) {
    if (r.a) (void)hipEventDestroy(r.a);
    if (r.b) (void)hipEventDestroy(r.b);
    return -1;
  }
  g_rec.recs.push_back(r);
  return (int)g_rec.recs.size() - 1;
}

void timing_end(int rec, hipStream_t s) {
  if (rec < 0 || rec >= (int)g_rec.recs.size()) return;
  (void)hipEventRecord(g_rec.recs[rec].b, s);
}

void timing_fill_count(const int64_t* stats, int stride, int tri_offset, int look_offset,
                       int heavy_base) {
  for (Rec& r : g_rec.recs) {
    if (r.t.pass != 0 || r.t.triangles >= 0) continue;
    r.t.triangles = stats[r.t.bucket * stride + tri_offset];
    if (r.t.bucket >= heavy_base) r.t.lookups = stats[r.t.bucket * stride + look_offset];
  }
}

}  // namespace aot

extern "C" {

int aot_timing_start(void) {
  aot::drop_events();
  aot::g_rec.on = true;
  return AOT_OK;
}

int aot_timing_stop(aot_timing* out, int32_t cap, int32_t* count) {
  if (cap < 0 || (cap > 0 && !out)) return AOT_E_ARG;
  aot::g_rec.on = false;
  int rc = AOT_OK;
  int32_t k = 0;
  for (aot::Rec& r : aot::g_rec.recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
      rc = AOT_E_HIP;
    r.t.ms = ms;
    if (k < cap) out[k] = r.t;
    ++k;
  }
  if (count) *count = k;
  if (k > cap && rc == AOT_OK) rc = AOT_E_CAPACITY;
  aot::drop_events();
  return rc;
}

}  // extern "C"
