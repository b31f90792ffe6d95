/*
 * aot.h -- C ABI of the MI355X (gfx950) AOT triangle-listing library.
 *
 * AOT is the adaptive-orientation edge-iterator of Yu, Qin, Zhang, Zhang and
 * Lin, "AOT: Pushing the Efficiency Boundary of Main-memory Triangle Listing"
 * (2020).  Given an undirected simple graph it lists every triangle exactly
 * once (Section 2.1, problem statement) in
 *     Theta( sum over directed edges <u,v> of min(deg+(u), deg+(v)) )
 * look-ups (Section 3.2, Time Complexity).
 *
 * Three stages, each one entry point:
 *   aot_orient  orientation (Section 2.2, "Orientation technique"; first step
 *               of Algorithm 3): rank vertices by (degree, id) ascending and
 *               keep each edge pointing up the order; out-lists sorted.
 *   aot_count   adaptive orientation (Section 3.1, "The main idea"; Algorithm
 *               3's two probe loops): every directed edge is charged to its
 *               endpoint with the larger (deg+, id) -- the owner -- and the
 *               other endpoint's out-list is probed into an index of the
 *               owner's out-list.  Produces the per-edge triangle offsets, the
 *               triangle count T and the probe count (sum of minima).
 *   aot_list    emits the triangles (Algorithm 3, "output triangle"), any
 *               window of the global list at a time.
 *
 * Conventions shared by every call
 *   - Pointers marked "device" are HIP device (or managed) memory on the
 *     current device; "host" pointers are ordinary host memory.
 *   - The caller owns every buffer; the library allocates no device memory.
 *     Workspace sizes come from the *_workspace() queries.  The one device
 *     array the library holds itself is the fixed scratch of
 *     aot_count_noalloc (64 MiB per device).
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Calls
 *     enqueue work on it; calls that return host values synchronise it.
 *   - Vertex ids are int32 in [0, n).  The input graph is a symmetric CSR:
 *     rowptr int64[n+1] (rowptr[0] = 0), col int32[nnz], nnz = 2m, every row
 *     strictly ascending, no self-loops.  m must be <= INT32_MAX.
 *   - Return value: AOT_OK (0) or a negative AOT_E_* code; on error
 *     aot_last_error() gives a thread-local message.  No call aborts.
 *   - Results are deterministic: the same input gives the same bytes for any
 *     dispatch choice, chunking or stream.
 */
#ifndef AOT_H
#define AOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define AOT_OK 0
#define AOT_E_ARG (-1)        /* null pointer, negative size, bad flag        */
#define AOT_E_GRAPH (-2)      /* validation found a malformed CSR             */
#define AOT_E_OVERFLOW (-3)   /* n, nnz or m beyond the int32 edge-id range   */
#define AOT_E_WORKSPACE (-4)  /* workspace smaller than *_workspace() asked   */
#define AOT_E_HIP (-5)        /* a HIP runtime call failed                    */
#define AOT_E_MODEL (-6)      /* cost model missing, malformed or not finite  */
#define AOT_E_CAPACITY (-7)   /* output window larger than the buffer         */

/* Flags for aot_orient. */
#define AOT_VALIDATE 1u       /* check the CSR on the device first (syncs)   */
#define AOT_IN_LISTS_BY_RANK 2u  /* sort every in-list into ascending rank;
                                    costs a segmented sort of m entries, and
                                    makes windows of a very large triangle
                                    list cost about their own triangles     */
#define AOT_ORDER_CORE 4u     /* rank by the core order instead of degree   */
#define AOT_LOCAL_BY_ID 8u    /* keep original ids as labels (random local
                                 order for inputs with permuted ids)        */

/* Text for a status code; never NULL. */
const char* aot_status_str(int status);
/* Detail of the last failing call on this thread ("" if none). */
const char* aot_last_error(void);
/* ABI version, currently 3 (aot_dispatch.strategy, AOT_ORDER_CORE, aot_support,
 * AOT_LOCAL_BY_ID). */
int aot_version(void);

/* Input graph (device pointers). */
typedef struct aot_graph {
  int32_t n;
  int64_t nnz;
  const int64_t* rowptr;  /* device, [n+1] */
  const int32_t* col;     /* device, [nnz] */
} aot_graph;

/* Oriented graph in label space.  By default the label of a vertex is its rank:
 * vertex r is the r-th vertex of the order eta (degree ascending, ties by
 * smaller original id; or the core order).  With AOT_LOCAL_BY_ID the label is
 * the original id (perm and rank are then the identity); eta still directs the
 * edges.  Below, "rank" means the label.  All arrays are device memory owned
 * by the caller; aot_orient fills them.  m = nnz / 2. */
typedef struct aot_oriented {
  int32_t n;
  int64_t m;
  int64_t* rowptr;     /* [n+1] out-list offsets (deg+(r) = rowptr[r+1]-rowptr[r]) */
  int32_t* col;        /* [m]   out-neighbour ranks, strictly ascending per row     */
  int32_t* tail;       /* [m]   source rank of each directed edge                   */
  int32_t* perm;       /* [n]   rank -> original id                                 */
  int32_t* rank;       /* [n]   original id -> rank                                 */
  int64_t* in_rowptr;  /* [n+1] in-list offsets                                     */
  int32_t* in_col;     /* [m]   in-neighbour ranks; per row in ascending ORIGINAL
                                id, or ascending rank with AOT_IN_LISTS_BY_RANK         */
} aot_oriented;

/* ------------------------------------------------------------------------
 * aot_orient -- Section 2.2 (orientation technique) with the degree order of
 * Algorithm 3's first step and Section 3.2's id tie-break.  Ranks vertices by
 * a stable LSD radix sort of degrees, keeps <u,v> iff rank(u) < rank(v), and
 * sorts every out-list ascending (the paper's "local order", Section 3.2,
 * taken ascending in rank space).  Also builds the in-lists that Algorithm 3's
 * second loop walks.
 *   g       input graph (device arrays).
 *   flags   0 or AOT_VALIDATE | AOT_IN_LISTS_BY_RANK | AOT_ORDER_CORE |
 *           AOT_LOCAL_BY_ID.
 *           AOT_ORDER_CORE: rank by the core (degeneracy) order that kClist
 *           orients by (Section 2.3) instead of degree; AOT works on any
 *           total order (Section 3.2).  The order is synchronous peeling:
 *           sub-round r raises the level to the least current degree left
 *           if that is larger and removes at once every remaining vertex of
 *           current degree <= level; ranks follow (sub-round, id).  Then
 *           deg+(r) <= the degeneracy.  Costs a few launches and one host
 *           read per 16 sub-rounds.
 *           AOT_LOCAL_BY_ID: the order still directs every edge, but
 *           vertices keep their original ids as labels, so each out-list is
 *           in ascending id instead of the degree local order (Section 3.2).
 *           On inputs whose ids are randomly permuted this is the random
 *           local order of AOT-randomOrder (Section 4.2).  Rows are indexed
 *           by id, perm and rank are the identity, and both in-list orders
 *           coincide (ascending id).  Counts, the probe count and the
 *           triangle set do not change; the list order follows the labels.
 *   out     caller-allocated arrays of the sizes listed in aot_oriented;
 *           out->n and out->m are written.
 *   ws      device workspace of at least aot_orient_workspace() bytes (6.5 to
 *           7 bytes per symmetric entry: each entry's rank, gathered once, and
 *           the unsorted out-lists, plus O(n)); not read by later calls, so
 *           work queued after this call on `stream` may reuse it.
 * Synchronises `stream` once (to size its launches).  AOT_E_GRAPH (only with
 * AOT_VALIDATE) if a row is unsorted, has a self-loop, a duplicate, an id out
 * of range, or the graph is not symmetric. */
int aot_orient_workspace(int32_t n, int64_t nnz, size_t* bytes);
int aot_orient(const aot_graph* g, uint32_t flags, aot_oriented* out,
               void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Dispatch of the probe kernels.  Edges are grouped into buckets; a bucket's
 * arm picks the index the probes go into and its tile the lanes per edge.
 * The plain rule (mode AOT_DISPATCH_PLAIN) is fixed: light tiles by bin, and
 * the LDS bitmap for every heavy class; aot_count_plan reports the arms it
 * chose.  A bitmap class reserves its widest out-list window, or 16 KiB (six
 * workgroups per CU) if that is wider, or the sorted copy's deg+ words if
 * those are more: an owner whose window does not fit takes the LDS sorted
 * copy.  A table (mode AOT_DISPATCH_TABLE) gives one code per bucket, e.g.
 * chosen by the cost model.  Every choice gives identical results.
 *   heavy_min   owners with deg+ >= heavy_min are processed owner-grouped with
 *               an LDS index (0 = library default, 64).
 *   table       host array of AOT_NUM_BUCKETS codes, or NULL: entry k in 0..7
 *               (light bin k, see the timing recorder) = tile << 8 with tile in
 *               {4, 8, 16, 32, 64} lanes per edge; entry 16 + h (heavy class h)
 *               = index arm 0 bitmap, 1 hash, 2 global binary search, 3 LDS
 *               sorted copy (an owner whose list does not fit the arm's LDS
 *               budget uses the next that does: bitmap or hash -> sorted
 *               -> global).  Other entries are ignored.  AOT_E_MODEL on a
 *               bad code.
 *   model       AOT_DISPATCH_LEARNED: after binning, aot_count computes every
 *               bucket's features, runs the cost model (aot_mlp_* below) and
 *               gives each bucket the option with the lowest predicted
 *               log(ns per probe).  A model whose parameters or predictions are
 *               not finite, or of the wrong shape, is not used: the bucket
 *               falls back to the plain rule (the call still succeeds;
 *               aot_count_plan reports which rule ran).
 *   strategy    which list each edge probes, and into what.  Every strategy
 *               gives the same tri_off and byte-identical lists; they differ
 *               in cost, which aot_count's result[1] reports:
 *     AOT_STRATEGY_ADAPTIVE  Algorithm 3 (Section 3.2): s probes into an index
 *                 of N+(b), built once per owner b; cost sum of
 *                 min(deg+(u), deg+(v)).  The default.
 *     AOT_STRATEGY_HEAD      the fixed orientation: edge <u,v> probes N+(v)
 *                 into an index of N+(u), built once per tail u; the cost
 *                 of kClist's analysis (Section 2.3), sum of deg+(v).
 *     AOT_STRATEGY_MERGE     Algorithm 1 (CF, Section 2.2): each edge merges
 *                 N+(u) with N+(v); cost sum of deg+(u) + deg+(v).
 *     AOT_STRATEGY_PER_EDGE  the CF-Hash remark of Section 2.2: the smaller
 *                 list probes the larger edge by edge, with no per-owner
 *                 index (every edge takes the light path's search of the
 *                 larger list in device memory); cost as ADAPTIVE.
 *               Non-adaptive strategies take AOT_DISPATCH_PLAIN or TABLE
 *               (AOT_E_ARG with LEARNED); MERGE and PER_EDGE ignore
 *               heavy_min and the heavy arms.
 * aot_count stores the plan and strategy it resolved in the workspace;
 * aot_list and aot_digest use that plan unless d gives a table (d = NULL, the
 * plain rule and the learned mode all take the count's plan), and always the
 * count's strategy.
 */
#define AOT_DISPATCH_PLAIN 0
#define AOT_DISPATCH_TABLE 1
#define AOT_DISPATCH_LEARNED 2
#define AOT_STRATEGY_ADAPTIVE 0
#define AOT_STRATEGY_HEAD 1
#define AOT_STRATEGY_MERGE 2
#define AOT_STRATEGY_PER_EDGE 3
#define AOT_NUM_BUCKETS 32
#define AOT_NUM_OPTIONS 9      /* cost-model outputs, see aot_bucket_features */
#define AOT_NUM_FEATURES 8
struct aot_mlp;
typedef struct aot_dispatch {
  int32_t mode;
  int32_t heavy_min;
  const int32_t* table;          /* AOT_DISPATCH_TABLE                       */
  const struct aot_mlp* model;   /* AOT_DISPATCH_LEARNED: the cost model      */
  int32_t strategy;              /* AOT_STRATEGY_*                            */
} aot_dispatch;

/* ------------------------------------------------------------------------
 * aot_count -- Algorithm 3's probe loops, as a count pass.  For every directed
 * edge e = <u,v>: s = endpoint with the smaller (deg+, rank), b = the other
 * (Section 3.2, Correctness, and its footnote); cnt(e) = |N+(s) n N+(b)|,
 * found by probing each w in N+(s) into an index of N+(b).
 *   g        oriented graph from aot_orient (device).
 *   d        dispatch (NULL = plain rule).
 *   tri_off  device int64[m+1], written: exclusive prefix sum of cnt; the
 *            triangles of edge e are global indices [tri_off[e], tri_off[e+1]).
 *   ws       device workspace of at least aot_count_workspace() bytes; keep it
 *            unchanged until the matching aot_list calls are done.
 *   result   host uint64[2], written: {T, probes}; probes = the strategy's
 *            cost, for the adaptive one the sum over edges of
 *            min(deg+(u), deg+(v)).
 * Synchronises `stream`. */
int aot_count_workspace(int32_t n, int64_t m, size_t* bytes);
int aot_count(const aot_oriented* g, const aot_dispatch* d, int64_t* tri_off,
              void* ws, size_t ws_bytes, uint64_t* result, void* stream);

/* ------------------------------------------------------------------------
 * aot_count_noalloc -- aot_count for callers that cannot allocate device
 * memory (serving loops and harnesses that forbid hipMalloc): the same count
 * pass, the same tri_off and result, with the count workspace taken from a
 * fixed scratch array inside the library instead of a `ws` argument.
 *   Limit: the graph's aot_count_workspace() must not exceed
 *          AOT_NOALLOC_SCRATCH_BYTES (64 MiB, about 4e6 edges); larger graphs
 *          get AOT_E_CAPACITY before anything is enqueued.
 *   Each device holds its own scratch from library load until the process
 *   ends; the first call on a device looks up its address.  Calls on one
 *   device share that scratch: calls that overlap in time on one device (two
 *   host threads, or two streams) race and must be serialised by the caller.
 *   Every call rewrites what it reads, so nothing carries over between calls.
 *   The resolved plan stays in the scratch only until the next call: listing
 *   afterwards needs aot_count with a workspace of its own.
 * Allocates nothing (no hipMalloc, hipFree or library allocation); synchronises
 * `stream`.  Arguments and errors otherwise as aot_count. */
#define AOT_NOALLOC_SCRATCH_BYTES (64u << 20)
int aot_count_noalloc(const aot_oriented* g, const aot_dispatch* d, int64_t* tri_off,
                      uint64_t* result, void* stream);

/* The plan the last aot_count on `ws` resolved: table (host int32[32], codes
 * as in aot_dispatch) and *learned = 1 if the cost model chose it, 0 if the
 * plain rule or a given table did. */
int aot_count_plan(const void* ws, size_t ws_bytes, int32_t n, int64_t m, int32_t* table,
                   int32_t* learned);

/* Features of every bucket of the last aot_count on `ws` (host float[32][8]),
 * the cost model's inputs, all from the count pass's own binning:
 *   0 heavy class (1) or light bin (0)   1 log2(1 + edges)
 *   2 log2(1 + mean min(deg+))           3 log2(1 + mean deg+ of the owner)
 *   4 log2(1 + widest owner-list span)   5 log2(1 + mean staged entries per item)
 *   6 log2(1 + work items)               7 bucket id / 32
 * present[b] = 1 when bucket b holds edges.  The cost model's outputs are the
 * predicted log(ns per probe) of the options 0..4 = light tile 4, 8, 16, 32,
 * 64 and 5..8 = heavy arm bitmap, hash, global, sorted. */
int aot_bucket_features(const void* ws, size_t ws_bytes, int32_t n, int64_t m, float* features,
                        uint8_t* present);

/* ------------------------------------------------------------------------
 * aot_list -- Algorithm 3's "output triangle" steps, as a write pass.  Writes
 * triangles [first, first + count) of the global list into out (device,
 * int32[3*count]): each triangle as its three ORIGINAL ids ascending; the
 * global order is edge order, then ascending third vertex (in rank space).
 * Requires the tri_off and workspace of a prior aot_count on the same graph.
 * count may run past T (only T - first are written).  Light edges are
 * visited only over the run of the edge order the window covers, and heavy
 * work items whose owned edges miss the window are skipped whole; with
 * in-lists in rank order (AOT_IN_LISTS_BY_RANK) the in-neighbour items of
 * long rows are narrow runs of the edge order, so a window of a very large
 * list costs about its own triangles.  Synchronises `stream` once at the start (to size its
 * launches); the writes themselves are left enqueued.
 *   written  host, optional: number of triangles written. */
int aot_list(const aot_oriented* g, const aot_dispatch* d, const int64_t* tri_off,
             void* ws, size_t ws_bytes, int64_t first, int64_t count,
             int32_t* out, int64_t* written, void* stream);

/* ------------------------------------------------------------------------
 * aot_digest -- validation mode of the write pass: the same triangles
 * aot_list would emit (each triangle exactly once, Section 3.2 Correctness),
 * digested instead of stored, for graphs whose list does not fit a buffer.
 * Each ascending triple (a, b, c) of original ids hashes to
 *     h = sm(sm(sm(a) ^ b) ^ c),  sm = SplitMix64's output function
 * and the digest is {number of triangles, sum of h mod 2^64, xor of h}.
 *   tri_off, ws   from a prior aot_count on the same graph.
 *   vertex_counts device uint64[n] or NULL: overwritten with the number of
 *                 triangles through each ORIGINAL vertex id (they sum to 3T).
 *   digest        host uint64[3], written.
 * Synchronises `stream`. */
int aot_digest(const aot_oriented* g, const aot_dispatch* d, const int64_t* tri_off,
               void* ws, size_t ws_bytes, uint64_t* vertex_counts, uint64_t* digest,
               void* stream);

/* ------------------------------------------------------------------------
 * aot_support -- the triangle counts that analyses built on triangle listing
 * consume (Section 1: clustering, truss-like cohesion), from the same write
 * pass in digest mode: every triangle found adds one to each of its three
 * oriented edges and, optionally, to each of its three vertices.
 *   tri_off, ws    from a prior aot_count on the same graph (any strategy).
 *   edge_support   device uint32[m], overwritten: for oriented edge e (index
 *                  into g->col), the number of triangles through it, i.e.
 *                  |N(u) n N(v)| of its endpoints.  They sum to 3T.
 *   vertex_counts  device uint64[n] or NULL: triangles through each ORIGINAL
 *                  vertex id (as aot_digest); local clustering coefficient of
 *                  v = 2 t(v) / (deg(v) (deg(v) - 1)).
 *   digest         host uint64[3] or NULL: as aot_digest.
 * Synchronises `stream`. */
int aot_support(const aot_oriented* g, const aot_dispatch* d, const int64_t* tri_off, void* ws,
                size_t ws_bytes, uint32_t* edge_support, uint64_t* vertex_counts,
                uint64_t* digest, void* stream);

/* ------------------------------------------------------------------------
 * Batches of graphs.  Many (small, uneven) graphs are listed as one: their
 * CSRs sit in one arena, the block-diagonal union, and one pass of
 * orientation, binning, count, scan and write covers all of them.  Graph g
 * keeps exactly its own result: the orientation ranks graph by graph and,
 * inside a graph, by (degree, id) as aot_orient does, so graph g's ranks,
 * oriented edges and triangle slots are a contiguous block whose contents
 * equal that graph's own aot_orient / aot_count / aot_list output shifted by
 * the block's offsets (triangles are the same local ids plus voff[g]).  A
 * triangle never spans two graphs (Section 2.1: a triangle is three mutually
 * adjacent vertices, and the union adds no edge).
 *
 * The probe passes run as persistent kernels: a grid of resident workgroups
 * drains a queue of work items (heavy owner windows, heaviest class first,
 * then chunks of light edges, largest c first) through an atomic cursor.  No
 * call reads anything back to the host, so the whole sequence can be
 * captured once in a HIP graph (aot_batch_capture) and replayed.
 *
 * aot_batch      count >= 1 graphs.  voff_host (host) and voff (device) hold
 *                the same int64[count+1] vertex offsets: graph g owns arena
 *                vertices [voff[g], voff[g+1]), voff[0] = 0,
 *                voff[count] = arena.n, non-decreasing.  arena is the union
 *                CSR (device): a row of graph g lists arena ids (local id +
 *                voff[g]) of graph g only, ascending.  AOT_E_OVERFLOW if a
 *                (graph, degree) sort key needs more than 31 bits, i.e.
 *                ceil(log2 count) + ceil(log2 max vertices of a graph) > 31.
 * aot_schedule   the choices an autotuner makes: heavy_min (light/heavy bin
 *                boundary, 0 = 64), use_table = 1 to use table (codes as in
 *                aot_dispatch's table; 0 = the plain rule), light_rounds
 *                (group-rounds of G lanes per light task, 0 = 4).  NULL =
 *                all defaults.  Every schedule gives the same bytes.
 * A batch always ranks by degree (no AOT_ORDER_CORE) and probes with the
 * adaptive strategy.
 */
typedef struct aot_batch {
  int32_t count;
  const int64_t* voff_host;
  const int64_t* voff;
  aot_graph arena;
} aot_batch;

typedef struct aot_schedule {
  int32_t heavy_min;
  int32_t use_table;
  int32_t table[AOT_NUM_BUCKETS];
  int32_t light_rounds;
} aot_schedule;

/* Device workspace for aot_batch_run / aot_batch_capture; it also serves as
 * the count workspace of aot_list / aot_digest on the batch afterwards. */
int aot_batch_workspace(const aot_batch* b, size_t* bytes);

/* Enqueues the whole pass over the batch on `stream`; does not synchronise.
 *   out        caller-allocated oriented arrays of the arena (sizes as for
 *              aot_orient with n = arena.n, m = arena.nnz / 2); rank space is
 *              graph by graph as described above.
 *   tri_off    device int64[m+1]: per-edge triangle offsets, as aot_count.
 *   graph_tri  device int64[count+1], written: graph g's triangles are global
 *              indices [graph_tri[g], graph_tri[g+1]); T = graph_tri[count].
 *   tri        device int32[3*cap]: triangles [0, min(T, cap)) of the global
 *              list (arena ids, ascending per triangle, order as aot_list).
 *              If T > cap, list the rest with aot_list(out, NULL, tri_off,
 *              ws, ...) windows: the same bytes.
 *   ws         at least aot_batch_workspace() bytes. */
int aot_batch_run(const aot_batch* b, const aot_schedule* sc, aot_oriented* out,
                  int64_t* tri_off, int64_t* graph_tri, int32_t* tri, int64_t cap, void* ws,
                  size_t ws_bytes, void* stream);

/* aot_batch_run captured once into a HIP graph (instantiated, opaque).  Every
 * pointer, size and schedule choice is fixed at capture; a launch recomputes
 * everything from the buffers' contents at that time (same shapes).  The
 * caller keeps every buffer alive until aot_batch_destroy.  Launches of one
 * graph must not overlap (they share the workspace). */
typedef struct aot_batch_graph aot_batch_graph;
int aot_batch_capture(const aot_batch* b, const aot_schedule* sc, aot_oriented* out,
                      int64_t* tri_off, int64_t* graph_tri, int32_t* tri, int64_t cap, void* ws,
                      size_t ws_bytes, aot_batch_graph** graph);
int aot_batch_launch(const aot_batch_graph* graph, void* stream);
int aot_batch_destroy(aot_batch_graph* graph);

/* ------------------------------------------------------------------------
 * Cost model of the dispatch: a fully connected network with ReLU, n_in ->
 * n_hidden -> n_hidden -> n_out (fp32), trained on the per-bucket timings the
 * recorder below collects.  `params` is a caller-owned device buffer of
 * aot_mlp_param_count floats: input mean[n_in], 1/std[n_in] (set from the
 * training data, not trained), W1[h][in], b1[h], W2[h][h], b2[h], W3[out][h],
 * b3[out].  n_in <= 16, n_hidden <= 64, n_out <= 16.
 *   aot_mlp_init       weights uniform in +-sqrt(6/fan_in) from a seeded
 *                      counter hash, biases 0, identity normalisation.
 *   aot_mlp_forward    y[batch][n_out] = net(x[batch][n_in]) (device arrays).
 *   aot_mlp_loss_grad  masked mean squared error
 *                      L = (1/N) sum mask[i][k] (y[i][k] - target[i][k])^2
 *                      (N = set mask entries) and its gradient (device
 *                      float[param_count - 2*n_in], trainable part in buffer
 *                      order); reduction order fixed, so results repeat.
 *   aot_mlp_train      sets the normalisation from x, then `epochs` full-batch
 *                      Adam steps (beta 0.9, 0.999, eps 1e-8) at rate lr;
 *                      losses (host float[epochs]) gets L before each step.
 * ws: device workspace of aot_mlp_workspace(net, batch) bytes. */
typedef struct aot_mlp {
  int32_t n_in, n_hidden, n_out;
  float* params;
} aot_mlp;
int aot_mlp_param_count(int32_t n_in, int32_t n_hidden, int32_t n_out, int64_t* count);
int aot_mlp_workspace(const aot_mlp* net, int32_t batch, size_t* bytes);
int aot_mlp_init(const aot_mlp* net, uint64_t seed, void* stream);
int aot_mlp_forward(const aot_mlp* net, const float* x, int32_t batch, float* y, void* stream);
int aot_mlp_loss_grad(const aot_mlp* net, const float* x, const float* target,
                      const uint8_t* mask, int32_t batch, float* grad, float* loss, void* ws,
                      size_t ws_bytes, void* stream);
int aot_mlp_train(const aot_mlp* net, const float* x, const float* target, const uint8_t* mask,
                  int32_t batch, int32_t epochs, float lr, float* losses, void* ws,
                  size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Timing recorder.  While on, every bucket launch of aot_count / aot_list on
 * the calling thread is bracketed by HIP events on its stream, and a record
 * keeps what the launch did -- the per-bucket timings the cost model of the
 * dispatch learns from.  Buckets: 0..7 = light bins of c = min(deg+)
 * ({1}, {2}, (2,4], ..., (64, inf)); 16 + h = heavy owners with
 * ceil(log2 deg+(b)) = h.  Recording adds event overhead; results are the
 * same bytes either way.
 *   aot_timing_start  clears earlier records and starts recording.
 *   aot_timing_stop   stops, waits for the recorded launches, copies up to
 *                     cap records to out (host) and the total to *count;
 *                     AOT_E_CAPACITY if records were dropped. */
typedef struct aot_timing {
  int32_t pass;       /* 0 = count pass, 1 = write pass                       */
  int32_t bucket;     /* see above                                            */
  int32_t arm;        /* heavy: requested index arm (0 bitmap, 1 hash,
                         2 global binary search, 3 LDS sorted copy); light: 0 */
  int32_t tile;       /* lanes per edge (light) or workgroup size (heavy)    */
  int64_t edges;      /* directed edges in the bucket                        */
  int64_t probes;     /* count pass: their sum of min(deg+); write pass: the
                         look-ups made (-1 for a launch over part of a light
                         bin)                                                  */
  int64_t staged;     /* owner out-list entries staged into LDS (heavy)      */
  int64_t triangles;  /* triangles the bucket's edges hold (-1 as probes)    */
  double ms;          /* launch time from HIP events on the launch stream    */
  int64_t lookups;    /* look-ups the launch made: heavy count launches start
                         each probed list at its last 32-entry line below the
                         owner's smallest out-neighbour, heavy write launches
                         at the edge's first hit; light launches make all
                         (-1 as probes)                                        */
} aot_timing;
int aot_timing_start(void);
int aot_timing_stop(aot_timing* out, int32_t cap, int32_t* count);

#ifdef __cplusplus
}
#endif

#endif /* AOT_H */
