/*
 * CPU oracle for AOT triangle listing -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, single-threaded C.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark load this library; the product path
 * never does.  It shares no code, header or table with the HIP library.
 *
 * What it computes (all from "AOT: Pushing the Efficiency Boundary of
 * Main-memory Triangle Listing", Yu, Qin, Zhang, Zhang, Lin, 2020):
 *
 *  orc_orient      -- the orientation technique (Section 2.2, "Orientation
 *                     technique"; Algorithm 3's first step): a total order
 *                     eta by degree, ties by smaller vertex id, and the edge
 *                     (u,v) kept as <u,v> iff eta(u) < eta(v).  The result is
 *                     returned relabelled by eta ("rank space") with every
 *                     out-list sorted ascending, together with perm/rank.
 *                     Its three steps are also exported (orc_rank,
 *                     orc_orient_count, orc_orient_write over rank ranges) so
 *                     that very large graphs can be oriented range by range.
 *  orc_vertex_triangles -- t(v), the triangles through v, as the number of
 *                     edges among the neighbours of v (definition of a
 *                     triangle, Section 2.1), by merging sorted rows.
 *  orc_edge_counts -- per directed edge <u,v>: |N+(u) n N+(v)| by the
 *                     merge-based intersection of Algorithm 1 (CF), Sec. 2.2.
 *  orc_list        -- Algorithm 1 (CF): for each u, each v in N+(u), every w in
 *                     N+(u) n N+(v) is the triangle (u,v,w); emitted as the
 *                     original ids sorted ascending, in edge order then
 *                     ascending w.
 *  orc_sum_min     -- sum over <u,v> of min(deg+(u), deg+(v)): the look-up
 *                     count of the adaptive orientation (Section 3.2, "Time
 *                     Complexity"); orc_sum_min_range over a rank range.
 *  orc_sum_head    -- sum over <u,v> of deg+(v): the kClist cost that
 *                     Example 1 compares against (Sections 2.3 and 3.2).
 *  orc_aot_ref     -- Algorithm 3 (AOT) as written: a |V|-entry bitmap H of
 *                     N+(u) per pivot u, the out-neighbour loop and the
 *                     in-neighbour loop, each probing only when the other
 *                     endpoint has the smaller out-degree, ties broken by
 *                     vertex id (Section 3.2, "Correctness" and its footnote),
 *                     neighbours visited in decreasing degree (Section 3.2,
 *                     "Exploiting Local Order").  Works in original ids.
 *  orc_fingerprint -- order-independent sums of a SplitMix64-chained hash of
 *                     each triple, and per-vertex triangle counts.
 *
 * Conventions: rowptr int64[n+1], col int32[nnz], symmetric simple graph with
 * sorted rows.  Return values < 0 signal an error (allocation or capacity).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { int64_t deg; int32_t id; } deg_id;

static int cmp_deg_id(const void* a, const void* b) {
  const deg_id* x = (const deg_id*)a;
  const deg_id* y = (const deg_id*)b;
  if (x->deg != y->deg) return x->deg < y->deg ? -1 : 1;
  return (x->id > y->id) - (x->id < y->id);
}

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* The order eta: perm[r] = original id of rank r, rank[v] = eta(v); degree
 * ascending, ties by smaller id (Section 2.2, with the degree order of
 * Algorithm 3's first step).  Returns 0, or -1 if out of memory. */
int orc_rank(int32_t n, const int64_t* rowptr, int32_t* perm, int32_t* rank) {
  deg_id* order = (deg_id*)malloc(sizeof(deg_id) * (size_t)(n > 0 ? n : 1));
  if (!order) return -1;
  for (int32_t v = 0; v < n; ++v) {
    order[v].deg = rowptr[v + 1] - rowptr[v];
    order[v].id = v;
  }
  qsort(order, (size_t)n, sizeof(deg_id), cmp_deg_id);
  for (int32_t r = 0; r < n; ++r) {
    perm[r] = order[r].id;
    rank[order[r].id] = r;
  }
  free(order);
  return 0;
}

/* deg+(r) for ranks r in [r_lo, r_hi): neighbours of perm[r] ranked above r. */
void orc_orient_count(const int64_t* rowptr, const int32_t* col, const int32_t* perm,
                      const int32_t* rank, int32_t r_lo, int32_t r_hi, int64_t* dplus) {
  for (int32_t r = r_lo; r < r_hi; ++r) {
    int32_t u = perm[r];
    int64_t c = 0;
    for (int64_t k = rowptr[u]; k < rowptr[u + 1]; ++k) c += rank[col[k]] > r;
    dplus[r - r_lo] = c;
  }
}

/* Out-lists of ranks [r_lo, r_hi) into ocol at orow[r], each sorted
 * ascending (ranks above r, relabelled by eta). */
void orc_orient_write(const int64_t* rowptr, const int32_t* col, const int32_t* perm,
                      const int32_t* rank, const int64_t* orow, int32_t r_lo, int32_t r_hi,
                      int32_t* ocol) {
  for (int32_t r = r_lo; r < r_hi; ++r) {
    int32_t u = perm[r];
    int64_t at = orow[r];
    for (int64_t k = rowptr[u]; k < rowptr[u + 1]; ++k) {
      int32_t rv = rank[col[k]];
      if (rv > r) ocol[at++] = rv;
    }
    qsort(ocol + orow[r], (size_t)(at - orow[r]), sizeof(int32_t), cmp_i32);
  }
}

/* Orientation: orc_rank, then keep <u,v> iff eta(u) < eta(v).  Outputs
 * perm, rank, orow[n+1], ocol[m] in rank space, each row ascending.
 * Returns m or -1. */
int64_t orc_orient(int32_t n, const int64_t* rowptr, const int32_t* col,
                   int32_t* perm, int32_t* rank, int64_t* orow, int32_t* ocol) {
  if (orc_rank(n, rowptr, perm, rank)) return -1;
  int64_t* dplus = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!dplus) return -1;
  orc_orient_count(rowptr, col, perm, rank, 0, n, dplus);
  orow[0] = 0;
  for (int32_t r = 0; r < n; ++r) orow[r + 1] = orow[r] + dplus[r];
  free(dplus);
  orc_orient_write(rowptr, col, perm, rank, orow, 0, n, ocol);
  return orow[n];
}

/* The core (degeneracy) order that kClist orients by (Section 2.3), taken as
 * synchronous peeling.  Sub-round r first raises the level to the smallest
 * current degree among the remaining vertices if that is larger, then
 * removes, all at once, every remaining vertex whose current degree is at
 * most the level, and lowers its remaining neighbours' current degrees by
 * one per removed neighbour.  round[v] = the sub-round that removes v.  A
 * vertex has at most `level` neighbours left when it goes, so ordering by
 * (round, id) gives every vertex at most that many out-neighbours, and the
 * largest level reached is the degeneracy.  Returns the number of
 * sub-rounds (*degeneracy = the largest level), or -1 if out of memory. */
int32_t orc_core_rounds(int32_t n, const int64_t* rowptr, const int32_t* col, int32_t* round,
                        int32_t* degeneracy) {
  int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int32_t* gone = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  if (!cur || !gone) { free(cur); free(gone); return -1; }
  int32_t left = n, r = 0;
  int64_t level = 0;
  for (int32_t v = 0; v < n; ++v) { cur[v] = rowptr[v + 1] - rowptr[v]; round[v] = -1; }
  while (left > 0) {
    int64_t low = -1;
    for (int32_t v = 0; v < n; ++v)
      if (round[v] < 0 && (low < 0 || cur[v] < low)) low = cur[v];
    if (low > level) level = low;
    int32_t k = 0;
    for (int32_t v = 0; v < n; ++v)
      if (round[v] < 0 && cur[v] <= level) gone[k++] = v;
    for (int32_t i = 0; i < k; ++i) round[gone[i]] = r;
    for (int32_t i = 0; i < k; ++i) {
      int32_t v = gone[i];
      for (int64_t e = rowptr[v]; e < rowptr[v + 1]; ++e)
        if (round[col[e]] < 0) --cur[col[e]];
    }
    left -= k;
    ++r;
  }
  *degeneracy = (int32_t)level;
  free(cur);
  free(gone);
  return r;
}

typedef struct { int32_t key; int32_t id; } key_id;

static int cmp_key_id(const void* a, const void* b) {
  const key_id* x = (const key_id*)a;
  const key_id* y = (const key_id*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return (x->id > y->id) - (x->id < y->id);
}

/* The orientation by the core order: rank = position in (round, id)
 * ascending, then as orc_orient.  Returns m, or -1. */
int64_t orc_orient_core(int32_t n, const int64_t* rowptr, const int32_t* col, int32_t* perm,
                        int32_t* rank, int64_t* orow, int32_t* ocol) {
  int32_t* round = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  key_id* order = (key_id*)malloc(sizeof(key_id) * (size_t)(n > 0 ? n : 1));
  int64_t* dplus = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int32_t degeneracy;
  if (!round || !order || !dplus || orc_core_rounds(n, rowptr, col, round, &degeneracy) < 0) {
    free(round); free(order); free(dplus);
    return -1;
  }
  for (int32_t v = 0; v < n; ++v) { order[v].key = round[v]; order[v].id = v; }
  qsort(order, (size_t)n, sizeof(key_id), cmp_key_id);
  for (int32_t r = 0; r < n; ++r) {
    perm[r] = order[r].id;
    rank[order[r].id] = r;
  }
  orc_orient_count(rowptr, col, perm, rank, 0, n, dplus);
  orow[0] = 0;
  for (int32_t r = 0; r < n; ++r) orow[r + 1] = orow[r] + dplus[r];
  orc_orient_write(rowptr, col, perm, rank, orow, 0, n, ocol);
  free(round); free(order); free(dplus);
  return orow[n];
}

/* Orientation that keeps the original ids as labels: the order eta (given as
 * rank[v]) still directs every edge, but the out-list of vertex u holds the
 * original ids of its neighbours v with eta(v) > eta(u), sorted ascending, and
 * rows are indexed by original id.  Inside each list, vertices then follow id
 * order instead of the degree local order of Section 3.2; for inputs with
 * randomly permuted ids this is the random local order of AOT-randomOrder
 * (Section 4.2).  Returns m. */
int64_t orc_orient_by_id(int32_t n, const int64_t* rowptr, const int32_t* col,
                         const int32_t* rank, int64_t* orow, int32_t* ocol) {
  orow[0] = 0;
  for (int32_t u = 0; u < n; ++u) {
    int64_t at = orow[u];
    for (int64_t k = rowptr[u]; k < rowptr[u + 1]; ++k)
      if (rank[col[k]] > rank[u]) ocol[at++] = col[k];
    qsort(ocol + orow[u], (size_t)(at - orow[u]), sizeof(int32_t), cmp_i32);
    orow[u + 1] = at;
  }
  return orow[n];
}

/* In-lists of the oriented graph (Algorithm 3's second loop walks them): for
 * rank r, every x with r in N+(x), in ascending rank x; ieid[j] is the index
 * in ocol of the edge <icol[j], r>.  Built as the transpose of the out-lists,
 * visiting the edges in order.  Returns m. */
int64_t orc_in_lists(int32_t n, const int64_t* orow, const int32_t* ocol, int64_t* irow,
                     int32_t* icol, int32_t* ieid) {
  const int64_t m = orow[n];
  for (int32_t r = 0; r <= n; ++r) irow[r] = 0;
  for (int64_t e = 0; e < m; ++e) irow[ocol[e] + 1] += 1;
  for (int32_t r = 0; r < n; ++r) irow[r + 1] += irow[r];
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!fill) return -1;
  for (int32_t r = 0; r < n; ++r) fill[r] = irow[r];
  for (int32_t x = 0; x < n; ++x)
    for (int64_t e = orow[x]; e < orow[x + 1]; ++e) {
      const int32_t r = ocol[e];
      icol[fill[r]] = x;
      ieid[fill[r]] = (int32_t)e;
      fill[r] += 1;
    }
  free(fill);
  return m;
}

/* |A n B| for two ascending lists, by merging. */
static int64_t merge_count(const int32_t* a, int64_t na, const int32_t* b, int64_t nb) {
  int64_t i = 0, j = 0, c = 0;
  while (i < na && j < nb) {
    if (a[i] < b[j]) ++i;
    else if (a[i] > b[j]) ++j;
    else { ++c; ++i; ++j; }
  }
  return c;
}

/* Support of every oriented edge e = <r, x> (rank space): the number of
 * triangles through it, |N(u) n N(v)| over the full neighbourhoods of its
 * original endpoints u = perm[r], v = perm[x] (an entry of A^2), by merging
 * the two sorted rows of the input. */
void orc_edge_support(int32_t n, const int64_t* rowptr, const int32_t* col, const int64_t* orow,
                      const int32_t* ocol, const int32_t* perm, int32_t* sup) {
  for (int32_t r = 0; r < n; ++r)
    for (int64_t e = orow[r]; e < orow[r + 1]; ++e) {
      int32_t u = perm[r], v = perm[ocol[e]];
      sup[e] = (int32_t)merge_count(col + rowptr[u], rowptr[u + 1] - rowptr[u],
                                    col + rowptr[v], rowptr[v + 1] - rowptr[v]);
    }
}

/* Source (rank) of directed edge e: the row r with orow[r] <= e < orow[r+1]. */
static int32_t edge_tail(int32_t n, const int64_t* orow, int64_t e) {
  int32_t lo = 0, hi = n - 1;
  while (lo < hi) {
    int32_t mid = lo + (hi - lo + 1) / 2;
    if (orow[mid] <= e) lo = mid; else hi = mid - 1;
  }
  return lo;
}

/* cnt[i] = |N+(u) n N+(v)| for edges e = e_lo + i, e < e_hi (CF's intersection step, Algorithm 1). */
void orc_edge_counts(int32_t n, const int64_t* orow, const int32_t* ocol,
                     int64_t e_lo, int64_t e_hi, int32_t* cnt) {
  if (e_hi <= e_lo) return;
  int32_t u = edge_tail(n, orow, e_lo);
  for (int64_t e = e_lo; e < e_hi; ++e) {
    while (orow[u + 1] <= e) ++u;
    int32_t v = ocol[e];
    cnt[e - e_lo] = (int32_t)merge_count(ocol + orow[u], orow[u + 1] - orow[u],
                                         ocol + orow[v], orow[v + 1] - orow[v]);
  }
}

/* Same, for an arbitrary list of edge ids (sampled checks). */
void orc_edge_counts_at(int32_t n, const int64_t* orow, const int32_t* ocol,
                        const int64_t* eids, int64_t k, int32_t* cnt) {
  for (int64_t i = 0; i < k; ++i) {
    int64_t e = eids[i];
    int32_t u = edge_tail(n, orow, e);
    int32_t v = ocol[e];
    cnt[i] = (int32_t)merge_count(ocol + orow[u], orow[u + 1] - orow[u],
                                  ocol + orow[v], orow[v + 1] - orow[v]);
  }
}

static void sort3(int32_t* t) {
  int32_t x;
  if (t[0] > t[1]) { x = t[0]; t[0] = t[1]; t[1] = x; }
  if (t[1] > t[2]) { x = t[1]; t[1] = t[2]; t[2] = x; }
  if (t[0] > t[1]) { x = t[0]; t[0] = t[1]; t[1] = x; }
}

/* Algorithm 1 (CF) over the edges of source ranks [r_lo, r_hi).  Triangles go
 * to out[3*i..3*i+2] as ascending original ids, in edge order then ascending
 * w.  Returns the number of triangles, or -(needed) if cap is too small
 * (nothing beyond cap is written). */
int64_t orc_list(int32_t n, const int64_t* orow, const int32_t* ocol, const int32_t* perm,
                 int32_t r_lo, int32_t r_hi, int32_t* out, int64_t cap) {
  (void)n;
  int64_t t = 0;
  for (int32_t u = r_lo; u < r_hi; ++u) {
    const int32_t* a = ocol + orow[u];
    int64_t na = orow[u + 1] - orow[u];
    for (int64_t k = 0; k < na; ++k) {
      int32_t v = a[k];
      const int32_t* b = ocol + orow[v];
      int64_t nb = orow[v + 1] - orow[v];
      int64_t i = 0, j = 0;
      while (i < na && j < nb) {
        if (a[i] < b[j]) ++i;
        else if (a[i] > b[j]) ++j;
        else {
          if (t < cap) {
            int32_t* o = out + 3 * t;
            o[0] = perm[u]; o[1] = perm[v]; o[2] = perm[a[i]];
            sort3(o);
          }
          ++t; ++i; ++j;
        }
      }
    }
  }
  return t <= cap ? t : -t;
}

/* sum over <u,v> of min(deg+(u), deg+(v)), rank space. */
/* sum over <u,v> with u in [r_lo, r_hi) of min(deg+(u), deg+(v)). */
uint64_t orc_sum_min_range(const int64_t* orow, const int32_t* ocol, int32_t r_lo, int32_t r_hi) {
  uint64_t s = 0;
  for (int32_t u = r_lo; u < r_hi; ++u) {
    int64_t du = orow[u + 1] - orow[u];
    for (int64_t e = orow[u]; e < orow[u + 1]; ++e) {
      int32_t v = ocol[e];
      int64_t dv = orow[v + 1] - orow[v];
      s += (uint64_t)(du < dv ? du : dv);
    }
  }
  return s;
}

uint64_t orc_sum_min(int32_t n, const int64_t* orow, const int32_t* ocol) {
  uint64_t s = 0;
  for (int32_t u = 0; u < n; ++u) {
    int64_t du = orow[u + 1] - orow[u];
    for (int64_t e = orow[u]; e < orow[u + 1]; ++e) {
      int32_t v = ocol[e];
      int64_t dv = orow[v + 1] - orow[v];
      s += (uint64_t)(du < dv ? du : dv);
    }
  }
  return s;
}

/* sum over <u,v> of deg+(v). */
uint64_t orc_sum_head(int32_t n, const int64_t* orow, const int32_t* ocol) {
  uint64_t s = 0;
  for (int32_t u = 0; u < n; ++u)
    for (int64_t e = orow[u]; e < orow[u + 1]; ++e) {
      int32_t v = ocol[e];
      s += (uint64_t)(orow[v + 1] - orow[v]);
    }
  return s;
}

/* sum over <u,v> of deg+(u) + deg+(v): the cost of Algorithm 1's merge
 * intersections (Section 2.2, Analysis). */
uint64_t orc_sum_merge(int32_t n, const int64_t* orow, const int32_t* ocol) {
  uint64_t s = 0;
  for (int32_t u = 0; u < n; ++u) {
    int64_t du = orow[u + 1] - orow[u];
    for (int64_t e = orow[u]; e < orow[u + 1]; ++e) {
      int32_t v = ocol[e];
      s += (uint64_t)du + (uint64_t)(orow[v + 1] - orow[v]);
    }
  }
  return s;
}

static uint64_t triple_hash(uint32_t a, uint32_t b, uint32_t c);

/* AOT (Algorithm 3, Section 3.2) on the original ids: the cross-check of the
 * CF procedure above, written from the algorithm's idea.
 *
 * Orientation: the degree order with the smaller id first on ties; each
 * out-list N+(x) is kept in decreasing degree order (the local order of
 * Section 3.2).  Then every vertex u takes one turn as the indexed vertex:
 * N+(u) is marked in a table H of |V| flags, and every neighbour x of u in
 * the undirected graph -- the edge may point out of u or into u -- whose key
 * (deg+(x), x) is below u's has each w in N+(x) looked up in H.  A hit closes
 * the triangle {u, x, w}.  So each edge is worked on from the endpoint with
 * the larger key only, and only the smaller out-list is read (Section 3.1;
 * the id tie-break of Section 3.2's footnote).  H is cleared after the turn.
 *   tie_break = 0 compares deg+ alone, strictly, so edges whose endpoints
 *               have equal deg+ are never worked on; kept to show that the
 *               tie rule is needed.
 * Output: with out != NULL, triangles (ascending ids) up to cap; with
 * fp != NULL, fp[0] = sum and fp[1] = xor of the triple hashes (as
 * orc_fingerprint).  *probes = number of look-ups in H.  Returns the triangle
 * count (-count if out was too short), or INT64_MIN on allocation failure. */
int64_t orc_aot_ref(int32_t n, const int64_t* rowptr, const int32_t* col, int tie_break,
                    int32_t* out, int64_t cap, uint64_t* fp, uint64_t* probes) {
  const size_t nn = (size_t)(n > 0 ? n : 1);
  int64_t m2 = rowptr[n];
  int32_t* eta = (int32_t*)malloc(sizeof(int32_t) * nn);
  deg_id* order = (deg_id*)malloc(sizeof(deg_id) * nn);
  int64_t* dplus = (int64_t*)calloc(nn, sizeof(int64_t));
  int64_t* orow = (int64_t*)malloc(sizeof(int64_t) * (nn + 1));
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * nn);
  int32_t* nplus = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m2 / 2 > 0 ? m2 / 2 : 1));
  unsigned char* H = (unsigned char*)calloc(nn, 1);
  if (!eta || !order || !dplus || !orow || !fill || !nplus || !H) {
    free(eta); free(order); free(dplus); free(orow); free(fill); free(nplus); free(H);
    return INT64_MIN;
  }
  for (int32_t v = 0; v < n; ++v) { order[v].deg = rowptr[v + 1] - rowptr[v]; order[v].id = v; }
  qsort(order, (size_t)n, sizeof(deg_id), cmp_deg_id);
  for (int32_t r = 0; r < n; ++r) eta[order[r].id] = r;
  for (int32_t x = 0; x < n; ++x)
    for (int64_t k = rowptr[x]; k < rowptr[x + 1]; ++k) dplus[x] += eta[col[k]] > eta[x];
  orow[0] = 0;
  for (int32_t x = 0; x < n; ++x) { orow[x + 1] = orow[x] + dplus[x]; fill[x] = orow[x]; }
  /* visiting the vertices from the top of the order down and appending each
   * to the out-list of every lower neighbour leaves every out-list in
   * decreasing degree order */
  for (int32_t r = n - 1; r >= 0; --r) {
    int32_t w = order[r].id;
    for (int64_t k = rowptr[w]; k < rowptr[w + 1]; ++k) {
      int32_t x = col[k];
      if (eta[x] < eta[w]) nplus[fill[x]++] = w;
    }
  }
  int64_t t = 0;
  uint64_t looked = 0, hsum = 0, hxor = 0;
  for (int32_t u = 0; u < n; ++u) {
    for (int64_t k = orow[u]; k < orow[u + 1]; ++k) H[nplus[k]] = 1;
    for (int64_t k = rowptr[u]; k < rowptr[u + 1]; ++k) {
      int32_t x = col[k];
      int below = dplus[x] < dplus[u] || (tie_break && dplus[x] == dplus[u] && x < u);
      if (!below) continue;
      for (int64_t j = orow[x]; j < orow[x + 1]; ++j) {
        int32_t w = nplus[j];
        ++looked;
        if (!H[w]) continue;
        int32_t tri[3] = {u, x, w};
        sort3(tri);
        if (out && t < cap) memcpy(out + 3 * t, tri, sizeof tri);
        if (fp) {
          uint64_t h = triple_hash((uint32_t)tri[0], (uint32_t)tri[1], (uint32_t)tri[2]);
          hsum += h;
          hxor ^= h;
        }
        ++t;
      }
    }
    for (int64_t k = orow[u]; k < orow[u + 1]; ++k) H[nplus[k]] = 0;
  }
  *probes = looked;
  if (fp) { fp[0] = hsum; fp[1] = hxor; }
  free(eta); free(order); free(dplus); free(orow); free(fill); free(nplus); free(H);
  return (!out || t <= cap) ? t : -t;
}

/* SplitMix64's output function (Steele, Lea, Flood 2014) on z + golden gamma. */
static uint64_t splitmix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

uint64_t orc_splitmix64(uint64_t z) { return splitmix64(z); }

/* Hash of an ascending triple: splitmix64 chained over a, b, c. */
static uint64_t triple_hash(uint32_t a, uint32_t b, uint32_t c) {
  return splitmix64(splitmix64(splitmix64((uint64_t)a) ^ (uint64_t)b) ^ (uint64_t)c);
}

/* Fingerprints of a triangle list (ascending triples): fp[0] = sum of hashes
 * mod 2^64, fp[1] = xor of hashes; tv[v] += 1 for each corner (if tv). */
void orc_fingerprint(const int32_t* tri, int64_t t, uint64_t* fp, uint64_t* tv) {
  uint64_t s = 0, x = 0;
  for (int64_t i = 0; i < t; ++i) {
    const int32_t* o = tri + 3 * i;
    uint64_t h = triple_hash((uint32_t)o[0], (uint32_t)o[1], (uint32_t)o[2]);
    s += h; x ^= h;
    if (tv) { tv[o[0]]++; tv[o[1]]++; tv[o[2]]++; }
  }
  fp[0] = s; fp[1] = x;
}

/* CF over source ranks [r_lo, r_hi) without storing triangles: the count, the
 * fingerprints and per-vertex counts (original ids) -- for graphs whose full
 * triangle list does not fit in host memory. */
int64_t orc_list_digest(int32_t n, const int64_t* orow, const int32_t* ocol, const int32_t* perm,
                        int32_t r_lo, int32_t r_hi, uint64_t* fp, uint64_t* tv) {
  (void)n;
  int64_t t = 0;
  uint64_t s = 0, x = 0;
  for (int32_t u = r_lo; u < r_hi; ++u) {
    const int32_t* a = ocol + orow[u];
    int64_t na = orow[u + 1] - orow[u];
    for (int64_t k = 0; k < na; ++k) {
      int32_t v = a[k];
      const int32_t* b = ocol + orow[v];
      int64_t nb = orow[v + 1] - orow[v];
      int64_t i = 0, j = 0;
      while (i < na && j < nb) {
        if (a[i] < b[j]) ++i;
        else if (a[i] > b[j]) ++j;
        else {
          int32_t o[3] = {perm[u], perm[v], perm[a[i]]};
          sort3(o);
          uint64_t h = triple_hash((uint32_t)o[0], (uint32_t)o[1], (uint32_t)o[2]);
          s += h; x ^= h;
          if (tv) { tv[o[0]]++; tv[o[1]]++; tv[o[2]]++; }
          ++t; ++i; ++j;
        }
      }
    }
  }
  fp[0] = s; fp[1] = x;
  return t;
}

/* Triangles through vertex v of the input graph (original ids), from the
 * plain definition: t(v) = number of edges {x, y} with x, y both neighbours of
 * v, i.e. half of the sum over x in N(v) of |N(v) n N(x)| (sorted rows,
 * merged).  out[i] = t(vs[i]). */
void orc_vertex_triangles(const int64_t* rowptr, const int32_t* col, const int32_t* vs, int64_t k,
                          int64_t* out) {
  for (int64_t i = 0; i < k; ++i) {
    int32_t v = vs[i];
    const int32_t* nv = col + rowptr[v];
    int64_t dv = rowptr[v + 1] - rowptr[v];
    int64_t twice = 0;
    for (int64_t j = 0; j < dv; ++j) {
      int32_t x = nv[j];
      twice += merge_count(nv, dv, col + rowptr[x], rowptr[x + 1] - rowptr[x]);
    }
    out[i] = twice / 2;
  }
}
