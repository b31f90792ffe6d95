"""Pins for the CPU oracle, against things other than the oracle itself:
brute force, dense matrix powers, closed forms, the paper's Example 1, the
published SplitMix64 outputs, and Algorithm 3 run literally (with the
tie-break footnote's rule shown necessary on a small counterexample)."""

import itertools
import math
import os

import numpy as np
import pytest

import oracle
from paper_2006_11494_amd import inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# ---------------------------------------------------------------- helpers

def random_graph(n, p, seed):
    rng = np.random.default_rng(seed)
    a = np.triu(rng.random((n, n)) < p, 1)
    iu, ju = np.nonzero(a)
    return inputs.csr_from_edges_np(n, zip(iu.tolist(), ju.tolist()))


def dense(csr):
    rp, col = csr.numpy()
    n = csr.n
    A = np.zeros((n, n), np.int64)
    rows = np.repeat(np.arange(n), np.diff(rp))
    A[rows, col] = 1
    return A


def brute_force(csr):
    """Every (a, b, c), a < b < c, with all three edges present."""
    A = dense(csr)
    return sorted(t for t in itertools.combinations(range(csr.n), 3)
                  if A[t[0], t[1]] and A[t[0], t[2]] and A[t[1], t[2]])


def as_set(tri):
    return sorted(map(tuple, np.asarray(tri).reshape(-1, 3).tolist()))


def cf_list(csr):
    rp, col = csr.numpy()
    return oracle.list_triangles(oracle.orient(rp, col))


def graph(n, edges):
    return inputs.csr_from_edges_np(n, edges)


SMALL = [(n, p, s) for s, (n, p) in enumerate(
    [(0, 0.5), (1, 0.5), (2, 1.0), (3, 1.0), (5, 0.6), (8, 0.5), (12, 0.3), (12, 0.9),
     (17, 0.4), (20, 0.15), (25, 0.5), (30, 0.25), (40, 0.2), (33, 0.7)])]


# ---------------------------------------------------------------- hashing

def test_splitmix64_published_outputs():
    # SplitMix64 seeded with 0 outputs these first four words; the k-th output
    # is the mix of state k * golden-gamma.
    gamma = 0x9E3779B97F4A7C15
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]
    got = [oracle.splitmix64((k * gamma) & (2**64 - 1)) for k in range(4)]
    assert got == want


# ---------------------------------------------------------------- orientation

@pytest.mark.parametrize("n,p,seed", SMALL + [(300, 0.05, 99), (500, 0.02, 98)])
def test_orientation_is_the_degree_order(n, p, seed):
    g = random_graph(n, p, seed)
    rp, col = g.numpy()
    o = oracle.orient(rp, col)
    deg = np.diff(rp)
    perm = np.lexsort((np.arange(n), deg)).astype(np.int32)  # degree asc, id asc
    assert np.array_equal(o.perm, perm)
    rank = np.empty(n, np.int64)
    rank[perm] = np.arange(n)
    assert np.array_equal(o.rank, rank)
    # every undirected edge appears exactly once, pointing up the order
    rows = np.repeat(np.arange(n), deg)
    up = rank[rows] < rank[col]
    want = sorted(zip(rank[rows[up]].tolist(), rank[col[up]].tolist()))
    tail = o.tail()
    got = list(zip(tail.tolist(), o.ocol.tolist()))
    assert got == want            # CSR order = sorted by (tail, head): rows ascending
    assert o.m == g.m
    assert all(a < b for a, b in got)   # acyclic: the order increases along every edge


def test_orientation_example1_directions():
    ex = load_example1()
    rp, col = ex["csr"].numpy()
    o = oracle.orient(rp, col)
    dplus = o.dplus
    name = lambda r: int(o.perm[r]) + 1
    out = {name(r): sorted(name(v) for v in o.ocol[o.orow[r]:o.orow[r + 1]]) for r in range(o.n)}
    # directions the example's text names
    for (u, v, _, _) in ex["cost"]:
        assert v in out[u], (u, v)
    assert out[3] == [4, 13, 14] and out[4] == [13, 14]
    assert out[1] == [3] and out[2] == [4]
    assert out[13] == [] and out[14] == []          # the two sinks
    assert sum(dplus) == 21


# ---------------------------------------------------------------- listing

@pytest.mark.parametrize("n,p,seed", SMALL)
def test_list_equals_brute_force(n, p, seed):
    g = random_graph(n, p, seed)
    tri = cf_list(g)
    assert as_set(tri) == brute_force(g)
    # rows are ascending triples and the list has no repeats
    assert all(a < b < c for a, b, c in tri.tolist())
    assert len(set(map(tuple, tri.tolist()))) == len(tri)


@pytest.mark.parametrize("n,p,seed", [(60, 0.3, 1), (200, 0.05, 2), (300, 0.1, 3), (400, 0.02, 4)])
def test_count_equals_trace_a3(n, p, seed):
    g = random_graph(n, p, seed)
    A = dense(g)
    A3 = A @ A @ A
    tri = cf_list(g)
    assert len(tri) == np.trace(A3) // 6
    (_, _), tv = oracle.fingerprint(tri, n)
    assert np.array_equal(tv.astype(np.int64), np.diag(A3) // 2)   # per-vertex counts
    assert int(tv.sum()) == 3 * len(tri)


@pytest.mark.parametrize("n,p,seed", [(40, 0.3, 5), (120, 0.1, 6), (250, 0.06, 7)])
def test_edge_counts_brute_force(n, p, seed):
    g = random_graph(n, p, seed)
    rp, col = g.numpy()
    o = oracle.orient(rp, col)
    A = dense(g)
    cnt = oracle.edge_counts(o)
    perm = o.perm
    tail = o.tail()
    for e in range(o.m):
        u, v = perm[tail[e]], perm[o.ocol[e]]
        # third corners ranked above both edge ends
        want = sum(1 for w in range(n) if A[u, w] and A[v, w] and o.rank[w] > o.rank[v])
        assert cnt[e] == want
    assert int(cnt.sum()) == len(brute_force(g)) if n <= 60 else True
    assert int(cnt.sum()) == np.trace(A @ A @ A) // 6
    # sampled edge ids give the same numbers
    pick = np.arange(0, o.m, 7)
    assert np.array_equal(oracle.edge_counts_at(o, pick), cnt[pick])
    # a sub-range too
    assert np.array_equal(oracle.edge_counts(o, 3, o.m - 2), cnt[3:o.m - 2])


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", range(3, 13))
def test_complete_graph(n):
    g = graph(n, itertools.combinations(range(n), 2))
    rp, col = g.numpy()
    o = oracle.orient(rp, col)
    assert len(oracle.list_triangles(o)) == math.comb(n, 3)
    # all degrees tie, so the order is by id and deg+(i) = n-1-i: every edge
    # <i,j> costs n-1-j and the total is C(n,3)
    assert oracle.sum_min(o) == math.comb(n, 3)
    assert oracle.sum_head(o) == math.comb(n, 3)
    # the tails add sum over i of deg+(i) * deg+(i) = 0^2 + 1^2 + ... + (n-1)^2
    assert oracle.sum_merge(o) == math.comb(n, 3) + (n - 1) * n * (2 * n - 1) // 6


@pytest.mark.parametrize("k", [1, 2, 5, 17])
def test_star_costs(k):
    # K_{1,k}: every leaf (degree 1) points at the hub (degree k >= 1, or the
    # larger id when k = 1), which has no out-neighbour: the head never costs
    # anything and CF still merges each leaf's one-entry list
    g = graph(k + 1, [(0, i) for i in range(1, k + 1)])
    rp, col = g.numpy()
    o = oracle.orient(rp, col)
    assert len(oracle.list_triangles(o)) == 0
    assert oracle.sum_min(o) == 0
    assert oracle.sum_head(o) == 0
    assert oracle.sum_merge(o) == k


def grid(a, b):
    idx = lambda i, j: i * b + j
    e = [(idx(i, j), idx(i + 1, j)) for i in range(a - 1) for j in range(b)]
    e += [(idx(i, j), idx(i, j + 1)) for i in range(a) for j in range(b - 1)]
    return graph(a * b, e)


def wheel(n):
    rim = n - 1
    e = [(0, i) for i in range(1, n)] + [(i, i % rim + 1) for i in range(1, n)]
    return graph(n, e)


@pytest.mark.parametrize("g,t", [
    (graph(7, [(i, 3 + j) for i in range(3) for j in range(4)]), 0),      # K_{3,4}
    (graph(11, [(i, 5 + j) for i in range(5) for j in range(6)]), 0),     # K_{5,6}
    (grid(5, 7), 0), (grid(1, 9), 0), (grid(12, 12), 0),
    (graph(8, [(i, (i + 1) % 8) for i in range(8)]), 0),                  # C_8
    (graph(3, [(0, 1), (1, 2), (2, 0)]), 1),                               # C_3
    (graph(5, [(i, (i + 1) % 5) for i in range(5)]), 0),                  # C_5
    (graph(10, [(0, i) for i in range(1, 10)]), 0),                       # star
    (graph(9, [(i, (i - 1) // 2) for i in range(1, 9)]), 0),              # binary tree
    (wheel(4), 4), (wheel(5), 4), (wheel(6), 5), (wheel(13), 12), (wheel(50), 49),
    (graph(6, []), 0), (graph(1, []), 0),
])
def test_closed_forms(g, t):
    assert len(cf_list(g)) == t
    assert len(brute_force(g)) == t


def test_disjoint_union_and_relabelling():
    g1 = random_graph(30, 0.3, 11)
    g2 = random_graph(25, 0.4, 12)
    r1, c1 = g1.numpy()
    r2, c2 = g2.numpy()
    e1 = [(u, int(v)) for u in range(30) for v in c1[r1[u]:r1[u + 1]] if u < v]
    e2 = [(u + 30, int(v) + 30) for u in range(25) for v in c2[r2[u]:r2[u + 1]] if u < v]
    t1, t2 = len(cf_list(g1)), len(cf_list(g2))
    assert len(cf_list(graph(55, e1 + e2))) == t1 + t2
    # relabelling maps the triangle set onto itself
    pi = np.random.default_rng(3).permutation(30)
    h = graph(30, [(int(pi[u]), int(pi[v])) for u, v in e1])
    want = sorted(tuple(sorted(int(pi[x]) for x in t)) for t in as_set(cf_list(g1)))
    assert as_set(cf_list(h)) == want


# ---------------------------------------------------------------- Example 1

def load_example1():
    edges, cost, vals = [], [], {}
    with open(os.path.join(GOLDEN, "example1.txt")) as f:
        for line in f:
            p = line.split()
            if not p or p[0].startswith("#"):
                continue
            if p[0] == "edge":
                edges.append((int(p[1]) - 1, int(p[2]) - 1))
            elif p[0] == "cost":
                cost.append(tuple(int(x) for x in p[1:]))
            else:
                vals[p[0]] = int(p[1])
    return {"csr": graph(vals["n"], edges), "cost": cost, **vals}


def test_example1_costs():
    ex = load_example1()
    rp, col = ex["csr"].numpy()
    o = oracle.orient(rp, col)
    assert o.n == ex["n"] and o.m == ex["edges"]
    d = o.dplus
    r = lambda name: int(o.rank[name - 1])
    for u, v, head, mn in ex["cost"]:
        assert d[r(v)] == head and min(d[r(u)], d[r(v)]) == mn
    tail = o.tail()
    assert int((d[o.ocol] > 0).sum()) == ex["positive_head_edges"]
    assert oracle.sum_head(o) == ex["sum_head"] == 21
    assert oracle.sum_min(o) == ex["sum_min"] == 12
    # the triangle set itself (derived, not printed): three copies of two triangles
    assert as_set(oracle.list_triangles(o)) == brute_force(ex["csr"])
    assert len(brute_force(ex["csr"])) == 6
    _, probes = oracle.aot_ref(rp, col)
    assert probes == 12
    del tail


def test_example1_descending_order_does_not_fit():
    """The descending-degree reading of the orientation contradicts the example
    (its sum of minima would be 21, not 12), so the ascending reading is used."""
    ex = load_example1()
    rp, col = ex["csr"].numpy()
    n = ex["n"]
    deg = np.diff(rp)
    order = np.lexsort((np.arange(n), -deg))
    rank = np.empty(n, np.int64)
    rank[order] = np.arange(n)
    rows = np.repeat(np.arange(n), deg)
    up = rank[rows] < rank[col]
    u, v = rank[rows[up]], rank[col[up]]
    dplus = np.bincount(u, minlength=n)
    assert int(np.minimum(dplus[u], dplus[v]).sum()) == 21


# ---------------------------------------------------------------- Algorithm 3

@pytest.mark.parametrize("n,p,seed", SMALL + [(200, 0.08, 21), (300, 0.04, 22)])
def test_aot_reference_matches_cf_and_probes_equal_sum_min(n, p, seed):
    g = random_graph(n, p, seed)
    rp, col = g.numpy()
    tri, probes = oracle.aot_ref(rp, col)
    o = oracle.orient(rp, col)
    assert as_set(tri) == as_set(oracle.list_triangles(o))
    assert len(set(map(tuple, tri.tolist()))) == len(tri)     # each exactly once
    assert probes == oracle.sum_min(o)


def test_tie_break_is_needed():
    """Two triangles; the one whose pivot edge joins two vertices of equal
    out-degree is lost when ties are not broken by id."""
    g = graph(5, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 4)])
    tri, _ = oracle.aot_ref(*g.numpy(), tie_break=True)
    assert as_set(tri) == [(0, 1, 2), (0, 1, 3)] == brute_force(g)
    lost, _ = oracle.aot_ref(*g.numpy(), tie_break=False)
    assert len(lost) == 1


def cf_on(n, mod):
    """The plain oriented lister on arbitrary out-lists: common out-neighbours
    of the two ends of every arc.  A triangle is found iff it is not cyclic."""
    return {tuple(sorted((u, v, w))) for u in range(n) for v in mod[u] for w in mod[u] & mod[v]}


def naive_reversal(n, edges):
    """The idea Section 1 (Challenges) and Section 3.1 reject: orient by
    (degree, id), reverse every edge whose head has the larger out-degree, and
    run the plain oriented lister (common out-neighbours of each edge's ends)
    on the result.  Returns its triangle set and the modified out-lists."""
    adj = [set() for _ in range(n)]
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    key = [(len(adj[v]), v) for v in range(n)]
    out = [{v for v in adj[u] if key[v] > key[u]} for u in range(n)]
    dplus = [len(o) for o in out]
    mod = [set() for _ in range(n)]
    for u in range(n):
        for v in out[u]:
            (mod[v] if dplus[v] > dplus[u] else mod[u]).add(v if dplus[v] <= dplus[u] else u)
    return cf_on(n, mod), mod


def sequential_reversal(n, edges):
    """The same idea with edges flipped one at a time, in row order, each
    judged by the out-degrees as they stand after the earlier flips."""
    adj = [set() for _ in range(n)]
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    key = [(len(adj[v]), v) for v in range(n)]
    mod = [{v for v in adj[u] if key[v] > key[u]} for u in range(n)]
    for u in range(n):
        for v in sorted(mod[u]):
            if v in mod[u] and len(mod[v]) > len(mod[u]):
                mod[u].discard(v)
                mod[v].add(u)
    return cf_on(n, mod)


def test_reversal_by_out_degree_is_another_total_order():
    """Section 1 (Challenges) and Section 3.1 reject reversing the edges
    whose head has the larger out-degree, since cyclic triangles would be
    missed.  Reversing every such edge at once by the orientation's deg+
    points every edge from larger to smaller deg+ (ties: up the order), which
    is itself a total order: acyclic, and no triangle is lost.  A cycle needs
    a reversal that follows no single order, like one flipped edge of the
    paper's figure; that triangle is then lost.  AOT reverses nothing: it
    keeps the orientation and only chooses which side to probe."""
    for seed in range(40):
        g = random_graph(14 + seed % 10, 0.35, 700 + seed)
        rp, col = g.numpy()
        rows = np.repeat(np.arange(g.n), np.diff(rp))
        edges = [(int(a), int(b)) for a, b in zip(rows, col) if a < b]
        got, mod = naive_reversal(g.n, edges)
        o = oracle.orient(rp, col)
        dplus = np.zeros(g.n, np.int64)
        dplus[o.perm] = o.dplus
        # every arc goes down the order (deg+ descending, then rank ascending)
        for u in range(g.n):
            for v in mod[u]:
                assert (-dplus[u], o.rank[u]) < (-dplus[v], o.rank[v])
        assert sorted(got) == brute_force(g)
        assert sorted(sequential_reversal(g.n, edges)) == brute_force(g)
    # one flipped edge of a transitive triangle: the cycle u -> x -> v -> u
    u, x, v = 0, 1, 2
    mod = [{x}, {v}, {u}]
    assert cf_on(3, mod) == set()
    assert cf_on(3, [{x, v}, {v}, set()]) == {(0, 1, 2)}


# ---------------------------------------------------------------- digests

def test_fingerprint_and_digest_agree():
    g = random_graph(150, 0.12, 31)
    rp, col = g.numpy()
    o = oracle.orient(rp, col)
    tri = oracle.list_triangles(o)
    fp, tv = oracle.fingerprint(tri, o.n)
    t, fp2, tv2 = oracle.list_digest(o)
    assert t == len(tri) and fp == fp2 and np.array_equal(tv, tv2)
    # order independence
    fp3, _ = oracle.fingerprint(tri[::-1].copy())
    assert fp3 == fp
    # split digests combine: sum adds mod 2^64, xor xors
    cut = o.n // 2
    ta, fa, _ = oracle.list_digest(o, 0, cut)
    tb, fb, _ = oracle.list_digest(o, cut, o.n)
    assert ta + tb == t
    assert ((fa[0] + fb[0]) % 2**64, fa[1] ^ fb[1]) == fp
    # a single changed triangle changes both words
    bad = tri.copy()
    bad[0, 2] += 1
    fpb, _ = oracle.fingerprint(bad)
    assert fpb[0] != fp[0] and fpb[1] != fp[1]


def test_parallel_ranges_give_the_same_list():
    g = inputs.workload("er2000")
    rp, col = g.numpy()
    o = oracle.orient(rp, col)
    a = oracle.list_triangles(o)
    b = oracle.list_triangles_parallel(o, threads=5)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("n,p,seed", SMALL + [(300, 0.05, 41)])
def test_in_lists_transpose_the_out_lists(n, p, seed):
    g = random_graph(n, p, seed)
    rp, col = g.numpy()
    o = oracle.orient(rp, col)
    irow, icol, ieid = oracle.in_lists(o)
    tail = o.tail()
    assert irow[-1] == o.m
    A = dense(g)
    for r in range(n):
        ins = icol[irow[r]:irow[r + 1]]
        # the neighbours of perm[r] that rank below r, in ascending rank
        below = sorted(o.rank[np.nonzero(A[o.perm[r]])[0]].tolist())
        assert ins.tolist() == [x for x in below if x < r]
        for x, e in zip(ins.tolist(), ieid[irow[r]:irow[r + 1]].tolist()):
            assert tail[e] == x and o.ocol[e] == r


# ---------------------------------------------------------------- large-graph helpers

@pytest.mark.parametrize("n,p,seed", SMALL)
def test_vertex_triangles_equal_a3_diagonal(n, p, seed):
    """t(v) = (A^3)_vv / 2 (closed walks of length 3 through v, each triangle
    walked in two directions)."""
    g = random_graph(n, p, seed)
    rp, col = g.numpy()
    A = dense(g)
    want = np.diag(A @ A @ A) // 2
    got = oracle.vertex_triangles(rp, col, np.arange(n))
    assert np.array_equal(got, want)
    assert got.sum() == 3 * len(brute_force(g))


@pytest.mark.parametrize("n", [5, 6, 9, 20])
def test_vertex_triangles_closed_forms(n):
    # wheel: hub in n-1 triangles, every rim vertex in 2
    rp, col = wheel(n).numpy()
    t = oracle.vertex_triangles(rp, col, np.arange(n))
    assert t[0] == n - 1 and np.all(t[1:] == 2)
    # K_n: every vertex in C(n-1, 2)
    rp, col = graph(n, itertools.combinations(range(n), 2)).numpy()
    assert np.all(oracle.vertex_triangles(rp, col, np.arange(n)) == math.comb(n - 1, 2))
    # a tree has none
    rp, col = graph(n, [(i, (i - 1) // 2) for i in range(1, n)]).numpy()
    assert np.all(oracle.vertex_triangles(rp, col, np.arange(n)) == 0)


@pytest.mark.parametrize("g", [
    lambda: inputs.rmat(13, 16, 3), lambda: inputs.erdos_renyi(2000, 0.01, 1),
    lambda: inputs.chung_lu(20000, 20.0, 2.1, 2000.0, 5), lambda: graph(0, []),
    lambda: graph(7, []), lambda: random_graph(40, 0.5, 9)])
@pytest.mark.parametrize("threads", [1, 3, 8])
def test_threaded_orientation_and_sum_min(g, threads):
    """Range-by-range orientation on threads equals the one-pass orientation;
    the ranged sum of minima equals the one-pass sum."""
    csr = g()
    rp, col = csr.numpy()
    a = oracle.orient(rp, col)
    b = oracle.orient_threaded(rp, col, threads=threads)
    assert np.array_equal(a.perm, b.perm) and np.array_equal(a.rank, b.rank)
    assert np.array_equal(a.orow, b.orow) and np.array_equal(a.ocol, b.ocol)
    assert oracle.sum_min_threaded(b, threads=threads) == oracle.sum_min(a)


# ---------------------------------------------------------------- core order

def brute_degeneracy(n, edges):
    """max over vertex subsets S of the least degree inside S."""
    adj = [0] * n
    for a, b in edges:
        adj[a] |= 1 << b
        adj[b] |= 1 << a
    best = 0
    for s in range(1, 1 << n):
        low = min(bin(adj[v] & s).count("1") for v in range(n) if s >> v & 1)
        best = max(best, low)
    return best


@pytest.mark.parametrize("seed", range(12))
def test_core_order_reaches_the_degeneracy(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(4, 11))
    p = float(rng.choice([0.2, 0.4, 0.6]))
    edges = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
    rp, col = graph(n, edges).numpy()
    rnd, k, d = oracle.core_rounds(rp, col)
    assert d == brute_degeneracy(n, edges)
    o = oracle.orient(rp, col, "core")
    # the first vertex of the densest core has all its core neighbours after it,
    # so no order does better than the degeneracy; the core order reaches it
    assert (o.dplus.max() if n else 0) == d
    assert sorted(set(rnd.tolist())) == list(range(k))      # every sub-round removes some
    # the order is (round, id)
    assert np.array_equal(o.perm, np.lexsort((np.arange(n), rnd)))


def test_core_order_hand_examples():
    # path 0-1-2-3-4: the ends go first, then their neighbours, then the middle
    rp, col = graph(5, [(0, 1), (1, 2), (2, 3), (3, 4)]).numpy()
    rnd, k, d = oracle.core_rounds(rp, col)
    assert rnd.tolist() == [0, 1, 2, 1, 0] and (k, d) == (3, 1)
    assert oracle.orient(rp, col, "core").perm.tolist() == [0, 4, 1, 3, 2]
    # star: leaves at level 1, then the hub (degree 0 by then)
    rp, col = graph(6, [(0, i) for i in range(1, 6)]).numpy()
    rnd, k, d = oracle.core_rounds(rp, col)
    assert rnd.tolist() == [1, 0, 0, 0, 0, 0] and (k, d) == (2, 1)
    # K_n: one sub-round at level n - 1, so the order is the id order
    rp, col = graph(7, itertools.combinations(range(7), 2)).numpy()
    rnd, k, d = oracle.core_rounds(rp, col)
    assert rnd.tolist() == [0] * 7 and (k, d) == (1, 6)
    # empty graph
    rnd, k, d = oracle.core_rounds(np.zeros(1, np.int64), np.zeros(0, np.int32))
    assert (len(rnd), k, d) == (0, 0, 0)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_core_order_lists_the_same_set(seed):
    """Any total order lists every triangle exactly once (Section 3.2)."""
    csr = inputs.rmat(11, 16, seed)
    rp, col = csr.numpy()
    a = oracle.orient(rp, col)
    b = oracle.orient(rp, col, "core")
    ta, tb = oracle.list_triangles(a), oracle.list_triangles(b)
    tb = tb[np.lexsort((tb[:, 2], tb[:, 1], tb[:, 0]))]
    ta = ta[np.lexsort((ta[:, 2], ta[:, 1], ta[:, 0]))]
    assert np.array_equal(ta, tb)
    assert int(oracle.edge_counts(b).sum()) == len(ta)
    _, _, d = oracle.core_rounds(rp, col)
    assert b.dplus.max() == d <= a.dplus.max()


# ---------------------------------------------------------------- labels by id

@pytest.mark.parametrize("n,p,seed", SMALL + [(300, 0.05, 99)])
def test_orientation_by_id_keeps_the_edges_in_id_order(n, p, seed):
    """Labels by id (AOT-randomOrder's local order, Section 4.2): the degree
    order, computed here from scratch, still directs every edge; rows are
    indexed by id and ascending in id."""
    g = random_graph(n, p, seed)
    rp, col = g.numpy()
    o = oracle.orient(rp, col, local="id")
    assert np.array_equal(o.perm, np.arange(n)) and np.array_equal(o.rank, np.arange(n))
    deg = np.diff(rp)
    key = deg.astype(np.int64) * (n + 1) + np.arange(n)        # (degree, id)
    rows = np.repeat(np.arange(n), deg)
    up = key[rows] < key[col]
    want = sorted(zip(rows[up].tolist(), col[up].tolist()))
    assert list(zip(o.tail().tolist(), o.ocol.tolist())) == want
    assert o.m == g.m


@pytest.mark.parametrize("n,p,seed", SMALL + [(60, 0.3, 61)])
def test_list_by_id_is_the_brute_force_set_in_edge_order(n, p, seed):
    g = random_graph(n, p, seed)
    rp, col = g.numpy()
    o = oracle.orient(rp, col, local="id")
    tri = oracle.list_triangles(o)
    assert as_set(tri) == brute_force(g)
    # Sigma min does not depend on the labels
    deg = np.diff(rp)
    key = deg.astype(np.int64) * (n + 1) + np.arange(n)
    rows = np.repeat(np.arange(n), deg)
    up = key[rows] < key[col]
    dplus = np.bincount(rows[up], minlength=n)
    assert oracle.sum_min(o) == int(np.minimum(dplus[rows[up]], dplus[col[up]]).sum())
    # per-edge counts from the oriented adjacency matrix
    D = np.zeros((n, n), np.int64)
    t = o.tail()
    D[t, o.ocol] = 1
    cnt = oracle.edge_counts(o)
    assert np.array_equal(cnt, (D[t] * D[o.ocol]).sum(1) if o.m else cnt)
    # order: edge by edge, each triangle holds both ends, third vertex ascending
    off = np.concatenate([[0], np.cumsum(cnt)])
    for e in range(o.m):
        seg = tri[off[e]:off[e + 1]].tolist()
        third = []
        for row in seg:
            assert t[e] in row and o.ocol[e] in row
            third.append([x for x in row if x not in (t[e], o.ocol[e])][0])
        assert third == sorted(set(third))


def test_orientation_by_id_with_the_core_order():
    csr = inputs.rmat(10, 16, 5)
    rp, col = csr.numpy()
    b = oracle.orient(rp, col, "core", local="id")
    a = oracle.orient(rp, col, "core")
    # the same directed edges, named by original id
    ea = sorted(zip(a.perm[a.tail()].tolist(), a.perm[a.ocol].tolist()))
    eb = list(zip(b.tail().tolist(), b.ocol.tolist()))
    assert eb == ea
    assert oracle.sum_min(a) == oracle.sum_min(b)


# ---------------------------------------------------------------- edge support

@pytest.mark.parametrize("seed", range(6))
def test_edge_support_is_a_squared(seed):
    """Triangles through edge {u,v} = (A^2)_uv; they sum to 3T."""
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(5, 60))
    p = float(rng.choice([0.1, 0.3, 0.6]))
    A = np.triu(rng.random((n, n)) < p, 1)
    A = (A | A.T).astype(np.int64)
    iu, ju = np.nonzero(np.triu(A, 1))
    rp, col = graph(n, zip(iu.tolist(), ju.tolist())).numpy()
    o = oracle.orient(rp, col)
    sup = oracle.edge_support(rp, col, o)
    A2 = A @ A
    u = o.perm[o.tail()]
    v = o.perm[o.ocol]
    assert np.array_equal(sup, A2[u, v])
    assert int(sup.sum()) == 3 * len(oracle.list_triangles(o)) == int(np.trace(A2 @ A)) // 2


def test_edge_support_closed_forms():
    # K_n: every edge lies in n - 2 triangles
    rp, col = graph(9, itertools.combinations(range(9), 2)).numpy()
    o = oracle.orient(rp, col)
    assert set(oracle.edge_support(rp, col, o).tolist()) == {7}
    # wheel with hub 0 and rim 1..8: spokes lie in 2 triangles, rim edges in 1
    n = 9
    e = [(0, i) for i in range(1, n)] + [(i, i % (n - 1) + 1) for i in range(1, n)]
    rp, col = graph(n, e).numpy()
    o = oracle.orient(rp, col)
    sup = oracle.edge_support(rp, col, o)
    spoke = (o.perm[o.tail()] == 0) | (o.perm[o.ocol] == 0)
    assert set(sup[spoke].tolist()) == {2} and set(sup[~spoke].tolist()) == {1}
    # the core order relabels, the support of each undirected edge stays
    oc = oracle.orient(rp, col, "core")
    key = lambda oo: {tuple(sorted(t)): s for t, s in zip(
        zip(oo.perm[oo.tail()].tolist(), oo.perm[oo.ocol].tolist()),
        oracle.edge_support(rp, col, oo).tolist())}
    assert key(o) == key(oc)
