"""Property tests of the oracle on random simple graphs (hypothesis): the
list equals brute-force enumeration, and the invariants that hold for every
graph -- counts add up, disjoint unions add, relabelling changes nothing, the
orientation is acyclic with m edges, any total order lists the same set."""

import itertools

import numpy as np
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from paper_2006_11494_amd import inputs

SETTINGS = settings(max_examples=60, deadline=None,
                    suppress_health_check=[HealthCheck.too_slow])


@st.composite
def graphs(draw, max_n=14):
    """(n, sorted list of distinct undirected edges (a < b))."""
    n = draw(st.integers(0, max_n))
    pairs = list(itertools.combinations(range(n), 2))
    if not pairs:
        return n, []
    keep = draw(st.lists(st.booleans(), min_size=len(pairs), max_size=len(pairs)))
    return n, [p for p, k in zip(pairs, keep) if k]


def csr(n, edges):
    return inputs.csr_from_edges_np(n, edges).numpy()


def brute(n, edges):
    es = set(edges)
    return sorted((a, b, c) for a, b, c in itertools.combinations(range(n), 3)
                  if (a, b) in es and (a, c) in es and (b, c) in es)


def sorted_list(tri):
    return sorted(map(tuple, np.asarray(tri).tolist()))


@SETTINGS
@given(graphs())
def test_list_is_the_brute_force_set_and_counts_add_up(g):
    n, edges = g
    rp, col = csr(n, edges)
    o = oracle.orient(rp, col)
    tri = oracle.list_triangles(o)
    want = brute(n, edges)
    assert sorted_list(tri) == want
    assert len(tri) == len(set(map(tuple, np.asarray(tri).tolist())))      # each once
    assert int(oracle.edge_counts(o).sum()) == len(want)
    if n:
        (_, _), tv = oracle.fingerprint(tri, n)
        assert int(np.asarray(tv, dtype=np.int64).sum()) == 3 * len(want)
    # oriented: m edges, each from a lower to a higher rank (so acyclic), rows sorted
    assert o.m == len(edges)
    assert np.all(o.ocol > o.tail()) if o.m else True
    for r in range(o.n):
        row = o.ocol[o.orow[r]:o.orow[r + 1]]
        assert np.all(np.diff(row) > 0)
    # every cost is at least the adaptive one
    assert oracle.sum_min(o) <= oracle.sum_head(o) <= oracle.sum_merge(o)


@SETTINGS
@given(graphs())
def test_id_labels_list_the_same_set_with_the_same_edges(g):
    """Original ids as labels (AOT-randomOrder's local order): the same
    directed edges, named by id, the brute-force set, and the same costs."""
    n, edges = g
    rp, col = csr(n, edges)
    a = oracle.orient(rp, col)
    b = oracle.orient(rp, col, local="id")
    ea = sorted(zip(a.perm[a.tail()].tolist(), a.perm[a.ocol].tolist())) if a.m else []
    assert list(zip(b.tail().tolist(), b.ocol.tolist())) == ea
    assert sorted_list(oracle.list_triangles(b)) == brute(n, edges)
    assert oracle.sum_min(a) == oracle.sum_min(b)
    assert oracle.sum_head(a) == oracle.sum_head(b)
    assert oracle.sum_merge(a) == oracle.sum_merge(b)


@SETTINGS
@given(graphs(max_n=9), graphs(max_n=9))
def test_disjoint_union_adds(g1, g2):
    (n1, e1), (n2, e2) = g1, g2
    union = e1 + [(a + n1, b + n1) for a, b in e2]
    rp, col = csr(n1 + n2, union)
    t = len(oracle.list_triangles(oracle.orient(rp, col)))
    assert t == len(brute(n1, e1)) + len(brute(n2, e2))


@SETTINGS
@given(graphs(), st.randoms(use_true_random=False))
def test_relabelling_changes_nothing(g, rnd):
    n, edges = g
    perm = list(range(n))
    rnd.shuffle(perm)
    relabelled = sorted(tuple(sorted((perm[a], perm[b]))) for a, b in edges)
    rp, col = csr(n, relabelled)
    tri = oracle.list_triangles(oracle.orient(rp, col))
    back = sorted(tuple(sorted(perm[x] for x in t)) for t in brute(n, edges))
    assert sorted_list(tri) == back


@SETTINGS
@given(graphs())
def test_core_order_lists_the_same_set_and_support_is_a_squared(g):
    n, edges = g
    rp, col = csr(n, edges)
    od = oracle.orient(rp, col)
    oc = oracle.orient(rp, col, "core")
    assert sorted_list(oracle.list_triangles(oc)) == sorted_list(oracle.list_triangles(od))
    _, _, d = oracle.core_rounds(rp, col)
    assert (int(oc.dplus.max()) if oc.m else 0) == d
    A = np.zeros((n, n), np.int64)
    for a, b in edges:
        A[a, b] = A[b, a] = 1
    A2 = A @ A
    for o in (od, oc):
        sup = oracle.edge_support(rp, col, o)
        assert np.array_equal(sup, A2[o.perm[o.tail()], o.perm[o.ocol]])
