"""GPU parity of the probe strategies: the adaptive rule of Algorithm 3, the
fixed orientation whose cost is kClist's (Section 2.3), Algorithm 1's merge
intersections (Section 2.2) and the CF-Hash remark's per-edge probing.  Each
strategy must give the oracle's per-edge counts and list byte for byte, and
report the oracle's cost of that strategy as its probe count."""

import os
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2006_11494_amd import aot, inputs
from test_gpu_parity import SMALL, graph, need_gpu, table

pytestmark = pytest.mark.gpu

DEV = "cuda"
S = aot.STRATEGIES


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def D(strategy, heavy_min=0, tiles=None, arm=0, mode=aot.AOT_DISPATCH_TABLE):
    return aot.Dispatch(mode, heavy_min, table(tiles, arm), None, S[strategy])


# (strategy, dispatch): every path each strategy can take
CASES = {
    "head_plain": ("head", aot.Dispatch(strategy=S["head"])),
    "head_heavy_bitmap": ("head", D("head", 1, arm=0)),
    "head_heavy_hash": ("head", D("head", 1, arm=1)),
    "head_heavy_global": ("head", D("head", 1, arm=2)),
    "head_heavy_sorted": ("head", D("head", 1, arm=3)),
    "head_light_tile4": ("head", D("head", 2**30, [4] * 8)),
    "head_light_tile64": ("head", D("head", 2**30, [64] * 8)),
    "head_mixed": ("head", D("head", 8, [8, 16, 32, 4, 64, 8, 16, 32], 1)),
    "merge_plain": ("merge", aot.Dispatch(strategy=S["merge"])),
    "merge_tile4": ("merge", D("merge", 0, [4] * 8)),
    "merge_tile64": ("merge", D("merge", 0, [64] * 8)),
    "merge_mixed": ("merge", D("merge", 0, [16, 64, 4, 32, 8, 64, 16, 4])),
    "per_edge_plain": ("per_edge", aot.Dispatch(strategy=S["per_edge"])),
    "per_edge_tile4": ("per_edge", D("per_edge", 0, [4] * 8)),
    "per_edge_tile64": ("per_edge", D("per_edge", 0, [64] * 8)),
}


def cost(o_ref, strategy):
    return {"aot": oracle.sum_min, "per_edge": oracle.sum_min, "head": oracle.sum_head,
            "merge": oracle.sum_merge}[strategy](o_ref)


def check_strategies(csr, name, cases=CASES, windows=True, local="rank"):
    need_gpu()
    rp, col = csr.numpy()
    o_ref = oracle.orient(rp, col, local=local)
    cnt_ref = oracle.edge_counts(o_ref)
    T = int(cnt_ref.sum())
    tri_ref = oracle.list_triangles(o_ref)
    g = csr.to(DEV)
    o = aot.orient(g.rowptr, g.col, local=local)
    for cname, (strategy, d) in cases.items():
        say(f"[gpu] strategy {name} {cname}")
        c = aot.count(o, d)
        assert (c.T, c.probes) == (T, cost(o_ref, strategy)), cname
        assert np.array_equal(np.diff(c.tri_off.cpu().numpy()), cnt_ref), cname
        # the write pass takes the count's strategy, whatever it is given
        for dd in (d, None):
            tri = aot.list_triangles(o, c, dispatch=dd).cpu().numpy()
            assert np.array_equal(tri, tri_ref), cname
        if windows and T > 1:
            rng = np.random.default_rng(T)
            for first in sorted({0, T - 1, *rng.integers(0, T, 3).tolist()}):
                for count in (1, 5, max(1, T // 3)):
                    got = aot.list_triangles(o, c, first=int(first), count=count).cpu().numpy()
                    assert np.array_equal(got, tri_ref[first:first + count]), (cname, first)
    return o, o_ref, tri_ref


@pytest.mark.parametrize("name", ["empty", "one_edge", "triangle", "k40", "tiebreak",
                                  "wheel50", "star300", "k_100_200", "rand_b", "rand_c",
                                  "dense_c"])
def test_small_graphs(name):
    check_strategies(SMALL[name], name)


def test_example1_costs():
    """Example 1 (Section 3.2): the fixed orientation probes the heads' lists,
    21 entries; the adaptive rule 12."""
    edges = []
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "example1.txt")
    for line in open(path):
        p = line.split()
        if p and p[0] == "edge":
            edges.append((int(p[1]) - 1, int(p[2]) - 1))
    need_gpu()
    o, o_ref, _ = check_strategies(graph(14, edges), "example1")
    assert aot.count(o, aot.Dispatch(strategy=S["head"])).probes == 21
    assert aot.count(o).probes == 12


def test_er2000():
    check_strategies(inputs.workload("er2000"), "er2000")


def test_rmat14():
    check_strategies(inputs.rmat(14, 16, 21), "rmat14")


def test_chung_lu_small():
    check_strategies(inputs.chung_lu(60000, 20.0, 2.1, 3000.0, 22), "chunglu60k",
                     windows=False)


@pytest.mark.parametrize("name", ["rand_b", "dense_c", "wheel50", "rmat14"])
def test_labels_by_id(name):
    """Every strategy on the id-labelled orientation (AOT-randomOrder's local
    order): same counts, costs and list as the oracle's id-labelled graph."""
    csr = SMALL[name] if name in SMALL else inputs.rmat(14, 16, 21)
    check_strategies(csr, name + "_by_id", local="id", windows=name != "rmat14")


def test_long_lists_merge():
    """Rows of several thousand out-neighbours: long merges split over 64 lanes."""
    a, b = 2100, 2200
    u = torch.arange(a, dtype=torch.int64).repeat_interleave(b)
    v = a + torch.arange(b, dtype=torch.int64).repeat(a)
    # plus a clique on 40 of the 2100 side: each of the 2200 others points at
    # all 2100 and closes a triangle with every clique edge (1.7 M in all)
    cu, cv = torch.triu_indices(40, 40, 1)
    csr = inputs.csr_from_pairs(a + b, torch.cat([u, cu]), torch.cat([v, cv]))
    check_strategies(csr, "k_2100_2200_k40",
                     cases={k: CASES[k] for k in ("merge_plain", "merge_tile4", "head_plain",
                                                  "per_edge_plain")}, windows=False)


@pytest.mark.parametrize("strategy", ["head", "merge", "per_edge"])
def test_digest_and_vertex_counts(strategy):
    need_gpu()
    csr = inputs.rmat(13, 16, 33)
    rp, col = csr.numpy()
    tri = oracle.list_triangles(oracle.orient(rp, col))
    (f1, f2), tv = oracle.fingerprint(tri, csr.n)
    g = csr.to(DEV)
    o = aot.orient(g.rowptr, g.col)
    c = aot.count(o, aot.Dispatch(strategy=S[strategy]))
    (t, s, x), vc = aot.digest(o, c)
    assert (t, s, x) == (len(tri), f1, f2)
    assert np.array_equal(vc.cpu().numpy().astype(np.uint64), tv)


def test_strategy_is_remembered_per_workspace():
    """A later count on another workspace does not change what an earlier
    one's write pass does."""
    need_gpu()
    csr = inputs.rmat(12, 16, 34)
    rp, col = csr.numpy()
    tri_ref = oracle.list_triangles(oracle.orient(rp, col))
    g = csr.to(DEV)
    o = aot.orient(g.rowptr, g.col)
    c_merge = aot.count(o, aot.Dispatch(strategy=S["merge"]))
    c_head = aot.count(o, aot.Dispatch(strategy=S["head"]))
    c_plain = aot.count(o)
    for c in (c_merge, c_head, c_plain):
        assert np.array_equal(aot.list_triangles(o, c).cpu().numpy(), tri_ref)
