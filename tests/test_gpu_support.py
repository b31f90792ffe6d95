"""GPU parity of aot_support: triangles through every oriented edge (the
A^2 entry of its endpoints, which the oracle merges from the input's rows,
independently of any listing), through every vertex, and the list digest --
for every probe arm, tile and strategy, and on the core order."""

import sys

import numpy as np
import pytest

import oracle
from paper_2006_11494_amd import aot, inputs
from test_gpu_parity import DISPATCHES, SMALL, need_gpu

pytestmark = pytest.mark.gpu

S = aot.STRATEGIES
CASES = dict(DISPATCHES)
CASES.update({
    "head": aot.Dispatch(strategy=S["head"]),
    "merge": aot.Dispatch(strategy=S["merge"]),
    "per_edge": aot.Dispatch(strategy=S["per_edge"]),
})


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def check_support(csr, name, cases=CASES, order="degree", local="rank"):
    need_gpu()
    rp, col = csr.numpy()
    o_ref = oracle.orient(rp, col, order, local)
    sup_ref = oracle.edge_support(rp, col, o_ref)
    tri = oracle.list_triangles(o_ref)
    (f1, f2), tv = oracle.fingerprint(tri, csr.n)
    assert int(sup_ref.sum()) == 3 * len(tri)
    g = csr.to("cuda")
    o = aot.orient(g.rowptr, g.col, order=order, local=local)
    for cname, d in cases.items():
        say(f"[gpu] support {name} {order} {local} {cname}")
        c = aot.count(o, d)
        es, vc, dig = aot.support(o, c)
        assert np.array_equal(es.cpu().numpy(), sup_ref), cname
        assert dig == (len(tri), f1, f2), cname
        if csr.n:
            assert np.array_equal(vc.cpu().numpy().astype(np.uint64), tv), cname
    # a second call overwrites, it does not add
    es2, _, _ = aot.support(o, c, vertex_counts=False)
    assert np.array_equal(es2.cpu().numpy(), sup_ref)


@pytest.mark.parametrize("name", ["empty", "one_edge", "triangle", "k40", "tiebreak", "wheel50",
                                  "star300", "k_100_200", "rand_b", "rand_c", "dense_c"])
def test_small_graphs(name):
    check_support(SMALL[name], name)


def test_er2000():
    check_support(inputs.workload("er2000"), "er2000")


@pytest.mark.parametrize("name", ["tiebreak", "wheel50", "rand_b", "dense_c", "rmat13"])
def test_id_labels(name):
    """Support, vertex counts and digest on the id-labelled orientation
    (AOT-randomOrder's local order), every arm, tile and strategy."""
    csr = SMALL[name] if name in SMALL else inputs.rmat(13, 16, 34)
    check_support(csr, name, local="id")


def test_rmat14():
    check_support(inputs.rmat(14, 16, 21), "rmat14")


def test_chung_lu_small():
    check_support(inputs.chung_lu(60000, 20.0, 2.1, 3000.0, 22), "chunglu60k")


def test_core_order():
    check_support(inputs.rmat(13, 16, 36), "rmat13",
                  cases={k: CASES[k] for k in ("plain", "all_heavy_hash", "head", "merge")},
                  order="core")


def test_clustering_coefficients():
    """Local clustering 2 t(v) / (deg(v) (deg(v) - 1)) from the vertex counts."""
    need_gpu()
    csr = inputs.rmat(12, 16, 37)
    rp, col = csr.numpy()
    deg = np.diff(rp)
    tri = oracle.list_triangles(oracle.orient(rp, col))
    _, tv = oracle.fingerprint(tri, csr.n)
    g = csr.to("cuda")
    o = aot.orient(g.rowptr, g.col)
    _, vc, _ = aot.support(o, aot.count(o))
    vc = vc.cpu().numpy()
    with np.errstate(divide="ignore", invalid="ignore"):
        cc = np.where(deg > 1, 2.0 * vc / (deg * (deg - 1.0)), 0.0)
        cc_ref = np.where(deg > 1, 2.0 * tv.astype(np.float64) / (deg * (deg - 1.0)), 0.0)
    assert np.array_equal(cc, cc_ref)
    assert np.all((cc >= 0) & (cc <= 1))
