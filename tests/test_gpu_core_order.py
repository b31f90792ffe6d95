"""GPU parity of the core (degeneracy) order, kClist's orientation (Section
2.3), under which AOT lists the same triangles (Section 3.2): ranks, oriented
lists, in-lists, per-edge counts, probe counts and the ordered list all equal
the oracle's on the same order, for every dispatch."""

import numpy as np
import pytest

import oracle
from paper_2006_11494_amd import aot, inputs
from test_gpu_parity import DISPATCHES, SMALL, check_all, need_gpu

pytestmark = pytest.mark.gpu

FEW = {k: DISPATCHES[k] for k in ("plain", "all_heavy_hash", "all_light_tile4", "mixed")}


@pytest.mark.parametrize("name", ["empty", "isolated", "one_edge", "triangle", "k40",
                                  "tiebreak", "wheel50", "star300", "k_100_200", "rand_a",
                                  "rand_c", "dense_c"])
def test_small_graphs(name):
    check_all(SMALL[name], name, order="core")


def test_er2000():
    check_all(inputs.workload("er2000"), "er2000", dispatches=FEW, order="core")


def test_rmat14():
    csr = inputs.rmat(14, 16, 21)
    o = check_all(csr, "rmat14", order="core")
    rp, col = csr.numpy()
    _, _, d = oracle.core_rounds(rp, col)
    assert int((o.rowptr[1:] - o.rowptr[:-1]).max()) == d


def test_chung_lu_small():
    check_all(inputs.chung_lu(60000, 20.0, 2.1, 3000.0, 22), "chunglu60k", dispatches=FEW,
              windows=False, order="core")


def test_strategies_on_the_core_order():
    need_gpu()
    csr = inputs.rmat(13, 16, 35)
    rp, col = csr.numpy()
    ref = oracle.orient(rp, col, "core")
    tri_ref = oracle.list_triangles(ref)
    g = csr.to("cuda")
    o = aot.orient(g.rowptr, g.col, order="core")
    for name, sid in aot.STRATEGIES.items():
        c = aot.count(o, aot.Dispatch(strategy=sid))
        want = {"head": oracle.sum_head, "merge": oracle.sum_merge}.get(name, oracle.sum_min)
        assert (c.T, c.probes) == (len(tri_ref), want(ref)), name
        assert np.array_equal(aot.list_triangles(o, c).cpu().numpy(), tri_ref), name
