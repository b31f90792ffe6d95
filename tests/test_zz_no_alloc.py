"""aot_count_noalloc, the count pass for callers that cannot allocate device
memory (its workspace is the library's fixed scratch), against aot_count with
a workspace of its own: the same tri_off, T and probe count -- and the
oracle's T and probe count -- on two calls in a row, the second on a smaller
graph, so the scratch's previous contents must not leak into the result."""

import numpy as np
import pytest
import torch

import oracle
from paper_2006_11494_amd import aot, inputs

pytestmark = pytest.mark.gpu


def test_count_noalloc_matches_count():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    for csr in (inputs.rmat(16, 16, 41), inputs.rmat(12, 8, 42), inputs.workload("er2000")):
        rp, col = csr.numpy()
        ref = oracle.orient(rp, col)
        g = csr.to("cuda")
        o = aot.orient(g.rowptr, g.col)
        assert aot.count_workspace(o.n, o.m) <= aot.AOT_NOALLOC_SCRATCH_BYTES
        c = aot.count(o)
        tri_off = torch.full((o.m + 1,), -1, dtype=torch.int64, device="cuda")
        T, probes = aot.count_noalloc(o, tri_off)
        assert (T, probes) == (c.T, c.probes) == (int(oracle.edge_counts(ref).sum()),
                                                  oracle.sum_min(ref)), csr.name
        assert torch.equal(tri_off, c.tri_off), csr.name
        # and with a table dispatch that forces the hash arm and 4-lane tiles
        table = [4 << 8] * 8 + [0] * 8 + [1] * 16
        tri_off.fill_(-1)
        d = aot.Dispatch(aot.AOT_DISPATCH_TABLE, 32, table)
        assert aot.count_noalloc(o, tri_off, d) == (T, probes)
        assert torch.equal(tri_off, c.tri_off), csr.name


def test_count_noalloc_rejects_a_graph_beyond_the_scratch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    g = inputs.rmat(18, 32, 43).to("cuda")
    o = aot.orient(g.rowptr, g.col)
    assert aot.count_workspace(o.n, o.m) > aot.AOT_NOALLOC_SCRATCH_BYTES
    tri_off = torch.empty(o.m + 1, dtype=torch.int64, device="cuda")
    with pytest.raises(aot.AotError) as e:
        aot.count_noalloc(o, tri_off)
    assert e.value.status == -7
    # the library still counts graphs that fit afterwards
    small = inputs.rmat(10, 8, 44).to("cuda")
    os_ = aot.orient(small.rowptr, small.col)
    t2 = torch.empty(os_.m + 1, dtype=torch.int64, device="cuda")
    assert aot.count_noalloc(os_, t2) == (aot.count(os_).T, aot.count(os_).probes)
