"""The synthetic input generators: seeded, chunk-independent, valid simple CSR."""

import math

import numpy as np
import pytest
import torch

from paper_2006_11494_amd import inputs


def check_csr(g):
    rp, col = g.numpy()
    n = g.n
    assert rp.dtype == np.int64 and col.dtype == np.int32
    assert rp[0] == 0 and rp[-1] == col.size and np.all(np.diff(rp) >= 0)
    rows = np.repeat(np.arange(n), np.diff(rp))
    assert np.all((col >= 0) & (col < n))
    assert not np.any(rows == col)                              # no self-loops
    key = rows.astype(np.int64) * n + col
    assert np.all(np.diff(key) > 0)                             # sorted rows, no duplicates
    rkey = np.sort(col.astype(np.int64) * n + rows)
    assert np.array_equal(rkey, key)                            # symmetric


@pytest.mark.parametrize("make", [
    lambda: inputs.erdos_renyi(300, 0.05, 7),
    lambda: inputs.erdos_renyi_m(5000, 12.0, 8),
    lambda: inputs.rmat(12, 8, 9),
    lambda: inputs.chung_lu(20000, 10.0, 2.1, 500.0, 10),
    lambda: inputs.random_geometric(4000, 20.0, 11),
])
def test_valid_and_deterministic(make):
    a, b = make(), make()
    check_csr(a)
    assert torch.equal(a.rowptr, b.rowptr) and torch.equal(a.col, b.col)


def test_seed_changes_graph():
    a = inputs.rmat(10, 8, 1)
    b = inputs.rmat(10, 8, 2)
    assert a.nnz != b.nnz or not torch.equal(a.col, b.col)


def test_rmat_chunking_invariant():
    a = inputs.rmat(11, 16, 3, chunk=1 << 20)
    b = inputs.rmat(11, 16, 3, chunk=777)
    assert torch.equal(a.rowptr, b.rowptr) and torch.equal(a.col, b.col)


def test_er2000_size_is_plausible():
    g = inputs.workload("er2000")
    mean = math.comb(2000, 2) * 0.01
    sd = math.sqrt(mean * 0.99)
    assert abs(g.m - mean) < 5 * sd


def test_rgg_mean_degree():
    g = inputs.random_geometric(50000, 20.0, 5)
    assert 17.0 < 2 * g.m / g.n < 21.0       # slightly under 20 from the boundary


def test_chung_lu_skew():
    g = inputs.chung_lu(100000, 40.0, 2.1, 5000.0, 6)
    deg = np.diff(g.numpy()[0])
    assert deg.max() > 20 * deg.mean() and 25.0 < deg.mean() < 41.0


def test_batch_spec():
    spec = inputs.batch_spec(512)
    assert len(spec) == 512 and spec == inputs.batch_spec(512)
    fams = {s[0] for s in spec}
    assert fams == {"er", "rmat", "rgg"}
    for fam, a, b, _ in spec:
        if fam == "rmat":
            assert 10 <= a <= 18 and 8 <= b <= 32
        elif fam == "er":
            assert 1000 <= a <= 200000 and 8 <= b <= 64
        else:
            assert 1000 <= a <= 200000


@pytest.mark.parametrize("scale,ef,parts", [(9, 16, 2), (11, 32, 5), (12, 8, 32), (6, 4, 100)])
def test_partitioned_csr_build_is_the_same_graph(scale, ef, parts):
    a = inputs.rmat(scale, ef, 17)
    b = inputs.rmat(scale, ef, 17, parts=parts)
    assert torch.equal(a.rowptr, b.rowptr) and torch.equal(a.col, b.col)
    u = inputs.rand32(3, 1, torch.arange(5000)) % 300
    v = inputs.rand32(3, 2, torch.arange(5000)) % 300
    x = inputs.csr_from_pairs(300, u, v)
    y = inputs.csr_from_pairs_partitioned(300, u.to(torch.int32), v.to(torch.int32), parts=parts)
    assert torch.equal(x.rowptr, y.rowptr) and torch.equal(x.col, y.col)
