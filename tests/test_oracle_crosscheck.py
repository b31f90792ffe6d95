"""The two CPU procedures of the oracle against each other on the measured
workloads: CF (Algorithm 1, the procedure of record) and AOT (Algorithm 3, run
vertex by vertex with a |V|-flag table) must give the same triangle set, and
AOT's look-up count must equal the sum over directed edges of
min(deg+(u), deg+(v)) (Section 3.2, Time Complexity).  Where the list is too
large to compare whole, both sides digest it: count, sum and xor of the
triple hashes."""

from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_2006_11494_amd import inputs


def cf_digest(o, threads=8):
    """CF over rank ranges on host threads, digests combined (sum mod 2^64,
    xor)."""
    cuts = np.linspace(0, o.n, 8 * threads + 1).astype(np.int64)
    ranges = [(int(a), int(b)) for a, b in zip(cuts[:-1], cuts[1:]) if b > a]
    with ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(lambda ab: oracle.list_digest(o, ab[0], ab[1], per_vertex=False),
                            ranges))
    t = sum(p[0] for p in parts)
    f1 = sum(p[1][0] for p in parts) % (1 << 64)
    f2 = 0
    for p in parts:
        f2 ^= p[1][1]
    return t, (f1, f2)


def test_er2000_aot_equals_cf():
    csr = inputs.workload("er2000")
    rp, col = csr.numpy()
    tri, probes = oracle.aot_ref(rp, col)
    o = oracle.orient(rp, col)
    cf = oracle.list_triangles(o)
    assert len(tri) == len(cf) > 1000
    assert np.array_equal(np.unique(tri, axis=0), np.unique(cf, axis=0))
    assert len(np.unique(tri, axis=0)) == len(tri)           # each triangle once
    assert probes == oracle.sum_min(o)
    assert oracle.aot_ref(rp, col, digest=True) == (len(cf), oracle.fingerprint(cf)[0], probes)


@pytest.mark.slow
def test_rmat20_aot_equals_cf():
    csr = inputs.workload("rmat20")
    rp, col = csr.numpy()
    t, fp, probes = oracle.aot_ref(rp, col, digest=True)
    o = oracle.orient(rp, col)
    assert (t, fp) == cf_digest(o)
    assert t == 424_180_754
    assert probes == oracle.sum_min(o) == 1_969_802_408


@pytest.mark.slow
def test_chunglu4m_aot_equals_cf():
    csr = inputs.workload("chunglu4m")
    rp, col = csr.numpy()
    t, fp, probes = oracle.aot_ref(rp, col, digest=True)
    o = oracle.orient(rp, col)
    assert (t, fp) == cf_digest(o)
    assert probes == oracle.sum_min(o)
