"""The large configuration: R-MAT scale 26, edge factor 32 (2^31 tuples; about
2e9 edges, so the symmetric input has more than INT32_MAX entries), generated
and counted on the device, listed in windows streamed to pinned host memory.

Its list (a few times 1e11 triangles) is far beyond what the CPU oracle can
store, so parity rests on everything the oracle computes at this size:
  * the whole orientation (ranks, out-list offsets, out-lists), exactly;
  * the probe count sum of min(deg+), exactly;
  * per-edge triangle counts at 200,000 random edges and at edges of the
    heaviest owners, exactly;
  * complete triangle lists of rank ranges at several depths of the order,
    exactly (the device windows that hold them, streamed to the host);
  * the digest of the whole list -- T, the sum and xor of the triple hashes
    and the triangles through every vertex (SHA-256 of the array, its sum and
    sampled entries) -- against the oracle's CF run stored in
    tests/golden/rmat26_digest.json (written by tests/golden/rmat26_digest.py,
    which calls only the oracle), after checking by SHA-256 that the stored
    run saw the same input;
and a second dispatch gives the same digest."""

import hashlib
import json
import os
import sys
import time

import numpy as np
import pytest
import torch

import oracle
from paper_2006_11494_amd import aot, inputs

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(1100)]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rmat26_digest.json")


def sha(a: np.ndarray) -> str:
    h = hashlib.sha256()
    flat = np.ascontiguousarray(a).view(np.uint8).reshape(-1)
    for i in range(0, flat.size, 1 << 28):
        h.update(flat[i:i + (1 << 28)])
    return h.hexdigest()


def test_rmat26_sampled_parity():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if torch.cuda.get_device_properties(0).total_memory < 160 * 2**30:
        pytest.skip("needs a GPU with at least 160 GiB")
    t0 = time.time()
    say("[gpu] rmat26: generating on the device")
    csr = inputs.workload("rmat26", device="cuda")
    torch.cuda.synchronize()
    n, nnz, m = csr.n, csr.nnz, csr.m
    say(f"[gpu] rmat26: n={n} nnz={nnz} m={m} in {time.time() - t0:.1f}s")
    assert nnz > 2**31 - 1 and m <= 2**31 - 1
    o = aot.alloc_oriented(n, m, "cuda")
    ows = torch.empty(aot.orient_workspace(n, nnz), dtype=torch.uint8, device="cuda")
    aot.orient(csr.rowptr, csr.col, out=o, ws=ows, in_by_rank=True)
    del ows
    cws = torch.empty(aot.count_workspace(n, m), dtype=torch.uint8, device="cuda")
    tri_off = torch.empty(m + 1, dtype=torch.int64, device="cuda")
    c = aot.count(o, ws=cws, tri_off=tri_off)
    torch.cuda.synchronize()
    say(f"[gpu] rmat26: T={c.T} probes={c.probes} at {time.time() - t0:.1f}s")
    rp, col = csr.numpy()
    del csr
    with open(GOLDEN) as f:
        gold = json.load(f)
    assert (gold["n"], gold["nnz"]) == (n, nnz)
    assert sha(rp.astype("<i8")) == gold["rowptr_sha256"]
    assert sha(col.astype("<i4")) == gold["col_sha256"]
    assert c.probes == gold["probes"] and c.T == gold["T"]
    say(f"[gpu] rmat26: same input as the stored oracle run; T and probes equal")
    say(f"[gpu] rmat26: input on the host; oracle orientation")
    ref = oracle.orient_threaded(rp, col, threads=16, log=say)
    del col
    assert np.array_equal(o.perm.cpu().numpy(), ref.perm)
    assert np.array_equal(o.rowptr.cpu().numpy(), ref.orow)
    assert np.array_equal(o.col.cpu().numpy(), ref.ocol)
    say(f"[gpu] rmat26: orientation equal at {time.time() - t0:.1f}s")
    assert oracle.sum_min_threaded(ref, threads=16) == c.probes
    say(f"[gpu] rmat26: probe count equal")

    rng = np.random.default_rng(26)
    dplus = np.diff(ref.orow)
    top = np.argpartition(dplus, -200)[-200:]
    heavy = np.concatenate([ref.orow[r] + rng.integers(0, dplus[r], 20) for r in top])
    eids = np.unique(np.concatenate([rng.integers(0, m, 200_000), heavy]))
    want = oracle.edge_counts_at(ref, eids)
    e = torch.from_numpy(eids).cuda()
    got = (tri_off[e + 1] - tri_off[e]).cpu().numpy()
    assert np.array_equal(got, want)
    say(f"[gpu] rmat26: {eids.size} sampled edge counts equal at {time.time() - t0:.1f}s")

    for q in (0.75, 0.9, 0.97, 0.99, 0.999, 0.99995):
        r_lo = int(q * n)
        r_hi = int(np.searchsorted(ref.orow, ref.orow[r_lo] + 20_000, side="right")) - 1
        r_hi = min(max(r_hi, r_lo + 1), n)
        want = oracle.list_triangles(ref, r_lo, r_hi)
        first = int(tri_off[int(ref.orow[r_lo])])
        last = int(tri_off[int(ref.orow[r_hi])])
        parts = []
        aot.stream_list(o, c, 1 << 20, lambda f, v: parts.append(v.numpy().copy()),
                        first=first, last=last)
        got = np.concatenate(parts) if parts else np.empty((0, 3), np.int32)
        assert np.array_equal(got, want), f"ranks [{r_lo}, {r_hi})"
        say(f"[gpu] rmat26: ranks [{r_lo}, {r_hi}): {len(want)} triangles equal")

    (t, s, x), vc = aot.digest(o, c)
    assert (t, s, x) == (gold["T"], gold["F1"], gold["F2"])
    vcn = vc.cpu().numpy().astype(np.uint64)
    assert int(vcn.sum(dtype=np.uint64)) == gold["vertex_counts_sum"] == 3 * t
    assert np.array_equal(vcn[np.array(gold["sample_vertices"])],
                          np.array(gold["sample_counts"], dtype=np.uint64))
    assert sha(vcn.astype("<u8")) == gold["vertex_counts_sha256"]
    del vc, vcn
    say(f"[gpu] rmat26: whole-list digest and every vertex count equal the oracle's")
    table = [tile << 8 for tile in (4, 4, 4, 8, 16, 32, 64, 64)] + [0] * 8 + [1] * 16
    d = aot.Dispatch(aot.AOT_DISPATCH_TABLE, 0, table)
    assert aot.digest(o, c, vertex_counts=False, dispatch=d)[0] == (t, s, x)
    say(f"[gpu] rmat26: digests agree ({t} triangles) at {time.time() - t0:.1f}s")
