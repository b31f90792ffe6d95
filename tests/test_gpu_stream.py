"""Listing in windows streamed to pinned host memory: the concatenated
windows equal the oracle's list, for window sizes that split edges, and for
a sub-range of the list."""

import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2006_11494_amd import aot, inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("chunk", [1, 777, 65536, 1 << 22])
def test_streamed_windows_equal_the_oracle(chunk):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    csr = inputs.rmat(15, 16, 31)
    rp, col = csr.numpy()
    ref = oracle.list_triangles_parallel(oracle.orient(rp, col), threads=8)
    g = csr.to("cuda")
    o = aot.orient(g.rowptr, g.col)
    c = aot.count(o)
    assert c.T == len(ref)
    first, last = (0, c.T) if chunk > 1 else (c.T // 3, c.T // 3 + 5000)
    got = []
    seen = []

    def take(f, view):
        seen.append(f)
        got.append(view.numpy().copy())

    say(f"[gpu] stream T={c.T} chunk={chunk} window [{first}, {last})")
    n = aot.stream_list(o, c, chunk, take, first=first, last=last)
    assert n == -(-(last - first) // chunk)
    assert seen == list(range(first, last, chunk))
    assert np.array_equal(np.concatenate(got), ref[first:last])
    # device-only windows, no host copy
    got.clear()
    seen.clear()
    aot.stream_list(o, c, chunk, lambda f, v: got.append(v.cpu().numpy()), first=first,
                    last=last, to_host=False)
    assert np.array_equal(np.concatenate(got), ref[first:last])


@pytest.mark.parametrize("in_by_rank", [False, True])
def test_streamed_windows_with_id_labels(in_by_rank):
    """AOT-randomOrder's id labels: windows of the list in id-labelled edge
    order, with in-lists in either order."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    csr = inputs.rmat(14, 16, 35)
    rp, col = csr.numpy()
    ref = oracle.list_triangles(oracle.orient(rp, col, local="id"))
    g = csr.to("cuda")
    o = aot.orient(g.rowptr, g.col, local="id", in_by_rank=in_by_rank)
    c = aot.count(o)
    assert c.T == len(ref)
    got = []
    say(f"[gpu] stream id labels T={c.T} in_by_rank={in_by_rank}")
    aot.stream_list(o, c, 100003, lambda f, v: got.append(v.numpy().copy()))
    assert np.array_equal(np.concatenate(got), ref)
