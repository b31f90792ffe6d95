"""The C ABI without a GPU: the library loads, exports every declared symbol,
and rejects bad arguments before touching the device."""

import ctypes
import os
import re

import pytest

from paper_2006_11494_amd import aot

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "aot.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(aot_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_exports():
    assert declared_functions() == sorted(aot.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = aot.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_version_and_status_strings():
    lib = aot.load()
    assert lib.aot_version() == aot.ABI_VERSION == 3
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert lib.aot_status_str(code)
    assert lib.aot_status_str(12345) == b"unknown status"


def test_workspace_queries():
    assert aot.orient_workspace(0, 0) > 0
    small = aot.orient_workspace(1000, 20000)
    big = aot.orient_workspace(1_000_000, 20_000_000)
    assert big > small
    assert aot.count_workspace(1000, 10000) < aot.count_workspace(10**6, 10**7)
    with pytest.raises(aot.AotError) as e:
        aot.orient_workspace(-1, 0)
    assert e.value.status == -1
    with pytest.raises(aot.AotError) as e:
        aot.orient_workspace(10, 7)             # odd nnz cannot be symmetric
    assert e.value.status == -2
    with pytest.raises(aot.AotError) as e:
        aot.orient_workspace(10, 2 * (2**31))   # m beyond int32 edge ids
    assert e.value.status == -3
    with pytest.raises(aot.AotError) as e:
        aot.count_workspace(10, 2**31)
    assert e.value.status == -3


FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: every case fails its checks first


def oriented(n=4, m=3, **kw):
    f = dict(rowptr=FAKE, col=FAKE, tail=FAKE, perm=FAKE, rank=FAKE, in_rowptr=FAKE,
             in_col=FAKE)
    f.update(kw)
    return aot.OrientedC(n, m, *[f[k] for k in ("rowptr", "col", "tail", "perm", "rank",
                                                "in_rowptr", "in_col")])


def test_orient_argument_errors():
    lib = aot.load()
    g = aot.Graph(4, 6, FAKE, FAKE)
    o = oriented()
    ok_ws = aot.orient_workspace(4, 6)
    call = lambda gg, flags, oo, ws, nb: lib.aot_orient(gg, flags, oo, ws, nb, None)
    assert call(None, 0, ctypes.byref(o), FAKE, ok_ws) == -1
    assert call(ctypes.byref(g), 0, None, FAKE, ok_ws) == -1
    assert call(ctypes.byref(g), 16, ctypes.byref(o), FAKE, ok_ws) == -1          # unknown flag
    assert call(ctypes.byref(aot.Graph(-1, 6, FAKE, FAKE)), 0, ctypes.byref(o), FAKE, ok_ws) == -1
    assert call(ctypes.byref(aot.Graph(4, 5, FAKE, FAKE)), 0, ctypes.byref(o), FAKE, ok_ws) == -2
    assert call(ctypes.byref(aot.Graph(4, 6, None, FAKE)), 0, ctypes.byref(o), FAKE, ok_ws) == -1
    assert call(ctypes.byref(aot.Graph(4, 6, FAKE, None)), 0, ctypes.byref(o), FAKE, ok_ws) == -1
    assert call(ctypes.byref(g), 0, ctypes.byref(oriented(col=None)), FAKE, ok_ws) == -1
    assert call(ctypes.byref(g), 0, ctypes.byref(oriented(perm=None)), FAKE, ok_ws) == -1
    assert call(ctypes.byref(g), 0, ctypes.byref(o), FAKE, ok_ws - 1) == -4       # workspace
    assert call(ctypes.byref(g), 0, ctypes.byref(o), None, ok_ws) == -4
    assert b"workspace" in lib.aot_last_error()


def test_count_and_list_argument_errors():
    lib = aot.load()
    o = oriented()
    res = (ctypes.c_uint64 * 2)()
    ws = aot.count_workspace(4, 3)
    d = aot.DispatchC(0, 0, None)
    assert lib.aot_count(None, None, FAKE, FAKE, ws, res, None) == -1
    assert lib.aot_count(ctypes.byref(o), None, None, FAKE, ws, res, None) == -1
    assert lib.aot_count(ctypes.byref(o), None, FAKE, FAKE, ws, None, None) == -1
    assert lib.aot_count(ctypes.byref(o), None, FAKE, FAKE, ws - 1, res, None) == -4
    assert lib.aot_count(ctypes.byref(oriented(m=-1)), None, FAKE, FAKE, ws, res, None) == -1
    assert lib.aot_count(ctypes.byref(oriented(m=2**31)), None, FAKE, FAKE, ws, res, None) == -3
    bad_mode = aot.DispatchC(7, 0, None)
    assert lib.aot_count(ctypes.byref(o), ctypes.byref(bad_mode), FAKE, FAKE, ws, res, None) == -1
    no_table = aot.DispatchC(1, 0, None)
    assert lib.aot_count(ctypes.byref(o), ctypes.byref(no_table), FAKE, FAKE, ws, res, None) == -6
    # table codes are checked before anything runs: a tile outside {4..64},
    # a light code with an arm byte, a heavy arm outside 0..3
    plain = [t << 8 for t in (4, 4, 4, 8, 16, 32, 64, 64)] + [0] * 24
    for k, code in ((2, 5 << 8), (0, (4 << 8) | 1), (16, 4), (31, -1)):
        codes = list(plain)
        codes[k] = code
        table = (ctypes.c_int32 * aot.AOT_NUM_BUCKETS)(*codes)
        bad = aot.DispatchC(aot.AOT_DISPATCH_TABLE, 0, ctypes.cast(table, ctypes.c_void_p).value)
        assert lib.aot_count(ctypes.byref(o), ctypes.byref(bad), FAKE, FAKE, ws, res, None) == -6
        assert b"unknown arm or tile" in lib.aot_last_error()
    neg = aot.DispatchC(0, -3, None)
    assert lib.aot_count(ctypes.byref(o), ctypes.byref(neg), FAKE, FAKE, ws, res, None) == -1
    bad_strategy = aot.DispatchC(0, 0, None, None, 4)
    assert lib.aot_count(ctypes.byref(o), ctypes.byref(bad_strategy), FAKE, FAKE, ws, res,
                         None) == -1
    learned_head = aot.DispatchC(aot.AOT_DISPATCH_LEARNED, 0, None, None, aot.AOT_STRATEGY_HEAD)
    assert lib.aot_count(ctypes.byref(o), ctypes.byref(learned_head), FAKE, FAKE, ws, res,
                         None) == -1
    assert b"adaptive" in lib.aot_last_error()
    sup = lambda es, off: lib.aot_support(ctypes.byref(o), None, off, FAKE, ws, es, None, None,
                                          None)
    assert sup(None, FAKE) == -1                    # m > 0 needs the edge array
    assert sup(FAKE, None) == -1
    lst = lambda oo, dd, off, w, nb, first, cnt, out: lib.aot_list(oo, dd, off, w, nb, first, cnt,
                                                                  out, None, None)
    assert lst(ctypes.byref(o), ctypes.byref(d), None, FAKE, ws, 0, 1, FAKE) == -1
    assert lst(ctypes.byref(o), ctypes.byref(d), FAKE, FAKE, ws, -1, 1, FAKE) == -1
    assert lst(ctypes.byref(o), ctypes.byref(d), FAKE, FAKE, ws, 0, -1, FAKE) == -1
    assert lst(ctypes.byref(o), ctypes.byref(d), FAKE, FAKE, ws, 0, 1, None) == -1
    assert lst(ctypes.byref(o), ctypes.byref(d), FAKE, FAKE, ws, 0, 2**62, FAKE) == -7
    assert lst(ctypes.byref(o), ctypes.byref(d), FAKE, FAKE, ws - 1, 0, 1, FAKE) == -4


def test_errors_are_thread_local():
    import threading
    lib = aot.load()
    lib.aot_orient(None, 0, None, None, 0, None)
    seen = []
    t = threading.Thread(target=lambda: seen.append(lib.aot_last_error()))
    t.start()
    t.join()
    assert seen == [b""] and lib.aot_last_error() != b""


def test_binding_refuses_a_missing_library(tmp_path, monkeypatch):
    monkeypatch.setattr(aot, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        aot.load(str(tmp_path / "libaot.so"))
