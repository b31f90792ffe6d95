"""CPU oracle for AOT triangle listing -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never loads it and
shares no code with it.  The arithmetic lives in ``oracle.c`` (plain C, one
thread); this file only builds it with gcc and marshals numpy arrays.

Section references are to Yu et al., "AOT: Pushing the Efficiency Boundary of
Main-memory Triangle Listing" (2020).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")


def build() -> str:
    """Compile oracle.c into liboracle.so with gcc (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    lib.orc_orient.argtypes = [i32, _i64p, _i32p, _i32p, _i32p, _i64p, _i32p]
    lib.orc_orient.restype = i64
    lib.orc_edge_counts.argtypes = [i32, _i64p, _i32p, i64, i64, _i32p]
    lib.orc_edge_counts.restype = None
    lib.orc_edge_counts_at.argtypes = [i32, _i64p, _i32p, _i64p, i64, _i32p]
    lib.orc_edge_counts_at.restype = None
    lib.orc_list.argtypes = [i32, _i64p, _i32p, _i32p, i32, i32, _i32p, i64]
    lib.orc_list.restype = i64
    lib.orc_sum_min.argtypes = [i32, _i64p, _i32p]
    lib.orc_sum_min.restype = u64
    lib.orc_sum_head.argtypes = [i32, _i64p, _i32p]
    lib.orc_sum_head.restype = u64
    lib.orc_edge_support.argtypes = [i32, _i64p, _i32p, _i64p, _i32p, _i32p, _i32p]
    lib.orc_edge_support.restype = None
    lib.orc_core_rounds.argtypes = [i32, _i64p, _i32p, _i32p, ctypes.POINTER(i32)]
    lib.orc_core_rounds.restype = i32
    lib.orc_orient_core.argtypes = [i32, _i64p, _i32p, _i32p, _i32p, _i64p, _i32p]
    lib.orc_orient_core.restype = i64
    lib.orc_orient_by_id.argtypes = [i32, _i64p, _i32p, _i32p, _i64p, _i32p]
    lib.orc_orient_by_id.restype = i64
    lib.orc_sum_merge.argtypes = [i32, _i64p, _i32p]
    lib.orc_sum_merge.restype = u64
    lib.orc_aot_ref.argtypes = [i32, _i64p, _i32p, ctypes.c_int, ctypes.c_void_p, i64,
                                ctypes.c_void_p, ctypes.POINTER(u64)]
    lib.orc_aot_ref.restype = i64
    lib.orc_fingerprint.argtypes = [_i32p, i64, _u64p, ctypes.c_void_p]
    lib.orc_fingerprint.restype = None
    lib.orc_list_digest.argtypes = [i32, _i64p, _i32p, _i32p, i32, i32, _u64p, ctypes.c_void_p]
    lib.orc_list_digest.restype = i64
    lib.orc_in_lists.argtypes = [i32, _i64p, _i32p, _i64p, _i32p, _i32p]
    lib.orc_in_lists.restype = i64
    lib.orc_rank.argtypes = [i32, _i64p, _i32p, _i32p]
    lib.orc_rank.restype = ctypes.c_int
    lib.orc_orient_count.argtypes = [_i64p, _i32p, _i32p, _i32p, i32, i32, _i64p]
    lib.orc_orient_count.restype = None
    lib.orc_orient_write.argtypes = [_i64p, _i32p, _i32p, _i32p, _i64p, i32, i32, ctypes.c_void_p]
    lib.orc_orient_write.restype = None
    lib.orc_sum_min_range.argtypes = [_i64p, _i32p, i32, i32]
    lib.orc_sum_min_range.restype = u64
    lib.orc_vertex_triangles.argtypes = [_i64p, _i32p, _i32p, i64, _i64p]
    lib.orc_vertex_triangles.restype = None
    lib.orc_splitmix64.argtypes = [u64]
    lib.orc_splitmix64.restype = u64
    _lib = lib
    return lib


def _arrays(rowptr, col):
    rowptr = np.ascontiguousarray(np.asarray(rowptr), dtype=np.int64)
    col = np.ascontiguousarray(np.asarray(col), dtype=np.int32)
    return rowptr, col


class Oriented:
    """Oriented graph in label space: labels are ranks (position in the order)
    by default, original ids with local="id" (perm and rank the identity)."""

    def __init__(self, n, perm, rank, orow, ocol):
        self.n, self.perm, self.rank, self.orow, self.ocol = n, perm, rank, orow, ocol

    @property
    def m(self) -> int:
        return int(self.orow[-1])

    @property
    def dplus(self):
        return np.diff(self.orow)

    def tail(self):
        return np.repeat(np.arange(self.n, dtype=np.int32), self.dplus)


def orient(rowptr, col, order: str = "degree", local: str = "rank") -> Oriented:
    """Degree order with id tie-break; <u,v> iff eta(u) < eta(v) (Sec. 2.2).
    order="core": the core order of kClist (Sec. 2.3), see core_rounds.
    local="id": the same edges with original ids as labels, so each out-list
    is in id order (AOT-randomOrder, Sec. 4.2, for inputs with permuted ids)."""
    lib = _load()
    rowptr, col = _arrays(rowptr, col)
    if local not in ("rank", "id"):
        raise ValueError(local)
    if local == "id":
        eta = orient(rowptr, col, order)
        n = eta.n
        orow = np.empty(n + 1, np.int64)
        ocol = np.empty(max(col.size // 2, 1), np.int32)
        m = lib.orc_orient_by_id(n, rowptr, _nonempty(col), _nonempty(eta.rank), orow, ocol)
        ident = np.arange(n, dtype=np.int32)
        return Oriented(n, ident, ident.copy(), orow, ocol[:m].copy())
    n = rowptr.size - 1
    perm = np.empty(max(n, 1), np.int32)
    rank = np.empty(max(n, 1), np.int32)
    orow = np.empty(n + 1, np.int64)
    ocol = np.empty(max(col.size // 2, 1), np.int32)
    if order not in ("degree", "core"):
        raise ValueError(order)
    fn = lib.orc_orient if order == "degree" else lib.orc_orient_core
    m = fn(n, rowptr, col, perm, rank, orow, ocol)
    if m < 0:
        raise MemoryError("oracle orientation failed")
    return Oriented(n, perm[:n], rank[:n], orow, ocol[:m].copy())


def _rank_ranges(rowptr, perm, parts):
    """Rank ranges holding about equal shares of the input's entries."""
    n = perm.size
    if n == 0:
        return []
    deg = np.diff(rowptr)[perm]
    cum = np.cumsum(deg)
    cuts = np.searchsorted(cum, np.linspace(0, cum[-1], parts + 1)[1:-1])
    b = sorted(set([0, n] + [int(c) for c in cuts]))
    return [(x, y) for x, y in zip(b[:-1], b[1:]) if y > x]


def orient_threaded(rowptr, col, threads: int = 16, log=None) -> Oriented:
    """The same orientation as orient(), for graphs with billions of entries:
    the order eta once, then deg+ and the sorted out-lists of rank ranges on
    host threads (the per-row procedure is unchanged)."""
    lib = _load()
    rowptr, col = _arrays(rowptr, col)
    n = rowptr.size - 1
    perm = np.empty(max(n, 1), np.int32)
    rank = np.empty(max(n, 1), np.int32)
    if lib.orc_rank(n, rowptr, perm, rank):
        raise MemoryError("oracle ranking failed")
    perm, rank = perm[:n], rank[:n]
    if log:
        log(f"[oracle] ranked {n} vertices")
    ranges = _rank_ranges(rowptr, perm, 8 * threads)
    dplus = np.zeros(max(n, 1), np.int64)
    col_ = _nonempty(col)

    def count(ab):
        a, b = ab
        part = np.empty(b - a, np.int64)
        lib.orc_orient_count(rowptr, col_, perm, rank, a, b, part)
        dplus[a:b] = part

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(count, ranges))
    orow = np.zeros(n + 1, np.int64)
    np.cumsum(dplus[:n], out=orow[1:])
    m = int(orow[-1])
    if log:
        log(f"[oracle] out-degrees of {n} ranks: m = {m}")
    ocol = np.empty(max(m, 1), np.int32)
    done = [0]

    def write(ab):
        a, b = ab
        lib.orc_orient_write(rowptr, col_, perm, rank, orow, a, b, ocol.ctypes.data)
        done[0] += 1
        if log and done[0] % threads == 0:
            log(f"[oracle] out-lists: {done[0]}/{len(ranges)} rank ranges written")

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(write, ranges))
    return Oriented(n, perm, rank, orow, ocol[:m])


def sum_min_threaded(o: Oriented, threads: int = 16) -> int:
    """sum_min over rank ranges on host threads."""
    lib = _load()
    ranges = [(a, b) for a, b in zip(*(lambda c: (c[:-1], c[1:]))(
        np.linspace(0, o.n, 8 * threads + 1).astype(np.int64))) if b > a]
    oc = _nonempty(o.ocol)
    with ThreadPoolExecutor(threads) as ex:
        parts = ex.map(lambda ab: int(lib.orc_sum_min_range(o.orow, oc, int(ab[0]), int(ab[1]))),
                       ranges)
        return sum(parts)


def vertex_triangles(rowptr, col, vs) -> np.ndarray:
    """t(v) for the given original ids: edges among the neighbours of v."""
    lib = _load()
    rowptr, col = _arrays(rowptr, col)
    vs = np.ascontiguousarray(vs, dtype=np.int32)
    out = np.zeros(max(vs.size, 1), np.int64)
    if vs.size:
        lib.orc_vertex_triangles(rowptr, _nonempty(col), vs, vs.size, out)
    return out[: vs.size]


def edge_support(rowptr, col, o: Oriented) -> np.ndarray:
    """Triangles through each oriented edge of o (in o's edge order): the
    A^2 entry of its endpoints, from the input's full rows."""
    rowptr, col = _arrays(rowptr, col)
    sup = np.empty(max(o.m, 1), np.int32)
    _load().orc_edge_support(o.n, rowptr, col, o.orow, _nonempty(o.ocol), _nonempty(o.perm), sup)
    return sup[:o.m]


def core_rounds(rowptr, col):
    """Synchronous peeling (the core order, Sec. 2.3): (round[v], sub-rounds,
    degeneracy); the order is (round, id) ascending."""
    rowptr, col = _arrays(rowptr, col)
    n = rowptr.size - 1
    rnd = np.empty(max(n, 1), np.int32)
    deg = ctypes.c_int32(0)
    k = _load().orc_core_rounds(n, rowptr, col, rnd, ctypes.byref(deg))
    if k < 0:
        raise MemoryError("oracle peeling failed")
    return rnd[:n], int(k), int(deg.value)


def in_lists(o: Oriented):
    """In-lists in ascending rank and the edge id of each in-edge <x, r>."""
    lib = _load()
    irow = np.empty(o.n + 1, np.int64)
    icol = np.empty(max(o.m, 1), np.int32)
    ieid = np.empty(max(o.m, 1), np.int32)
    k = lib.orc_in_lists(o.n, o.orow, _nonempty(o.ocol), irow, icol, ieid)
    if k < 0:
        raise MemoryError("oracle in-lists failed")
    return irow, icol[:k].copy(), ieid[:k].copy()


def edge_counts(o: Oriented, e_lo: int = 0, e_hi: int | None = None) -> np.ndarray:
    """|N+(u) n N+(v)| for each directed edge in [e_lo, e_hi) (Algorithm 1's intersection step)."""
    lib = _load()
    e_hi = o.m if e_hi is None else e_hi
    out = np.zeros(max(e_hi - e_lo, 1), np.int32)
    lib.orc_edge_counts(o.n, o.orow, _nonempty(o.ocol), e_lo, e_hi, out)
    return out[: e_hi - e_lo]


def edge_counts_at(o: Oriented, eids) -> np.ndarray:
    lib = _load()
    eids = np.ascontiguousarray(eids, dtype=np.int64)
    out = np.zeros(max(eids.size, 1), np.int32)
    if eids.size:
        lib.orc_edge_counts_at(o.n, o.orow, _nonempty(o.ocol), eids, eids.size, out)
    return out[: eids.size]


def _nonempty(a):
    return a if a.size else np.zeros(1, a.dtype)


def list_triangles(o: Oriented, r_lo: int = 0, r_hi: int | None = None, cap: int | None = None) -> np.ndarray:
    """Algorithm 1 (CF) over sources [r_lo, r_hi): (T, 3) int32, ascending ids
    per row, in edge order then ascending third vertex."""
    lib = _load()
    r_hi = o.n if r_hi is None else r_hi
    if cap is None:
        cap = int(edge_counts(o, int(o.orow[r_lo]), int(o.orow[r_hi])).sum()) if r_hi > r_lo else 0
    out = np.empty(max(3 * cap, 3), np.int32)
    t = lib.orc_list(o.n, o.orow, _nonempty(o.ocol), _nonempty(o.perm), r_lo, r_hi, out, cap)
    if t < 0:
        raise ValueError(f"capacity {cap} below triangle count {-t}")
    return out[: 3 * t].reshape(t, 3)


def list_triangles_parallel(o: Oriented, threads: int = 8) -> np.ndarray:
    """The same list, computed over source-rank ranges on several threads (the
    per-range procedure is unchanged; ranges are concatenated in order)."""
    if o.n == 0:
        return np.empty((0, 3), np.int32)
    cuts = np.linspace(0, o.m, threads + 1).astype(np.int64)
    bounds = sorted(set(int(np.searchsorted(o.orow, c, side="right") - 1) for c in cuts[1:-1]))
    ranges = list(zip([0] + bounds, bounds + [o.n]))
    ranges = [(a, b) for a, b in ranges if b > a]
    with ThreadPoolExecutor(len(ranges)) as ex:
        parts = list(ex.map(lambda ab: list_triangles(o, ab[0], ab[1]), ranges))
    return np.concatenate(parts) if parts else np.empty((0, 3), np.int32)


def sum_min(o: Oriented) -> int:
    """sum over <u,v> of min(deg+(u), deg+(v)) (Section 3.2, Time Complexity)."""
    return int(_load().orc_sum_min(o.n, o.orow, _nonempty(o.ocol)))


def sum_head(o: Oriented) -> int:
    """sum over <u,v> of deg+(v) (the kClist cost, Section 2.3)."""
    return int(_load().orc_sum_head(o.n, o.orow, _nonempty(o.ocol)))


def sum_merge(o: Oriented) -> int:
    """sum over <u,v> of deg+(u) + deg+(v) (the CF merge cost, Section 2.2)."""
    return int(_load().orc_sum_merge(o.n, o.orow, _nonempty(o.ocol)))


def aot_ref(rowptr, col, tie_break: bool = True, cap: int | None = None, digest: bool = False):
    """AOT (Algorithm 3) on original ids, the cross-check of CF.  Returns
    (triangles (T,3), probes), or with digest=True (T, (F1, F2), probes)
    without storing the list."""
    lib = _load()
    rowptr, col = _arrays(rowptr, col)
    n = rowptr.size - 1
    probes = ctypes.c_uint64(0)
    if digest:
        fp = np.zeros(2, np.uint64)
        t = lib.orc_aot_ref(n, rowptr, _nonempty(col), int(tie_break), None, 0, fp.ctypes.data,
                            ctypes.byref(probes))
        if t == np.iinfo(np.int64).min:
            raise MemoryError("oracle AOT reference failed")
        return int(t), (int(fp[0]), int(fp[1])), int(probes.value)
    if cap is None:
        cap = max(16, col.size * 4)
    out = np.empty(3 * cap, np.int32)
    t = lib.orc_aot_ref(n, rowptr, _nonempty(col), int(tie_break), out.ctypes.data, cap, None,
                        ctypes.byref(probes))
    if t == np.iinfo(np.int64).min:
        raise MemoryError("oracle AOT reference failed")
    if t < 0:
        return aot_ref(rowptr, col, tie_break, cap=-t)
    return out[: 3 * t].reshape(t, 3).copy(), int(probes.value)


def fingerprint(tri: np.ndarray, n: int | None = None):
    """(F1, F2) = (sum mod 2^64, xor) of splitmix64-chained triple hashes, and
    per-vertex counts when n is given."""
    lib = _load()
    tri = np.ascontiguousarray(tri, dtype=np.int32).reshape(-1, 3)
    fp = np.zeros(2, np.uint64)
    tv = np.zeros(n, np.uint64) if n else None
    lib.orc_fingerprint(_nonempty(tri.reshape(-1)), tri.shape[0], fp,
                        tv.ctypes.data if tv is not None else None)
    return (int(fp[0]), int(fp[1])), tv


def splitmix64(z: int) -> int:
    """The hash the fingerprints chain (SplitMix64 output of state z)."""
    return int(_load().orc_splitmix64(z))


def list_digest(o: Oriented, r_lo: int = 0, r_hi: int | None = None, per_vertex: bool = True):
    """CF over sources [r_lo, r_hi) without storing the list: (T, (F1, F2), t[v])."""
    lib = _load()
    r_hi = o.n if r_hi is None else r_hi
    fp = np.zeros(2, np.uint64)
    tv = np.zeros(o.n, np.uint64) if per_vertex else None
    t = lib.orc_list_digest(o.n, o.orow, _nonempty(o.ocol), _nonempty(o.perm), r_lo, r_hi, fp,
                            tv.ctypes.data if tv is not None else None)
    return int(t), (int(fp[0]), int(fp[1])), tv


def list_digest_threaded(o: Oriented, threads: int = 16, per_vertex: bool = True, log=None):
    """list_digest over the whole graph, with source-rank ranges of about equal
    edge counts spread over host threads (the per-range procedure is
    unchanged).  Sums combine mod 2^64, xors by xor, per-vertex counts by
    addition."""
    lib = _load()
    if o.n == 0:
        return 0, (0, 0), (np.zeros(0, np.uint64) if per_vertex else None)
    cuts = np.searchsorted(o.orow, np.linspace(0, o.m, 64 * threads + 1), side="left")
    bounds = sorted(set([0, o.n] + [int(c) for c in cuts]))
    ranges = [(a, b) for a, b in zip(bounds[:-1], bounds[1:]) if b > a]
    oc, pm = _nonempty(o.ocol), _nonempty(o.perm)
    state = {"next": 0, "done": 0}
    import threading
    lock = threading.Lock()

    def worker(_):
        tv = np.zeros(o.n, np.uint64) if per_vertex else None
        t, f1, f2 = 0, 0, 0
        fp = np.zeros(2, np.uint64)
        while True:
            with lock:
                i = state["next"]
                state["next"] += 1
            if i >= len(ranges):
                return t, f1, f2, tv
            a, b = ranges[i]
            t += int(lib.orc_list_digest(o.n, o.orow, oc, pm, a, b, fp,
                                         tv.ctypes.data if tv is not None else None))
            f1 = (f1 + int(fp[0])) % (1 << 64)
            f2 ^= int(fp[1])
            with lock:
                state["done"] += 1
                if log and state["done"] % (4 * threads) == 0:
                    log(f"[oracle] digest: {state['done']}/{len(ranges)} rank ranges")

    with ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(worker, range(threads)))
    t = sum(p[0] for p in parts)
    f1 = sum(p[1] for p in parts) % (1 << 64)
    f2 = 0
    for p in parts:
        f2 ^= p[2]
    tv = None
    if per_vertex:
        tv = parts[0][3]
        for p in parts[1:]:
            tv += p[3]
    return t, (f1, f2), tv
