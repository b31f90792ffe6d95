"""Python binding of libaot.so (include/aot.h): argument marshalling only.

Device buffers are torch tensors on a ROCm device; every step of the method
runs in the library's HIP kernels.  There is no fallback: if the library is
not built, loading raises.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libaot.so")

ABI_VERSION = 3          # the aot_version() this binding's structs match
AOT_NOALLOC_SCRATCH_BYTES = 64 << 20   # fixed scratch of aot_count_noalloc (include/aot.h)
AOT_OK = 0
AOT_VALIDATE = 1
AOT_IN_LISTS_BY_RANK = 2
AOT_ORDER_CORE = 4
AOT_LOCAL_BY_ID = 8
AOT_DISPATCH_PLAIN = 0
AOT_DISPATCH_TABLE = 1
AOT_DISPATCH_LEARNED = 2
AOT_STRATEGY_ADAPTIVE = 0
AOT_STRATEGY_HEAD = 1
AOT_STRATEGY_MERGE = 2
AOT_STRATEGY_PER_EDGE = 3
STRATEGIES = {"aot": AOT_STRATEGY_ADAPTIVE, "head": AOT_STRATEGY_HEAD,
              "merge": AOT_STRATEGY_MERGE, "per_edge": AOT_STRATEGY_PER_EDGE}
AOT_NUM_BUCKETS = 32
AOT_NUM_OPTIONS = 9
AOT_NUM_FEATURES = 8

# every symbol include/aot.h declares
EXPORTS = (
    "aot_status_str", "aot_last_error", "aot_version",
    "aot_orient_workspace", "aot_orient",
    "aot_count_workspace", "aot_count", "aot_count_noalloc",
    "aot_list", "aot_digest", "aot_support", "aot_count_plan", "aot_bucket_features",
    "aot_mlp_param_count", "aot_mlp_workspace", "aot_mlp_init", "aot_mlp_forward",
    "aot_mlp_loss_grad", "aot_mlp_train",
    "aot_timing_start", "aot_timing_stop",
    "aot_batch_workspace", "aot_batch_run", "aot_batch_capture", "aot_batch_launch",
    "aot_batch_destroy",
)


class AotError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: status {status}")
        self.status = status


class Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("rowptr", ctypes.c_void_p), ("col", ctypes.c_void_p)]


class OrientedC(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int64),
                ("rowptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("tail", ctypes.c_void_p), ("perm", ctypes.c_void_p),
                ("rank", ctypes.c_void_p), ("in_rowptr", ctypes.c_void_p),
                ("in_col", ctypes.c_void_p)]


class TimingC(ctypes.Structure):
    _fields_ = [("pass_", ctypes.c_int32), ("bucket", ctypes.c_int32), ("arm", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("edges", ctypes.c_int64), ("probes", ctypes.c_int64),
                ("staged", ctypes.c_int64), ("triangles", ctypes.c_int64),
                ("ms", ctypes.c_double), ("lookups", ctypes.c_int64)]


class DispatchC(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("heavy_min", ctypes.c_int32),
                ("table", ctypes.c_void_p), ("model", ctypes.c_void_p),
                ("strategy", ctypes.c_int32)]


class BatchC(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("voff_host", ctypes.c_void_p),
                ("voff", ctypes.c_void_p), ("arena", Graph)]


class ScheduleC(ctypes.Structure):
    _fields_ = [("heavy_min", ctypes.c_int32), ("use_table", ctypes.c_int32),
                ("table", ctypes.c_int32 * AOT_NUM_BUCKETS), ("light_rounds", ctypes.c_int32)]


class MlpC(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int32), ("n_hidden", ctypes.c_int32),
                ("n_out", ctypes.c_int32), ("params", ctypes.c_void_p)]


_lib = None


def load(path: str = LIB_PATH):
    """Loads libaot.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2006_11494_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    sz = ctypes.POINTER(ctypes.c_size_t)
    lib.aot_status_str.argtypes = [ctypes.c_int]
    lib.aot_status_str.restype = ctypes.c_char_p
    lib.aot_last_error.argtypes = []
    lib.aot_last_error.restype = ctypes.c_char_p
    lib.aot_version.argtypes = []
    lib.aot_version.restype = ctypes.c_int
    lib.aot_orient_workspace.argtypes = [i32, i64, sz]
    lib.aot_orient.argtypes = [ctypes.POINTER(Graph), u32, ctypes.POINTER(OrientedC), vp,
                               ctypes.c_size_t, vp]
    lib.aot_count_workspace.argtypes = [i32, i64, sz]
    lib.aot_count.argtypes = [ctypes.POINTER(OrientedC), ctypes.POINTER(DispatchC), vp, vp,
                              ctypes.c_size_t, ctypes.POINTER(ctypes.c_uint64), vp]
    lib.aot_count_noalloc.argtypes = [ctypes.POINTER(OrientedC), ctypes.POINTER(DispatchC), vp,
                                      ctypes.POINTER(ctypes.c_uint64), vp]
    lib.aot_list.argtypes = [ctypes.POINTER(OrientedC), ctypes.POINTER(DispatchC), vp, vp,
                             ctypes.c_size_t, i64, i64, vp, ctypes.POINTER(ctypes.c_int64), vp]
    lib.aot_digest.argtypes = [ctypes.POINTER(OrientedC), ctypes.POINTER(DispatchC), vp, vp,
                               ctypes.c_size_t, vp, ctypes.POINTER(ctypes.c_uint64), vp]
    lib.aot_support.argtypes = [ctypes.POINTER(OrientedC), ctypes.POINTER(DispatchC), vp, vp,
                                ctypes.c_size_t, vp, vp, ctypes.POINTER(ctypes.c_uint64), vp]
    lib.aot_count_plan.argtypes = [vp, ctypes.c_size_t, i32, i64, ctypes.POINTER(i32),
                                   ctypes.POINTER(i32)]
    lib.aot_bucket_features.argtypes = [vp, ctypes.c_size_t, i32, i64,
                                        ctypes.POINTER(ctypes.c_float),
                                        ctypes.POINTER(ctypes.c_uint8)]
    mp = ctypes.POINTER(MlpC)
    lib.aot_mlp_param_count.argtypes = [i32, i32, i32, ctypes.POINTER(i64)]
    lib.aot_mlp_workspace.argtypes = [mp, i32, ctypes.POINTER(ctypes.c_size_t)]
    lib.aot_mlp_init.argtypes = [mp, ctypes.c_uint64, vp]
    lib.aot_mlp_forward.argtypes = [mp, vp, i32, vp, vp]
    lib.aot_mlp_loss_grad.argtypes = [mp, vp, vp, vp, i32, vp, vp, vp, ctypes.c_size_t, vp]
    lib.aot_mlp_train.argtypes = [mp, vp, vp, vp, i32, i32, ctypes.c_float,
                                  ctypes.POINTER(ctypes.c_float), vp, ctypes.c_size_t, vp]
    bp, sp, op = ctypes.POINTER(BatchC), ctypes.POINTER(ScheduleC), ctypes.POINTER(OrientedC)
    lib.aot_batch_workspace.argtypes = [bp, sz]
    lib.aot_batch_run.argtypes = [bp, sp, op, vp, vp, vp, i64, vp, ctypes.c_size_t, vp]
    lib.aot_batch_capture.argtypes = [bp, sp, op, vp, vp, vp, i64, vp, ctypes.c_size_t,
                                      ctypes.POINTER(vp)]
    lib.aot_batch_launch.argtypes = [vp, vp]
    lib.aot_batch_destroy.argtypes = [vp]
    lib.aot_timing_start.argtypes = []
    lib.aot_timing_stop.argtypes = [ctypes.POINTER(TimingC), i32, ctypes.POINTER(i32)]
    for f in EXPORTS:
        if f in ("aot_status_str", "aot_last_error", "aot_version"):
            continue
        getattr(lib, f).restype = ctypes.c_int
    if lib.aot_version() != ABI_VERSION:
        raise RuntimeError(f"{path}: ABI version {lib.aot_version()}, this binding needs "
                           f"{ABI_VERSION}; rebuild with python -m paper_2006_11494_amd.build")
    _lib = lib
    return lib


def _check(status: int, what: str):
    if status != AOT_OK:
        lib = load()
        msg = lib.aot_last_error().decode() or lib.aot_status_str(status).decode()
        raise AotError(status, f"{what}: {msg}")


def _ptr(t: torch.Tensor | None):
    return None if t is None or t.numel() == 0 else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


@dataclass
class Oriented:
    """Oriented graph in rank space (device tensors); see aot_oriented."""
    n: int
    m: int
    rowptr: torch.Tensor
    col: torch.Tensor
    tail: torch.Tensor
    perm: torch.Tensor
    rank: torch.Tensor
    in_rowptr: torch.Tensor
    in_col: torch.Tensor

    def cstruct(self) -> OrientedC:
        return OrientedC(self.n, self.m, _ptr(self.rowptr), _ptr(self.col), _ptr(self.tail),
                         _ptr(self.perm), _ptr(self.rank), _ptr(self.in_rowptr),
                         _ptr(self.in_col))

    @property
    def dplus(self) -> torch.Tensor:
        return self.rowptr[1:] - self.rowptr[:-1]


@dataclass
class Dispatch:
    """Probe-kernel dispatch: the plain rule, a per-bucket code table, or the
    learned cost model (`model`, an Mlp), and the probe strategy
    (AOT_STRATEGY_*; the write pass always uses the count's)."""
    mode: int = AOT_DISPATCH_PLAIN
    heavy_min: int = 0
    table: list | None = None
    model: "Mlp | None" = None
    strategy: int = AOT_STRATEGY_ADAPTIVE

    def cstruct(self):
        self._table = None
        tp = None
        if self.table is not None:
            self._table = (ctypes.c_int32 * AOT_NUM_BUCKETS)(*self.table)
            tp = ctypes.cast(self._table, ctypes.c_void_p)
        mp = None
        if self.model is not None:
            self._model = self.model.cstruct()
            mp = ctypes.cast(ctypes.pointer(self._model), ctypes.c_void_p)
        return DispatchC(self.mode, self.heavy_min, tp, mp, self.strategy)


class Mlp:
    """The dispatch cost model: parameters in a device float32 tensor, every
    operation one of the library's HIP kernels."""

    def __init__(self, n_in=AOT_NUM_FEATURES, n_hidden=32, n_out=AOT_NUM_OPTIONS,
                 device="cuda", params: torch.Tensor | None = None):
        self.n_in, self.n_hidden, self.n_out = n_in, n_hidden, n_out
        cnt = ctypes.c_int64(0)
        _check(load().aot_mlp_param_count(n_in, n_hidden, n_out, ctypes.byref(cnt)),
               "aot_mlp_param_count")
        self.n_params = cnt.value
        self.params = params if params is not None else torch.zeros(
            cnt.value, dtype=torch.float32, device=device)
        assert self.params.numel() == self.n_params and self.params.dtype == torch.float32

    def cstruct(self) -> MlpC:
        return MlpC(self.n_in, self.n_hidden, self.n_out, self.params.data_ptr())

    def _ws(self, batch):
        b = ctypes.c_size_t(0)
        net = self.cstruct()
        _check(load().aot_mlp_workspace(ctypes.byref(net), batch, ctypes.byref(b)),
               "aot_mlp_workspace")
        return torch.empty(b.value, dtype=torch.uint8, device=self.params.device)

    def init(self, seed: int, stream=None):
        net = self.cstruct()
        _check(load().aot_mlp_init(ctypes.byref(net), seed, _stream(stream)), "aot_mlp_init")
        return self

    def forward(self, x: torch.Tensor, stream=None) -> torch.Tensor:
        x = x.contiguous().to(torch.float32)
        y = torch.empty((x.shape[0], self.n_out), dtype=torch.float32, device=x.device)
        net = self.cstruct()
        _check(load().aot_mlp_forward(ctypes.byref(net), _ptr(x), x.shape[0], _ptr(y),
                                      _stream(stream)), "aot_mlp_forward")
        return y

    def loss_grad(self, x, target, mask, stream=None):
        b = x.shape[0]
        grad = torch.empty(self.n_params - 2 * self.n_in, dtype=torch.float32,
                           device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        ws = self._ws(b)
        net = self.cstruct()
        _check(load().aot_mlp_loss_grad(ctypes.byref(net), _ptr(x.contiguous()),
                                        _ptr(target.contiguous()), _ptr(mask.contiguous()), b,
                                        _ptr(grad), _ptr(loss), _ptr(ws), ws.numel(),
                                        _stream(stream)), "aot_mlp_loss_grad")
        return float(loss.item()), grad

    def train(self, x, target, mask, epochs: int, lr: float, stream=None):
        b = x.shape[0]
        losses = (ctypes.c_float * max(epochs, 1))()
        ws = self._ws(b)
        net = self.cstruct()
        _check(load().aot_mlp_train(ctypes.byref(net), _ptr(x.contiguous()),
                                    _ptr(target.contiguous()), _ptr(mask.contiguous()), b,
                                    epochs, lr, losses, _ptr(ws), ws.numel(), _stream(stream)),
               "aot_mlp_train")
        return [losses[i] for i in range(epochs)]


@dataclass
class Counted:
    """Result of aot_count; keeps the workspace that aot_list needs."""
    T: int
    probes: int
    tri_off: torch.Tensor
    ws: torch.Tensor


def orient_workspace(n: int, nnz: int) -> int:
    b = ctypes.c_size_t(0)
    _check(load().aot_orient_workspace(n, nnz, ctypes.byref(b)), "aot_orient_workspace")
    return b.value


def count_workspace(n: int, m: int) -> int:
    b = ctypes.c_size_t(0)
    _check(load().aot_count_workspace(n, m, ctypes.byref(b)), "aot_count_workspace")
    return b.value


def alloc_oriented(n: int, m: int, device) -> Oriented:
    """Output buffers of aot_orient for a graph with n vertices and m edges."""
    i32 = dict(dtype=torch.int32, device=device)
    i64 = dict(dtype=torch.int64, device=device)
    return Oriented(n, m, torch.empty(n + 1, **i64), torch.empty(m, **i32),
                    torch.empty(m, **i32), torch.empty(n, **i32), torch.empty(n, **i32),
                    torch.empty(n + 1, **i64), torch.empty(m, **i32))


def orient(rowptr: torch.Tensor, col: torch.Tensor, validate: bool = False, stream=None,
           ws: torch.Tensor | None = None, out: Oriented | None = None,
           in_by_rank: bool = False, order: str = "degree", local: str = "rank") -> Oriented:
    """aot_orient on a symmetric device CSR (rowptr int64[n+1], col int32[nnz]);
    order "degree" (Algorithm 3) or "core" (kClist's, AOT_ORDER_CORE); local
    "rank" (labels are ranks: the degree local order of Section 3.2) or "id"
    (labels are original ids, AOT_LOCAL_BY_ID: AOT-randomOrder of Section 4.2
    on inputs with permuted ids)."""
    if order not in ("degree", "core"):
        raise ValueError(f"unknown order {order!r}")
    if local not in ("rank", "id"):
        raise ValueError(f"unknown local order {local!r}")
    assert rowptr.dtype == torch.int64 and col.dtype == torch.int32
    assert rowptr.is_contiguous() and col.is_contiguous()
    dev = rowptr.device
    n = rowptr.numel() - 1
    nnz = col.numel()
    m = nnz // 2
    o = out if out is not None else alloc_oriented(n, m, dev)
    assert (o.n, o.m) == (n, m)
    need = orient_workspace(n, nnz)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    g = Graph(n, nnz, _ptr(rowptr) or ctypes.c_void_p(rowptr.data_ptr()), _ptr(col))
    oc = o.cstruct()
    flags = (AOT_VALIDATE if validate else 0) | (AOT_IN_LISTS_BY_RANK if in_by_rank else 0) | (
        AOT_ORDER_CORE if order == "core" else 0) | (AOT_LOCAL_BY_ID if local == "id" else 0)
    _check(load().aot_orient(ctypes.byref(g), flags, ctypes.byref(oc),
                             _ptr(ws), ws.numel(), _stream(stream)), "aot_orient")
    return o


def count(o: Oriented, dispatch: Dispatch | None = None, stream=None,
          ws: torch.Tensor | None = None, tri_off: torch.Tensor | None = None) -> Counted:
    """aot_count: per-edge triangle offsets, T and the probe count."""
    dev = o.rowptr.device
    need = count_workspace(o.n, o.m)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    if tri_off is None:
        tri_off = torch.empty(o.m + 1, dtype=torch.int64, device=dev)
    res = (ctypes.c_uint64 * 2)()
    oc = o.cstruct()
    dc = (dispatch or Dispatch()).cstruct()
    _check(load().aot_count(ctypes.byref(oc), ctypes.byref(dc), _ptr(tri_off), _ptr(ws),
                            ws.numel(), res, _stream(stream)), "aot_count")
    return Counted(int(res[0]), int(res[1]), tri_off, ws)


def count_noalloc(o: Oriented, tri_off: torch.Tensor, dispatch: Dispatch | None = None,
                  stream=None) -> tuple[int, int]:
    """aot_count_noalloc: the count pass with the library's fixed scratch as
    its workspace (no allocation); writes tri_off and returns (T, probes)."""
    assert tri_off.dtype == torch.int64 and tri_off.numel() >= o.m + 1
    res = (ctypes.c_uint64 * 2)()
    oc = o.cstruct()
    dc = (dispatch or Dispatch()).cstruct()
    _check(load().aot_count_noalloc(ctypes.byref(oc), ctypes.byref(dc), _ptr(tri_off), res,
                                    _stream(stream)), "aot_count_noalloc")
    return int(res[0]), int(res[1])


def list_triangles(o: Oriented, c: Counted, first: int = 0, count: int | None = None,
                   out: torch.Tensor | None = None, dispatch: Dispatch | None = None,
                   stream=None) -> torch.Tensor:
    """aot_list: triangles [first, first+count) as an int32 (k, 3) device tensor."""
    if count is None:
        count = max(0, c.T - first)
    k = max(0, min(count, c.T - first))
    if out is None:
        out = torch.empty((max(k, 0), 3), dtype=torch.int32, device=o.rowptr.device)
    oc = o.cstruct()
    dc = (dispatch or Dispatch()).cstruct()
    _check(load().aot_list(ctypes.byref(oc), ctypes.byref(dc), _ptr(c.tri_off), _ptr(c.ws),
                           c.ws.numel(), first, k, _ptr(out), None, _stream(stream)), "aot_list")
    return out[:k]


def digest(o: Oriented, c: Counted, vertex_counts: bool = True,
           dispatch: Dispatch | None = None, stream=None):
    """aot_digest: (T, hash sum, hash xor) and per-vertex counts (uint64 as
    int64 device tensor) of the triangle list, without storing it."""
    vc = torch.empty(max(o.n, 1), dtype=torch.int64, device=o.rowptr.device) if vertex_counts else None
    res = (ctypes.c_uint64 * 3)()
    oc = o.cstruct()
    dc = (dispatch or Dispatch()).cstruct()
    _check(load().aot_digest(ctypes.byref(oc), ctypes.byref(dc), _ptr(c.tri_off), _ptr(c.ws),
                             c.ws.numel(), _ptr(vc), res, _stream(stream)), "aot_digest")
    return (int(res[0]), int(res[1]), int(res[2])), (vc[:o.n] if vc is not None else None)


def support(o: Oriented, c: Counted, vertex_counts: bool = True, stream=None):
    """aot_support: triangles through each oriented edge (int32 device
    tensor [m], in the edge order of o.col), through each original vertex
    (int64 device tensor [n] or None) and the digest (T, hash sum, hash xor)."""
    dev = o.rowptr.device
    es = torch.empty(max(o.m, 1), dtype=torch.int32, device=dev)
    vc = torch.empty(max(o.n, 1), dtype=torch.int64, device=dev) if vertex_counts else None
    res = (ctypes.c_uint64 * 3)()
    oc = o.cstruct()
    _check(load().aot_support(ctypes.byref(oc), None, _ptr(c.tri_off), _ptr(c.ws), c.ws.numel(),
                              _ptr(es), _ptr(vc), res, _stream(stream)), "aot_support")
    return es[:o.m], (vc[:o.n] if vc is not None else None), (int(res[0]), int(res[1]),
                                                               int(res[2]))


def count_plan(o: Oriented, c: Counted):
    """The table the last aot_count resolved and whether the cost model chose it."""
    t = (ctypes.c_int32 * AOT_NUM_BUCKETS)()
    learned = ctypes.c_int32(0)
    _check(load().aot_count_plan(_ptr(c.ws), c.ws.numel(), o.n, o.m, t, ctypes.byref(learned)),
           "aot_count_plan")
    return list(t), bool(learned.value)


def bucket_features(o: Oriented, c: Counted):
    """(features float32 [32, 8], present bool [32]) of the last aot_count."""
    import numpy as np
    f = (ctypes.c_float * (AOT_NUM_BUCKETS * AOT_NUM_FEATURES))()
    pr = (ctypes.c_uint8 * AOT_NUM_BUCKETS)()
    _check(load().aot_bucket_features(_ptr(c.ws), c.ws.numel(), o.n, o.m, f, pr),
           "aot_bucket_features")
    return (np.ctypeslib.as_array(f).reshape(AOT_NUM_BUCKETS, AOT_NUM_FEATURES).copy(),
            np.ctypeslib.as_array(pr).astype(bool).copy())


def timing_start():
    """Starts the per-launch recorder of this thread."""
    _check(load().aot_timing_start(), "aot_timing_start")


def timing_stop(cap: int = 4096) -> list[dict]:
    """Stops recording; returns one dict per recorded bucket launch."""
    buf = (TimingC * cap)()
    n = ctypes.c_int32(0)
    _check(load().aot_timing_stop(buf, cap, ctypes.byref(n)), "aot_timing_stop")
    keys = ("bucket", "arm", "tile", "edges", "probes", "staged", "triangles", "ms", "lookups")
    return [dict({"pass": buf[i].pass_}, **{k: getattr(buf[i], k) for k in keys})
            for i in range(min(n.value, cap))]


# ---------------------------------------------------------------- batches

@dataclass
class Batch:
    """A batch of graphs in one arena (see aot_batch): graph g owns arena
    vertices [voff[g], voff[g+1]); rowptr/col are the union CSR (device)."""
    voff: torch.Tensor       # host int64 [count+1]
    voff_dev: torch.Tensor   # device int64 [count+1]
    rowptr: torch.Tensor     # device int64 [n+1]
    col: torch.Tensor        # device int32 [nnz]

    @property
    def count(self) -> int:
        return self.voff.numel() - 1

    @property
    def n(self) -> int:
        return self.rowptr.numel() - 1

    @property
    def nnz(self) -> int:
        return self.col.numel()

    def cstruct(self) -> BatchC:
        self._voff = self.voff.contiguous()
        g = Graph(self.n, self.nnz, ctypes.c_void_p(self.rowptr.data_ptr()), _ptr(self.col))
        return BatchC(self.count, ctypes.c_void_p(self._voff.data_ptr()),
                      ctypes.c_void_p(self.voff_dev.data_ptr()), g)


@dataclass
class Schedule:
    """What the autotuner picks for the persistent passes (aot_schedule)."""
    heavy_min: int = 0
    table: list | None = None
    light_rounds: int = 0

    def cstruct(self) -> ScheduleC:
        t = (ctypes.c_int32 * AOT_NUM_BUCKETS)(*(self.table or [0] * AOT_NUM_BUCKETS))
        return ScheduleC(self.heavy_min, 1 if self.table is not None else 0, t,
                         self.light_rounds)


@dataclass
class BatchRun:
    """Buffers of one batch pass: the arena's oriented graph, per-edge and
    per-graph triangle offsets, the triangle window [0, cap) and the
    workspace (which also serves aot_list on the arena afterwards)."""
    o: Oriented
    tri_off: torch.Tensor
    graph_tri: torch.Tensor
    tri: torch.Tensor
    ws: torch.Tensor

    def counted(self) -> Counted:
        t = int(self.graph_tri[-1].item())
        return Counted(t, -1, self.tri_off, self.ws)


def batch_workspace(b: Batch) -> int:
    n = ctypes.c_size_t(0)
    bc = b.cstruct()
    _check(load().aot_batch_workspace(ctypes.byref(bc), ctypes.byref(n)), "aot_batch_workspace")
    return n.value


def alloc_batch(b: Batch, cap: int) -> BatchRun:
    dev = b.rowptr.device
    o = alloc_oriented(b.n, b.nnz // 2, dev)
    return BatchRun(o, torch.empty(o.m + 1, dtype=torch.int64, device=dev),
                    torch.empty(b.count + 1, dtype=torch.int64, device=dev),
                    torch.empty((max(cap, 0), 3), dtype=torch.int32, device=dev),
                    torch.empty(max(batch_workspace(b), 1), dtype=torch.uint8, device=dev))


def batch_run(b: Batch, cap: int, schedule: Schedule | None = None, run: BatchRun | None = None,
              stream=None) -> BatchRun:
    """aot_batch_run: orient, count and list the whole batch in one pass
    (enqueued, no synchronisation)."""
    r = run if run is not None else alloc_batch(b, cap)
    assert r.tri.shape[0] >= cap
    bc, oc = b.cstruct(), r.o.cstruct()
    sc = schedule.cstruct() if schedule is not None else None
    _check(load().aot_batch_run(ctypes.byref(bc), ctypes.byref(sc) if sc is not None else None,
                                ctypes.byref(oc), _ptr(r.tri_off), _ptr(r.graph_tri), _ptr(r.tri),
                                cap, _ptr(r.ws), r.ws.numel(), _stream(stream)), "aot_batch_run")
    return r


class BatchGraph:
    """aot_batch_run captured once in a HIP graph; launch() replays it."""

    def __init__(self, b: Batch, cap: int, schedule: Schedule | None = None,
                 run: BatchRun | None = None):
        self.b = b
        self.run = run if run is not None else alloc_batch(b, cap)
        bc, oc = b.cstruct(), self.run.o.cstruct()
        sc = schedule.cstruct() if schedule is not None else None
        h = ctypes.c_void_p(None)
        r = self.run
        _check(load().aot_batch_capture(ctypes.byref(bc),
                                        ctypes.byref(sc) if sc is not None else None,
                                        ctypes.byref(oc), _ptr(r.tri_off), _ptr(r.graph_tri),
                                        _ptr(r.tri), cap, _ptr(r.ws), r.ws.numel(),
                                        ctypes.byref(h)), "aot_batch_capture")
        self._h = h

    def launch(self, stream=None):
        _check(load().aot_batch_launch(self._h, _stream(stream)), "aot_batch_launch")

    def close(self):
        if self._h:
            load().aot_batch_destroy(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- streaming

def stream_list(o: Oriented, c: Counted, chunk: int, consume=None, first: int = 0,
                last: int | None = None, dispatch: Dispatch | None = None,
                to_host: bool = True, stream=None):
    """Lists triangles [first, last) window by window (aot_list into a device
    buffer of `chunk` triangles) and, with to_host, copies each window to
    one of two pinned host buffers on a second stream while the next window
    is being listed into the other of two device buffers.  consume(first_index, host_view) is called
    for each window in order; the view stays valid until the call returns.
    Returns the number of windows."""
    last = c.T if last is None else min(last, c.T)
    if last <= first:
        return 0
    dev = o.rowptr.device
    k = max(1, min(chunk, last - first))
    cs = stream if stream is not None else torch.cuda.current_stream()
    # without host copies one device buffer suffices (the windows are
    # listed one after another on one stream)
    one = torch.empty((k, 3), dtype=torch.int32, device=dev)
    dbuf = [one, torch.empty((k, 3), dtype=torch.int32, device=dev) if to_host else one]
    hbuf, xs = None, None
    if to_host:
        hbuf = [torch.empty((k, 3), dtype=torch.int32, pin_memory=True) for _ in range(2)]
        xs = torch.cuda.Stream(device=dev)          # default priority
    pending = [None, None]       # per slot: (event, first index, count)

    def finish(slot):
        ev, f, n = pending[slot]
        ev.synchronize()
        if consume is not None:
            consume(f, hbuf[slot][:n] if to_host else dbuf[slot][:n])
        pending[slot] = None

    windows = 0
    for i, f in enumerate(range(first, last, k)):
        slot = i % 2
        n = min(k, last - f)
        if pending[slot] is not None:
            finish(slot)          # the copy out of this slot is done and consumed
        list_triangles(o, c, first=f, count=n, out=dbuf[slot], dispatch=dispatch, stream=cs)
        done = torch.cuda.Event()
        done.record(cs)
        if to_host:
            xs.wait_event(done)
            with torch.cuda.stream(xs):
                hbuf[slot][:n].copy_(dbuf[slot][:n], non_blocking=True)
                copied = torch.cuda.Event()
                copied.record(xs)
            pending[slot] = (copied, f, n)
        else:
            # one shared device buffer: hand the window over before the next
            # one overwrites it
            pending[slot] = (done, f, n)
            finish(slot)
        windows += 1
    for j in range(windows, windows + 2):
        if pending[j % 2] is not None:
            finish(j % 2)
    return windows
