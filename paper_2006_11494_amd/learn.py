"""Learned dispatch of the probe kernels.

The cost model (an Mlp, trained and run by the library's HIP kernels) maps a
bucket's features -- computed by the count pass from its own binning -- to
the predicted log(ns per probe) of each dispatch option: a light bin's lanes
per edge (4, 8, 16, 32, 64) or a heavy owner class's LDS index (bitmap, hash,
global binary search, sorted copy).  Training data are the per-bucket timings
the method records about itself (aot_timing_*) while exploration tables force
each option in turn.  This module only orchestrates those calls: which tables
to run, which rows to keep; all arithmetic of the model runs on the GPU.

The plain rule stays both the fallback (a model that is missing, malformed or
not finite is ignored by the library) and the judge: a trained model is kept
only if, on calibration graphs it was not trained on, its plans run faster
than the plain rule's.

The heavy/light boundary decides which buckets exist at all, so the model is
not asked to choose it: exploration covers every BOUNDARIES value, and the
judge times the model's plans at each and keeps the faster.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

from . import aot, inputs

TILES = (4, 8, 16, 32, 64)          # options 0..4 (light bins)
BOUNDARIES = (0, 32)                # heavy_min: the library default (64), and 32
ARMS = (0, 1, 2, 3)                 # options 5..8 (heavy classes): bitmap, hash, global, sorted
N_EXPLORE = 5


def exploration_table(i: int) -> list[int]:
    """Table i forces light tile TILES[i] on every light bin and arm i % 4 on
    every heavy class, so five tables cover every option."""
    t = [0] * aot.AOT_NUM_BUCKETS
    for k in range(8):
        t[k] = TILES[i] << 8
    for h in range(16):
        t[16 + h] = ARMS[i % 4]
    return t


def option_of(bucket: int, i: int) -> int:
    return i if bucket < 16 else 5 + (i % 4)


def plain_table() -> list[int]:
    t = [0] * aot.AOT_NUM_BUCKETS
    for k, tile in enumerate((4, 4, 4, 8, 16, 32, 64, 64)):
        t[k] = tile << 8
    return t


RESIDENT = 1 << 28     # lists up to this many triangles go into one buffer


def out_buffer(c, device):
    """Output buffer for timing runs: the whole list, or one window of it."""
    return torch.empty((max(1, min(c.T, RESIDENT)), 3), dtype=torch.int32, device=device)


def list_all(o, c, d, out):
    """The whole write pass: into `out` if it holds the list, else window by
    window (device windows, nothing copied to the host)."""
    if c.T <= out.shape[0]:
        aot.list_triangles(o, c, out=out, dispatch=d)
    else:
        aot.stream_list(o, c, out.shape[0], None, dispatch=d, to_host=False)


def _timed(o, d, repeats: int, out):
    """Per-bucket milliseconds (count + write launch) averaged over repeats,
    after one untimed warm-up, and the bucket's probe counts (from the count
    pass's records)."""
    ms: dict[int, float] = {}
    probes: dict[int, int] = {}
    for r in range(repeats + 1):
        aot.timing_start()
        c = aot.count(o, d)
        list_all(o, c, d, out)
        recs = aot.timing_stop(cap=1 << 17)
        if r == 0:
            continue
        for rec in recs:
            ms[rec["bucket"]] = ms.get(rec["bucket"], 0.0) + rec["ms"] / repeats
            if rec["pass"] == 0:          # the count pass covers every bucket whole
                probes[rec["bucket"]] = rec["probes"]
    return ms, probes


def record(csr, repeats: int = 3, boundaries=BOUNDARIES):
    """Exploration on one graph, binned at each heavy/light boundary in turn:
    rows (features[8], option, log ns per probe)."""
    o = aot.orient(csr.rowptr, csr.col)
    rows = []
    out = None
    for hm in boundaries:
        c = aot.count(o, aot.Dispatch(aot.AOT_DISPATCH_PLAIN, hm))
        feats, present = aot.bucket_features(o, c)
        if out is None:
            out = out_buffer(c, csr.rowptr.device)
        for i in range(N_EXPLORE):
            d = aot.Dispatch(aot.AOT_DISPATCH_TABLE, hm, exploration_table(i))
            ms, probes = _timed(o, d, repeats, out)
            for b, t in ms.items():
                if not present[b]:
                    continue
                y = math.log(max(t, 1e-6) * 1e6 / max(probes.get(b, 1), 1))
                rows.append((feats[b].copy(), option_of(b, i), y))
    return rows


@dataclass
class Dataset:
    x: torch.Tensor       # [N, 8] float32
    target: torch.Tensor  # [N, 9] float32
    mask: torch.Tensor    # [N, 9] uint8


def dataset(rows, device="cuda") -> Dataset:
    n = len(rows)
    x = np.zeros((n, aot.AOT_NUM_FEATURES), np.float32)
    t = np.zeros((n, aot.AOT_NUM_OPTIONS), np.float32)
    m = np.zeros((n, aot.AOT_NUM_OPTIONS), np.uint8)
    for i, (f, opt, y) in enumerate(rows):
        x[i] = f
        t[i, opt] = y
        m[i, opt] = 1
    return Dataset(torch.from_numpy(x).to(device), torch.from_numpy(t).to(device),
                   torch.from_numpy(m).to(device))


def train(data: Dataset, hidden: int = 16, epochs: int = 1000, lr: float = 3e-3,
          seed: int = 7) -> tuple[aot.Mlp, list[float]]:
    net = aot.Mlp(n_hidden=hidden, device=data.x.device).init(seed)
    losses = net.train(data.x, data.target, data.mask, epochs, lr)
    return net, losses


def step_ms(o, d, repeats: int, out) -> float:
    """Median wall time of count + list with dispatch d."""
    ts = []
    for r in range(repeats + 1):
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        c = aot.count(o, d)
        list_all(o, c, d, out)
        b.record()
        torch.cuda.synchronize()
        if r:
            ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def judge(net: aot.Mlp, graphs, repeats: int = 5, margin: float = 0.02,
          boundaries=BOUNDARIES):
    """Plain vs learned time (ms) summed over calibration graphs, the learned
    plans timed at every boundary.  Returns (plain ms, learned ms at the best
    boundary, accepted, that boundary); the model is accepted only if it is
    faster than the plain rule by more than `margin` (timing noise)."""
    plain = 0.0
    learned = {hm: 0.0 for hm in boundaries}
    for csr in graphs:
        o = aot.orient(csr.rowptr, csr.col)
        c = aot.count(o)
        out = out_buffer(c, csr.rowptr.device)
        plain += step_ms(o, None, repeats, out)
        for hm in boundaries:
            d = aot.Dispatch(aot.AOT_DISPATCH_LEARNED, hm, None, net)
            learned[hm] += step_ms(o, d, repeats, out)
    best = min(boundaries, key=lambda hm: learned[hm])
    return plain, learned[best], learned[best] < plain * (1.0 - margin), best


def training_graphs(device="cuda", scale: int = 1):
    """Seeded graphs of every family the workloads use (seeds >= 1000, disjoint
    from the benchmark's)."""
    return [
        inputs.rmat(15 + scale, 16, 1001, device=device),
        inputs.rmat(14 + scale, 32, 1002, device=device),
        inputs.rmat(16 + scale, 8, 1003, device=device),
        inputs.chung_lu(100_000 * scale, 40.0, 2.1, 10_000.0, 1004, device=device),
        inputs.chung_lu(200_000 * scale, 20.0, 2.1, 20_000.0, 1005, device=device),
        inputs.erdos_renyi_m(50_000 * scale, 48.0, 1006, device=device),
        inputs.random_geometric(100_000 * scale, 20.0, 1007, device=device),
    ]


def calibration_graphs(device="cuda", scale: int = 1):
    return [inputs.rmat(16 + scale, 16, 1010, device=device),
            inputs.chung_lu(150_000 * scale, 40.0, 2.1, 20_000.0, 1011, device=device)]


def workload_graphs(workload: str, seeds, device="cuda"):
    """Graphs of a named workload's own recipe with other seeds (>= 1000)."""
    return [inputs.workload(workload, s, device=device) for s in seeds]


def learn(training=None, calibration=None, device="cuda", scale: int = 1, epochs: int = 1000,
          repeats: int = 3, log=None):
    """Exploration on the training graphs, training, and the judge on the
    calibration graphs.  Returns (model or None if the judge rejects it,
    report); report["heavy_min"] is the boundary to use the model at."""
    training = training if training is not None else training_graphs(device, scale)
    calibration = calibration if calibration is not None else calibration_graphs(device, scale)
    rows = []
    for csr in training:
        rows += record(csr, repeats)
        if log:
            log(f"[learn] explored {csr.name}: {len(rows)} rows")
    data = dataset(rows, device)
    net, losses = train(data, epochs=epochs)
    plain, learned, ok, heavy_min = judge(net, calibration)
    report = {"rows": len(rows), "loss_first": losses[0] if losses else None,
              "loss_last": losses[-1] if losses else None, "judge_plain_ms": plain,
              "judge_learned_ms": learned, "accepted": ok, "heavy_min": heavy_min,
              "training": [g.name for g in training], "calibration": [g.name for g in calibration]}
    if log:
        log(f"[learn] loss {report['loss_first']:.3f} -> {report['loss_last']:.3f}; judge: "
            f"plain {plain:.3f} ms, learned {learned:.3f} ms (heavy_min {heavy_min or 'default'})"
            f" -> {'accept' if ok else 'reject'}")
    return (net if ok else None), report
