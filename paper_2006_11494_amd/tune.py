"""Autotuner of the batched form's schedule (aot_schedule).

The persistent passes take four kinds of choices: the light/heavy boundary
heavy_min (which owners get an LDS index), the lanes per edge of every light
bin, the LDS index arm of every heavy owner class, and how many edges one
light task holds.  Every choice gives the same bytes, so the tuner may try
anything: it times whole batch passes (the library's own kernels, HIP events
on the stream) and walks the choices one coordinate at a time from the plain
rule, keeping a change only when the pass gets faster by more than the
noise margin.  The tuned schedule is therefore never slower than the plain
rule on the batch it was tuned on.  Results can be cached on disk (JSON)
under a key that describes the batch's shape.
"""

from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np
import torch

from . import aot, learn

HEAVY_MINS = (8, 16, 32, 64, 128)
ROUNDS = (1, 2, 4, 8, 16)


def signature(b: aot.Batch) -> str:
    """Key of a batch's shape: graph count, sizes and a hash of the offsets."""
    h = hashlib.sha1(b.voff.numpy().tobytes()).hexdigest()[:16]
    return f"{b.count}:{b.n}:{b.nnz}:{h}"


def _table(sc: aot.Schedule) -> list[int]:
    return list(sc.table) if sc.table is not None else learn.plain_table()


def pass_ms(b: aot.Batch, run: aot.BatchRun, sc: aot.Schedule, cap: int, repeats: int = 3,
            stream=None) -> float:
    """Median time of one whole batch pass (orient, count, scan, write of
    [0, cap)) with schedule sc, after one untimed pass."""
    ts = []
    for r in range(repeats + 1):
        a = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        a.record()
        aot.batch_run(b, cap, schedule=sc, run=run, stream=stream)
        e.record()
        e.synchronize()
        if r:
            ts.append(a.elapsed_time(e))
    return float(np.median(ts))


def present_buckets(run: aot.BatchRun):
    """Which light bins and heavy classes hold edges after a pass."""
    _, present = aot.bucket_features(run.o, run.counted())
    return present


def tune(b: aot.Batch, cap: int | None = None, repeats: int = 3, margin: float = 0.01,
         cache: str | None = None, log=None) -> tuple[aot.Schedule, dict]:
    """Coordinate descent over (heavy_min, light_rounds, light tiles, heavy
    arms) from the plain rule.  cap defaults to the batch's T (whole list)."""
    key = signature(b)
    if cache and os.path.exists(cache):
        with open(cache) as f:
            stored = json.load(f)
        if key in stored:
            d = stored[key]
            return aot.Schedule(d["heavy_min"], d["table"], d["light_rounds"]), dict(
                d["report"], cached=True)
    t0 = time.time()
    probe = aot.batch_run(b, 0)
    torch.cuda.synchronize()
    T = int(probe.graph_tri[-1].item())
    cap = T if cap is None else cap
    run = aot.alloc_batch(b, cap)
    best = aot.Schedule(0, learn.plain_table(), 0)
    best_ms = plain_ms = pass_ms(b, run, best, cap, repeats)
    tried = 1

    def attempt(sc):
        nonlocal best, best_ms, tried
        ms = pass_ms(b, run, sc, cap, repeats)
        tried += 1
        if ms < best_ms * (1.0 - margin):
            best, best_ms = sc, ms
            return True
        return False

    for h in HEAVY_MINS:
        if h != (best.heavy_min or 64):
            attempt(aot.Schedule(h, _table(best), best.light_rounds))
    for r in ROUNDS:
        if r != (best.light_rounds or 4):
            attempt(aot.Schedule(best.heavy_min, _table(best), r))
    aot.batch_run(b, cap, schedule=best, run=run)
    torch.cuda.synchronize()
    present = present_buckets(run)
    for k in range(8):
        if not present[k]:
            continue
        for tile in learn.TILES:
            t = _table(best)
            if t[k] == tile << 8:
                continue
            t[k] = tile << 8
            attempt(aot.Schedule(best.heavy_min, t, best.light_rounds))
    for h in range(16):
        if not present[16 + h]:
            continue
        for arm in learn.ARMS:
            t = _table(best)
            if t[16 + h] == arm:
                continue
            t[16 + h] = arm
            attempt(aot.Schedule(best.heavy_min, t, best.light_rounds))
    report = {"plain_ms": plain_ms, "tuned_ms": best_ms, "tried": tried,
              "seconds": time.time() - t0, "T": T,
              "heavy_min": best.heavy_min, "light_rounds": best.light_rounds,
              "table": _table(best)}
    if log:
        log(f"[tune] {tried} schedules in {report['seconds']:.1f}s: plain {plain_ms:.3f} ms "
            f"-> tuned {best_ms:.3f} ms")
    if cache:
        stored = {}
        if os.path.exists(cache):
            with open(cache) as f:
                stored = json.load(f)
        stored[key] = {"heavy_min": best.heavy_min, "table": _table(best),
                       "light_rounds": best.light_rounds, "report": report}
        with open(cache, "w") as f:
            json.dump(stored, f)
    return best, report
