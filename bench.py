"""Benchmark of the AOT hot path on one MI355X.

One step = the whole path on one synthetic graph already resident in HBM:
aot_orient (degree-order ranking, orientation, out-list sort, in-lists),
aot_count (binning, probe count pass, scan) and aot_list (write pass of every
triangle into device memory).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload rmat20]

Prints one JSON line: value = triangles/s of the whole step, plus per-pass
times, probes/s, the dominant kernel's roofline (algorithmic bytes per launch
over its live HIP-event launch time) and the CPU oracle baseline.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


_T0 = time.time()


def log(*a):
    print(f"[{time.time() - _T0:7.1f}s]", *a, file=sys.stderr, flush=True)


HEADLINE = "rmat26"
# the other configurations, measured as extra keys of the headline run
EXTRAS = ("rmat20", "chunglu4m")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--workload", default=HEADLINE)
    p.add_argument("--seed", type=int, default=None)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample", type=float, default=None,
                   help="fraction of the oriented edges the CPU oracle lists (default 0.5, "
                        "or 0.01 for a list listed in windows)")
    p.add_argument("--heavy-arm", default=None, choices=["bitmap", "hash", "global", "sorted"],
                   help="force one index arm for every heavy owner class")
    p.add_argument("--heavy-min", type=int, default=0)
    p.add_argument("--no-learned", action="store_true",
                   help="skip the learned-dispatch legs (training the cost model)")
    p.add_argument("--learned-steps", type=int, default=3,
                   help="timed steps of each of plain and learned in the learned leg")
    p.add_argument("--no-ablation", action="store_true",
                   help="skip the probe-strategy ablation (fixed orientation, CF merge, per edge)")
    p.add_argument("--no-batch", action="store_true",
                   help="skip the batched leg (512 uneven graphs, one captured pass)")
    p.add_argument("--no-extras", action="store_true",
                   help="headline workload only: skip the other configurations' legs")
    p.add_argument("--batch-count", type=int, default=512)
    p.add_argument("--resident-gb", type=float, default=48.0,
                   help="list into one device buffer up to this size, else in windows")
    p.add_argument("--chunk", type=int, default=1 << 33,
                   help="triangles per device window when the list is not resident "
                        "(capped at 60%% of the free device memory)")
    p.add_argument("--stream-chunk", type=int, default=1 << 29,
                   help="triangles per window streamed to pinned host memory")
    p.add_argument("--stream", action="store_true",
                   help="also stream every window of a list too large to hold to pinned host "
                        "memory (the PCIe-inclusive rate; about a minute at R-MAT scale 26)")
    p.add_argument("--save-csr", default=None, metavar="PREFIX",
                   help="only generate the workload and save its CSR to PREFIX_rowptr.npy and "
                        "PREFIX_col.npy (for a profiled run that should not run the generator)")
    p.add_argument("--load-csr", default=None, metavar="PREFIX",
                   help="read the workload's CSR from files written by --save-csr instead of "
                        "generating it")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain 1 GiB read + 1 GiB write elementwise kernel, the "
                        "reference that scales rocprofv3's FETCH_SIZE / WRITE_SIZE counters")
    return p.parse_args()


def copy_calibration():
    import torch

    n = (1 << 30) // 4
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.add(src, 1, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"read_bytes": 4 * n, "write_bytes": 4 * n,
                                           "launches": 3}}), flush=True)


def copy_bandwidth(reps: int = 5) -> float:
    """Achievable HBM bandwidth on this device: a 1 GiB device-to-device copy
    (1 GiB read + 1 GiB written), median of `reps` timed with events."""
    import torch

    n = (1 << 30) // 4
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    ts = []
    for _ in range(reps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        dst.copy_(src)
        ev[1].record()
        ev[1].synchronize()
        ts.append(ev[0].elapsed_time(ev[1]))
    del src, dst
    return 2 * 4 * n / (sorted(ts)[reps // 2] / 1000.0) / 1e9


# Algorithmic bytes of one bucket launch (what the method must move):
#  count pass: 4 B per look-up made (the probed out-list id; heavy owners skip
#    each probed list's lines below their smallest out-neighbour), 4 B per
#    staged owner list entry, 8 B per edge (its id and its count);
#  write pass: the same (heavy owners probe from each edge's first hit) plus,
#    per edge, 8 B for its two triangle offsets and 4 B for the original id of
#    its probed endpoint, and per triangle 4 B for the original id of its third
#    vertex (the list is in original ids: perm of the hit) and 12 B written.
def launch_bytes(r) -> int:
    looks = r.get("lookups", r["probes"])
    b = 4 * looks + 4 * r["staged"] + 8 * r["edges"]
    if r["pass"] == 1:
        b += 12 * r["edges"] + 16 * r["triangles"]
    return b


def kernel_of(r) -> str:
    path = "k_heavy" if r["bucket"] >= 16 else f"k_light<{r['tile']}>"
    return f"{path}<{'write' if r['pass'] == 1 else 'count'}>"


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("count.hip", "common.hpp", "kernels.hpp"):
        with open(os.path.join(ROOT, "paper_2006_11494_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(kernel: str, workload: str, launches: int):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary (its bytes over one whole pass, spread over this run's `launches`
    launches of that pass), or None when there is none for this kernel and
    workload or the kernel source changed since it was taken."""
    if kernel not in ("k_heavy<write>", "k_heavy<count>"):
        return None
    path = os.path.join(ROOT, "profiles", f"k_heavy_write_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        prof = json.load(f)
    if prof.get("source_hash") != kernel_source_hash():
        return None
    if kernel == "k_heavy<count>":        # the same runs' figures for the count pass
        prof = prof["count_pass"]
    return prof["traffic_bytes_per_pass"] / max(launches, 1)


def roofline(recs, workload: str, windowed: bool = False):
    """HBM roofline of the kernel with the most recorded time.  Windowed
    listing splits a bucket's write work over many launches: then a write
    kernel's algorithmic bytes are those of its buckets' whole write pass
    over the summed time of all its write launches.  A heavy write record
    carries its whole bucket's figures (the write pass probes the hit spans
    the count pass found); a light bin's write work is its count-pass
    record's, plus the triangles."""
    per = {}
    seen = set()
    count_rec = {r["bucket"]: r for r in recs if r["pass"] == 0}
    for r in recs:
        k = kernel_of(r)
        d = per.setdefault(k, {"ms": 0.0, "bytes": 0, "launches": 0})
        d["ms"] += r["ms"]
        d["launches"] += 1
        if not windowed:
            d["bytes"] += launch_bytes(r)
        elif (r["pass"], r["bucket"]) not in seen:
            seen.add((r["pass"], r["bucket"]))
            whole = r if r["pass"] == 0 or r["probes"] >= 0 else \
                dict(count_rec[r["bucket"]], **{"pass": 1})
            d["bytes"] += launch_bytes(whole)
    kern, d = max(((k, v) for k, v in per.items() if v["launches"]), key=lambda kv: kv[1]["ms"])
    achieved = d["bytes"] / (d["ms"] / 1000.0) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": profiled_traffic(kern, workload, d["launches"]),
            "kernel": kern,
            "launches": d["launches"], "avg_launch_ms": d["ms"] / d["launches"],
            "bytes_per_launch": d["bytes"] / d["launches"],
            "per_unit": "4 B/look-up made + 4 B/staged owner-list entry + 8 B/edge"
                        " (+ 12 B/edge and 16 B/triangle in the write pass: offsets,"
                        " original ids read, 12 B written); heavy owners probe each"
                        " list from its line below their smallest out-neighbour (count)"
                        " or from the edge's first hit (write)"}


def cpu_baseline(csr, frac: float, threads: int = 1):
    """The CPU oracle (plain C, one thread) on a bounded sample of the same
    graph: orientation of the whole graph, then the oracle's CF listing over
    64 source-rank ranges spread across the edge list that together hold
    about `frac` of the oriented edges; triangles/s extrapolated to the
    whole graph as (T_sample / f) / (t_orient + t_list / f)."""
    import numpy as np

    import oracle

    from concurrent.futures import ThreadPoolExecutor

    rp, col = csr.numpy()
    t0 = time.perf_counter()
    o = oracle.orient(rp, col) if threads == 1 else oracle.orient_threaded(rp, col, threads, log)
    t_orient = time.perf_counter() - t0
    m = o.m
    k = 64
    ranges = []
    if frac >= 1.0:
        # the whole graph: k consecutive rank ranges of about m / k edges each
        cuts = np.searchsorted(o.orow, np.linspace(0, m, k + 1).astype(np.int64), side="left")
        cuts[0], cuts[-1] = 0, o.n
        ranges = [(int(a), int(b)) for a, b in zip(cuts[:-1], cuts[1:]) if b > a]
    else:
        per = max(1, int(frac * m / k))
        for st in np.linspace(0, m, k, endpoint=False).astype(np.int64):
            r_lo = int(np.searchsorted(o.orow, st, side="right") - 1)
            r_hi = int(np.searchsorted(o.orow, min(m, st + per), side="left"))
            r_hi = max(r_hi, r_lo + 1)
            if not ranges or r_lo >= ranges[-1][1]:
                ranges.append((r_lo, min(r_hi, o.n)))
    edges = sum(int(o.orow[b] - o.orow[a]) for a, b in ranges)
    f = edges / max(m, 1)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        tri = sum(ex.map(lambda ab: len(oracle.list_triangles(o, ab[0], ab[1])), ranges))
    t_list = time.perf_counter() - t0
    value = (tri / f) / (t_orient + t_list / f)
    log(f"[bench] cpu oracle: orient {t_orient:.2f}s, list {t_list:.2f}s over {f * 100:.1f}% "
        f"of the edges ({tri} triangles)")
    return {"value": value, "unit": "triangles/s", "cores": threads, "kind": "oracle",
            "sample": f"orientation of the whole graph ({t_orient:.2f} s) + CF listing of "
                      f"{len(ranges)} source-rank ranges holding {f * 100:.1f}% of the oriented "
                      f"edges ({t_list:.2f} s, {tri} triangles), extrapolated to all edges; "
                      f"host: {os.cpu_count()} cores visible, oracle on {threads} thread(s)"}


def host_info():
    """CPU model and memory of the host the oracle ran on."""
    model, ram = None, None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                ram = round(int(line.split()[1]) / 2**20, 1)
                break
    except OSError:
        pass
    return {"cpu_model": model, "ram_gib": ram, "cores_visible": os.cpu_count()}


# Graphs the cost model trains and is judged on when the workload itself is
# too large to hold twice: same recipe, smaller scale, other seeds.
PROXY = {"rmat26": ("rmat22x32", "rmat23x32")}
JUDGE_PROXY = {"rmat26": "rmat24x32"}


def alternate_ms(fns, reps):
    """Wall time per call of each fn (ms), the fns run in turn `reps` times
    after one untimed round, so that drift hits every fn alike; each call is
    bracketed by device synchronisation.  Returns the mean of each."""
    import torch

    tot = [0.0] * len(fns)
    for r in range(reps + 1):
        for i, fn in enumerate(fns):
            torch.cuda.synchronize()
            t = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            if r:
                tot[i] += (time.perf_counter() - t) * 1000.0
    return [x / max(reps, 1) for x in tot]


def learned_leg(aot, name, o, step, T, probes, reps, log, scale=2, repeats=2):
    """Train the cost model on other graphs (seeds >= 1000), judge it on a
    calibration graph, then time the whole step with the plain rule and with
    the learned dispatch in turn (same timing, recorder off) on this graph."""
    from paper_2006_11494_amd import learn

    t0 = time.time()
    # training: the standard family mix plus two graphs of this workload's own
    # recipe; judge: a third graph of the recipe (all seeds >= 1000)
    names = PROXY.get(name, (name, name))
    training = learn.training_graphs(scale=scale) + [
        learn.workload_graphs(nm, (seed,))[0] for nm, seed in zip(names, (1021, 1022))]
    calibration = learn.workload_graphs(JUDGE_PROXY.get(name, name), (1020,))
    net, report = learn.learn(training, calibration, epochs=1000, repeats=repeats, log=log)
    del training, calibration
    train_s = time.time() - t0
    res = {"train_s": train_s, **report}
    if net is None:
        log(f"[bench] {name}: the judge kept the plain rule; the learned step is the plain step")
        return res
    d = aot.Dispatch(aot.AOT_DISPATCH_LEARNED, report["heavy_min"], None, net)
    got = {}

    def run(disp, key):
        cc = step(disp)
        assert (cc.T, cc.probes) == (T, probes)
        got[key] = cc

    plain_ms, learned_ms = alternate_ms([lambda: run(None, "plain"), lambda: run(d, "learned")],
                                        reps)
    table, used = aot.count_plan(o, got["learned"])
    log(f"[bench] {name}: plain {plain_ms:.3f} ms, learned {learned_ms:.3f} ms per step "
        f"({plain_ms / learned_ms:.3f}x, model used: {used})")
    res.update({"plain_ms_per_step": plain_ms, "ms_per_step": learned_ms,
                "value": T / (learned_ms / 1000.0), "unit": "triangles/s",
                "gain_vs_plain": plain_ms / learned_ms, "model_used": used, "plan": table,
                "timed_steps_each": reps,
                "timing": "plain and learned steps alternated, wall clock, recorder off"})
    return res


ABLATION_NOTE = ("count + list of the whole graph per (order, probe strategy): aot = adaptive "
                 "orientation (Algorithm 3); head = fixed orientation, kClist's cost; "
                 "merge = CF's merge intersections (Algorithm 1); per_edge = min side into "
                 "the larger list edge by edge, no per-owner index (CF-Hash); core_* = the "
                 "same on the core order (core_head: kClist's order and cost), whose "
                 "ms_orient includes the peeling; random_order = aot with original ids as "
                 "labels, i.e. a random local order on these permuted-id inputs "
                 "(AOT-randomOrder)")
# (name, order, labels, probe strategy)
ABLATION_CASES = (("aot", "degree", "rank", "aot"), ("head", "degree", "rank", "head"),
                  ("merge", "degree", "rank", "merge"),
                  ("per_edge", "degree", "rank", "per_edge"),
                  ("random_order", "degree", "id", "aot"),
                  ("core_aot", "core", "rank", "aot"), ("core_head", "core", "rank", "head"))


def ablation_leg(aot, csr, o, ows, cws, tri_off, out, T, args):
    """Section 4's comparisons on this graph: the same count + list with each
    probe strategy, on the degree order and on the core order, and with the
    local order of Section 3.2 replaced by id order.  All give the same
    triangles; probes are each strategy's cost on that order."""
    import torch

    def med(xs):
        return float(np.median(xs))

    reps = max(args.steps, 3)
    res = {}
    oriented = {("degree", "rank"): o}
    orient_ms = {("degree", "rank"): None}
    for name, order, labels, strategy in ABLATION_CASES:
        key = (order, labels)
        if key not in oriented:
            oo = aot.alloc_oriented(csr.n, csr.m, csr.rowptr.device)
            ts = []
            for r in range(reps + 1):
                ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
                ev[0].record()
                aot.orient(csr.rowptr, csr.col, out=oo, ws=ows, order=order, local=labels)
                ev[1].record()
                ev[1].synchronize()
                if r:
                    ts.append(ev[0].elapsed_time(ev[1]))
            oriented[key], orient_ms[key] = oo, med(ts)
        oo = oriented[key]
        d = aot.Dispatch(strategy=aot.STRATEGIES[strategy])
        cc = aot.count(oo, d, ws=cws, tri_off=tri_off)
        aot.list_triangles(oo, cc, out=out)
        assert cc.T == T
        tc, tl = [], []
        for _ in range(reps):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            ev[0].record()
            cc = aot.count(oo, d, ws=cws, tri_off=tri_off)
            ev[1].record()
            aot.list_triangles(oo, cc, out=out)
            ev[2].record()
            ev[2].synchronize()
            tc.append(ev[0].elapsed_time(ev[1]))
            tl.append(ev[1].elapsed_time(ev[2]))
        ms_c, ms_l = med(tc), med(tl)
        dmax = int((oo.rowptr[1:] - oo.rowptr[:-1]).max()) if csr.n else 0
        res[name] = {"order": order, "labels": labels, "strategy": strategy,
                     "probes": cc.probes,
                     "max_out_degree": dmax, "ms_orient": orient_ms[key],
                     "ms_count": ms_c, "ms_list": ms_l,
                     "triangles_per_s": T / ((ms_c + ms_l) / 1000.0)}
        log(f"[bench] {name}: probes {cc.probes} count {ms_c:.3f} ms list {ms_l:.3f} ms"
            + (f" (orient {orient_ms[key]:.3f} ms)" if orient_ms[key] else ""))
    base = res["aot"]["ms_count"] + res["aot"]["ms_list"]
    for r in res.values():
        r["aot_speedup"] = (r["ms_count"] + r["ms_list"]) / base
    del oriented
    res["note"] = ABLATION_NOTE
    return res


def _time_ms(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t) * 1000.0)
    return float(sorted(ts)[len(ts) // 2])


def batched_leg(aot, args, dev):
    """The uneven batch: 512 graphs (n log-uniform in [1e3, 2e5]; ER, R-MAT,
    RGG), listed (a) graph by graph through aot_orient / aot_count / aot_list,
    (b) as one persistent pass captured in a HIP graph, with the plain rule and
    with the schedule the autotuner picks on a tuning batch of other seeds."""
    import torch

    from paper_2006_11494_amd import inputs, tune

    t0 = time.time()
    csrs = [inputs.batch_member(s, device=dev) for s in inputs.batch_spec(args.batch_count, 4)]
    voff, rowptr, col = inputs.arena(csrs)
    b = aot.Batch(voff, voff.to(dev), rowptr, col)
    torch.cuda.synchronize()
    log(f"[batch] generated {b.count} graphs: n={b.n} m={b.nnz // 2} in {time.time() - t0:.1f}s")
    t0 = time.time()
    tcs = [inputs.batch_member(s, device=dev) for s in inputs.batch_spec(128, 1004)]
    tv, tr, tc = inputs.arena(tcs)
    tb = aot.Batch(tv, tv.to(dev), tr, tc)
    sched, rep = tune.tune(tb, log=log)
    del tcs, tb, tv, tr, tc
    log(f"[batch] tuned on 128 graphs of other seeds in {time.time() - t0:.1f}s")

    probe = aot.batch_run(b, 0)
    torch.cuda.synchronize()
    T = int(probe.graph_tri[-1].item())
    gtri = probe.graph_tri.cpu()
    del probe
    out = torch.empty((max(T, 1), 3), dtype=torch.int32, device=dev)
    max_n = max(c.n for c in csrs)
    max_nnz = max(c.nnz for c in csrs)
    # every buffer of the per-graph baseline is allocated once, outside the
    # timed loop: each graph's oriented arrays and offsets are views of them
    ows = torch.empty(aot.orient_workspace(max_n, max_nnz), dtype=torch.uint8, device=dev)
    cws = torch.empty(aot.count_workspace(max_n, max_nnz // 2), dtype=torch.uint8, device=dev)
    big = aot.alloc_oriented(max_n, max_nnz // 2, dev)
    toff = torch.empty(max_nnz // 2 + 1, dtype=torch.int64, device=dev)
    views = [aot.Oriented(c.n, c.m, big.rowptr[:c.n + 1], big.col[:c.m], big.tail[:c.m],
                          big.perm[:c.n], big.rank[:c.n], big.in_rowptr[:c.n + 1],
                          big.in_col[:c.m]) for c in csrs]
    per_T = []

    def per_graph():
        per_T.clear()
        pos = 0
        for c, o in zip(csrs, views):
            aot.orient(c.rowptr, c.col, out=o, ws=ows)
            cc = aot.count(o, ws=cws, tri_off=toff[:c.m + 1])
            aot.list_triangles(o, cc, out=out[pos:pos + cc.T])
            pos += cc.T
            per_T.append(cc.T)

    ms_per_graph = _time_ms(per_graph, 2)
    assert per_T == (gtri[1:] - gtri[:-1]).tolist(), "per-graph T differs from the batch"
    log(f"[batch] per-graph launches: {ms_per_graph:.1f} ms for T={T}")
    run = aot.alloc_batch(b, T)
    ms_eager = _time_ms(lambda: aot.batch_run(b, T, run=run), 3)
    g_plain = aot.BatchGraph(b, T, run=run)
    ms_graph_plain = _time_ms(g_plain.launch, 5)
    g_plain.close()
    g = aot.BatchGraph(b, T, schedule=sched, run=run)
    ms_graph = _time_ms(g.launch, 5)
    torch.cuda.synchronize()
    # the batched list equals the per-graph lists (sampled graphs, arena ids
    # shifted back to local ids)
    rng = np.random.default_rng(0)
    for j in sorted(set(rng.integers(0, b.count, 24).tolist()) | {int(np.argmax(per_T))}):
        lo, hi = int(gtri[j]), int(gtri[j + 1])
        assert torch.equal(run.tri[lo:hi] - int(voff[j]), out[lo:hi]), f"graph {j}"
    g.close()
    log(f"[batch] eager pass {ms_eager:.1f} ms; captured graph: plain {ms_graph_plain:.1f} ms, "
        f"tuned {ms_graph:.1f} ms; per-graph {ms_per_graph:.1f} ms")
    m = b.nnz // 2
    return {"graphs": b.count, "n": b.n, "m": m, "triangles": T,
            "per_graph_ms": ms_per_graph, "eager_pass_ms": ms_eager,
            "graph_plain_ms": ms_graph_plain, "graph_tuned_ms": ms_graph,
            "value": T / (ms_graph / 1000.0), "unit": "triangles/s",
            "per_graph_value": T / (ms_per_graph / 1000.0),
            "speedup_vs_per_graph": ms_per_graph / ms_graph,
            "tuned_vs_plain": ms_graph_plain / ms_graph,
            "schedule": {"heavy_min": sched.heavy_min, "light_rounds": sched.light_rounds,
                         "table": sched.table},
            "tune": {k: rep[k] for k in ("plain_ms", "tuned_ms", "tried", "seconds")},
            "tuning_batch": "128 graphs of the same recipe, seeds mix(1004, j)"}


class Workload:
    """One graph resident in HBM with every buffer the step needs."""

    def __init__(self, aot, name, seed, dev, args, dispatch=None, load=None):
        import torch

        t0 = time.time()
        self.aot, self.name, self.args, self.dispatch = aot, name, args, dispatch
        if load:
            self.csr = csr = load_csr(load, dev)
            log(f"[bench] loaded {csr.name} from {load}_*.npy: n={csr.n} m={csr.m} in "
                f"{time.time() - t0:.1f}s")
        else:
            self.csr = csr = inputs_mod().workload(name, seed, device=dev)
            torch.cuda.synchronize()
            log(f"[bench] generated {csr.name}: n={csr.n} m={csr.m} in {time.time() - t0:.1f}s")
        self.o = aot.alloc_oriented(csr.n, csr.m, dev)
        self.ows = torch.empty(aot.orient_workspace(csr.n, csr.nnz), dtype=torch.uint8,
                               device=dev)
        self.cws = torch.empty(aot.count_workspace(csr.n, csr.m), dtype=torch.uint8, device=dev)
        self.tri_off = torch.empty(csr.m + 1, dtype=torch.int64, device=dev)
        aot.orient(csr.rowptr, csr.col, out=self.o, ws=self.ows)
        c = aot.count(self.o, dispatch, ws=self.cws, tri_off=self.tri_off)
        self.T, self.probes = c.T, c.probes
        self.windowed = self.T * 12 > args.resident_gb * 1e9
        self.chunk = args.chunk
        if self.windowed:
            # free device memory plus what torch's allocator holds unused (the
            # generator's temporaries), so the windows do not depend on
            # whether the input was generated here or loaded
            free, _ = torch.cuda.mem_get_info(dev)
            free += torch.cuda.memory_reserved(dev) - torch.cuda.memory_allocated(dev)
            self.chunk = int(min(args.chunk, self.T, 0.6 * free // 12))
        self.out = None if self.windowed else torch.empty((max(self.T, 1), 3), dtype=torch.int32,
                                                          device=dev)
        # a list too large to hold is listed in windows: in-lists in rank
        # order make each window cost about its own triangles
        self.in_by_rank = self.windowed
        log(f"[bench] {name}: T={self.T} probes={self.probes}; output {self.T * 12 / 1e9:.2f} GB"
            + (f", listed in windows of {self.chunk} triangles" if self.windowed else ""))

    def list_all(self, cc, d):
        if self.windowed:
            self.aot.stream_list(self.o, cc, self.chunk, None, dispatch=d, to_host=False)
        else:
            self.aot.list_triangles(self.o, cc, out=self.out, dispatch=d)

    def step(self, d=None, ev=None):
        """orient + count + list of the whole graph (optional events between
        the passes)."""
        aot, csr = self.aot, self.csr
        d = self.dispatch if d is None else d
        if ev:
            ev[0].record()
        aot.orient(csr.rowptr, csr.col, out=self.o, ws=self.ows, in_by_rank=self.in_by_rank)
        if ev:
            ev[1].record()
        cc = aot.count(self.o, d, ws=self.cws, tri_off=self.tri_off)
        if ev:
            ev[2].record()
        self.list_all(cc, d)
        if ev:
            ev[3].record()
        return cc

    def timed(self, steps, warmup):
        """`steps` whole steps after `warmup` untimed ones, wall clock between
        device synchronisations, with per-pass event times; the timing
        recorder is off."""
        import torch

        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            cc = self.step(ev=evs[k])
            assert (cc.T, cc.probes) == (self.T, self.probes)
        torch.cuda.synchronize()
        ms_step = (time.perf_counter() - t0) * 1000.0 / steps
        per = [sum(e[i].elapsed_time(e[i + 1]) for e in evs) / steps for i in range(3)]
        log(f"[bench] {self.name}: step {ms_step:.3f} ms: orient {per[0]:.3f} count {per[1]:.3f} "
            f"list {per[2]:.3f}")
        return {"ms_per_step": ms_step, "value": self.T / (ms_step / 1000.0),
                "ms_orient": per[0], "ms_count": per[1], "ms_list": per[2],
                "probes_per_s": self.probes / (per[1] / 1000.0)}

    def records(self):
        """One more step with the per-launch recorder on: the per-bucket launch
        times the roofline is computed from."""
        self.aot.timing_start()
        cc = self.step()
        assert (cc.T, cc.probes) == (self.T, self.probes)
        return self.aot.timing_stop(cap=1 << 16)

    def config(self):
        csr = self.csr
        return {"workload": self.name, "graph": csr.name, "n": csr.n, "m": csr.m,
                "triangles": self.T, "probes": self.probes,
                "listing": f"windows of {self.chunk} triangles in device memory"
                           if self.windowed else "one device buffer"}


def inputs_mod():
    from paper_2006_11494_amd import inputs
    return inputs


def save_csr(csr, prefix):
    """The CSR as two .npy files (plain arrays, no pickled objects) and its
    name in a text file."""
    rp, col = csr.numpy()
    np.save(prefix + "_rowptr.npy", rp)
    np.save(prefix + "_col.npy", col)
    with open(prefix + "_name.txt", "w") as f:
        f.write(csr.name)


def load_csr(prefix, dev):
    import torch

    rp = np.load(prefix + "_rowptr.npy", mmap_mode="r")
    col = np.load(prefix + "_col.npy", mmap_mode="r")
    with open(prefix + "_name.txt") as f:
        name = f.read().strip()
    rowptr = torch.from_numpy(np.array(rp)).to(dev)
    c = torch.empty(col.shape[0], dtype=torch.int32, device=dev)
    step = 1 << 28
    for i in range(0, col.shape[0], step):          # bounded host copies
        c[i:i + step].copy_(torch.from_numpy(np.array(col[i:i + step])))
    return inputs_mod().Csr(rp.shape[0] - 1, rowptr, c, name)


def bucket_summary(recs):
    """Per-bucket totals of the recorded launches (both passes)."""
    out = {}
    for r in recs:
        k = f"{'write' if r['pass'] else 'count'}:{r['bucket']}"
        d = out.setdefault(k, {"launches": 0, "ms": 0.0, "edges": r["edges"],
                               "probes": r["probes"], "lookups": r.get("lookups", r["probes"]),
                               "staged": r["staged"], "triangles": r["triangles"]})
        d["launches"] += 1
        d["ms"] += r["ms"]
    return out


def extra_leg(aot, name, dev, args):
    """Another configuration: plain steps, and plain against learned."""
    import torch

    w = Workload(aot, name, None, dev, args)
    res = {"config": w.config(), **w.timed(max(3, args.steps // 2), 1)}
    if not args.no_learned:
        res["learned"] = learned_leg(aot, name, w.o, w.step, w.T, w.probes,
                                     max(3, args.learned_steps), log, scale=1, repeats=1)
    if name == "rmat20" and not args.no_ablation:
        res["ablation"] = ablation_leg(aot, w.csr, w.o, w.ows, w.cws, w.tri_off, w.out, w.T,
                                       args)
    del w
    torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    import torch

    from paper_2006_11494_amd import aot

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    dispatch = None
    if args.heavy_arm or args.heavy_min:
        table = None
        if args.heavy_arm:
            arm = ["bitmap", "hash", "global", "sorted"].index(args.heavy_arm)
            table = [t << 8 for t in (4, 4, 4, 8, 16, 32, 64, 64)] + [0] * 8 + [arm] * 16
        dispatch = aot.Dispatch(aot.AOT_DISPATCH_TABLE if table else aot.AOT_DISPATCH_PLAIN,
                                args.heavy_min, table)
    if args.save_csr:
        csr = inputs_mod().workload(args.workload, args.seed, device=dev)
        torch.cuda.synchronize()
        save_csr(csr, args.save_csr)
        log(f"[bench] saved {csr.name} to {args.save_csr}_*.npy")
        return
    w = Workload(aot, args.workload, args.seed, dev, args, dispatch, load=args.load_csr)
    T, probes = w.T, w.probes
    timed = w.timed(args.steps, args.warmup)
    recs = w.records()
    ms_step = timed["ms_per_step"]

    streamed = None
    if w.windowed and args.stream:
        state = {"windows": 0, "last": time.time()}

        def consume(first, view):
            state["windows"] += 1
            if time.time() - state["last"] > 20:
                log(f"[bench] streamed {first + len(view)} of {T} triangles to the host")
                state["last"] = time.time()

        aot.orient(w.csr.rowptr, w.csr.col, out=w.o, ws=w.ows, in_by_rank=True)
        torch.cuda.synchronize()
        t = time.perf_counter()
        cc = aot.count(w.o, dispatch, ws=w.cws, tri_off=w.tri_off)
        aot.stream_list(w.o, cc, args.stream_chunk, consume, dispatch=dispatch, to_host=True)
        torch.cuda.synchronize()
        s_ms = (time.perf_counter() - t) * 1000.0
        streamed = {"ms_count_and_list": s_ms, "windows": state["windows"],
                    "window_triangles": args.stream_chunk, "bytes_to_host": 12 * T,
                    "host_GB_per_s": 12 * T / (s_ms / 1000.0) / 1e9,
                    "triangles_per_s": T / (s_ms / 1000.0),
                    "note": "count + every window copied to pinned host memory (PCIe-inclusive)"}
        log(f"[bench] streamed to host: {s_ms:.1f} ms for {12 * T / 1e9:.1f} GB "
            f"({streamed['host_GB_per_s']:.1f} GB/s)")

    torch.cuda.empty_cache()        # return cached window buffers before the next legs
    ablation = None
    if not args.no_ablation and not w.windowed:
        ablation = ablation_leg(aot, w.csr, w.o, w.ows, w.cws, w.tri_off, w.out, T, args)
    learned = None
    if not args.no_learned and not args.heavy_arm:
        learned = learned_leg(aot, args.workload, w.o, w.step, T, probes, args.learned_steps, log)

    roof = roofline(recs, args.workload, w.windowed)
    log(f"[bench] dominant kernel {roof['kernel']}: {roof['achieved']:.1f} GB/s "
        f"({roof['frac'] * 100:.1f}% of peak) over {roof['launches']} launches")
    copy_gbs = copy_bandwidth()
    hbm_gbs = (roof["traffic"] / (roof["avg_launch_ms"] / 1000.0) / 1e9
               if roof["traffic"] else None)
    log(f"[bench] device copy: {copy_gbs:.1f} GB/s ({copy_gbs / HBM_PEAK_GBS * 100:.1f}% of peak); "
        f"dominant kernel at {roof['achieved'] / copy_gbs * 100:.1f}% of it")
    base = None
    if not args.no_cpu_baseline:
        # the large list is sampled on the host's share of cores (16 per GPU)
        # only; smaller ones on one thread and on all of them
        cores = min(16, os.cpu_count() or 1)
        if w.windowed:
            base = cpu_baseline(w.csr, args.cpu_sample or 0.01, cores)
        else:
            base = cpu_baseline(w.csr, args.cpu_sample or 0.5, 1)
            wide = cpu_baseline(w.csr, args.cpu_sample or 0.5, cores)
            base["all_cores"] = {k: wide[k] for k in ("value", "cores", "sample")}
        base["host"] = host_info()
    config = dict(w.config(), dispatch=args.heavy_arm or "plain",
                  heavy_min=args.heavy_min or 64)
    del w
    torch.cuda.empty_cache()

    extras = {}
    if args.workload == HEADLINE and not args.no_extras:
        for name in EXTRAS:
            extras[name] = extra_leg(aot, name, dev, args)
    batched = None
    if not args.no_batch and (args.workload != HEADLINE or not args.no_extras):
        batched = batched_leg(aot, args, dev)

    result = {
        "metric": "triangles/s (whole orient+count+list step); probes/s = sum of min(deg+) "
                  "per second of the count pass",
        "value": T / (ms_step / 1000.0),
        "unit": "triangles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": config,
        "probes_per_s": timed["probes_per_s"],
        "ms_orient": timed["ms_orient"],
        "ms_count": timed["ms_count"],
        "ms_list": timed["ms_list"],
        "roofline": {k: roof[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")},
        "roofline_kernel": dict({k: roof[k] for k in ("kernel", "launches", "avg_launch_ms",
                                                      "bytes_per_launch", "per_unit")},
                                copy_GBs=copy_gbs, frac_of_copy=roof["achieved"] / copy_gbs,
                                # rocprofv3's FETCH_SIZE + WRITE_SIZE bytes of one launch over
                                # this run's average launch time (null without a profile)
                                hbm_measured_GBs=hbm_gbs,
                                hbm_measured_frac=hbm_gbs / HBM_PEAK_GBS if hbm_gbs else None,
                                records="one extra step with the per-launch recorder on, "
                                        "outside the timed steps"),
        "buckets": bucket_summary(recs),
        "cpu_baseline": base,
        "learned": learned,
        "ablation": ablation,
        "batched": batched,
        "streamed": streamed,
        "extras": extras,
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
