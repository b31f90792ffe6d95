"""The batched form on the GPU: many uneven graphs in one arena, one
persistent pass (eager or replayed from a captured HIP graph).  Every graph's
slice of the result must equal the CPU oracle's orientation and triangle list
of that graph alone, shifted by the graph's offsets; every schedule gives the
same bytes; windows past the capacity continue the list exactly."""

import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2006_11494_amd import aot, inputs, learn

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def complete(n):
    i, j = torch.triu_indices(n, n, 1)
    return inputs.csr_from_pairs(n, i, j, f"K{n}")


def empty(n):
    z = torch.zeros(0, dtype=torch.int64)
    return inputs.csr_from_pairs(n, z, z, f"empty{n}")


def mixed(seed, count=24, nmax=3000):
    """Small graphs of the batch's families, plus degenerate members."""
    out = []
    for j in range(count):
        s = inputs.mix_seed(seed, j)
        r = inputs.rand32(s, 9, torch.arange(3, dtype=torch.int64)).double() / 2**32
        n = int(20 + r[0].item() * (nmax - 20))
        fam = j % 3
        if fam == 0:
            out.append(inputs.erdos_renyi_m(n, 8 + 40 * r[1].item(), s))
        elif fam == 1:
            out.append(inputs.rmat(max(4, int(np.log2(n))), 8 + int(24 * r[1].item()), s))
        else:
            out.append(inputs.random_geometric(n, 20.0, s))
    out.insert(3, empty(1))
    out.insert(7, complete(12))
    out.insert(11, empty(0))
    out.insert(15, empty(40))
    return out


def make_batch(csrs):
    voff, rowptr, col = inputs.arena(csrs, device="cuda")
    return aot.Batch(voff, voff.cuda(), rowptr, col)


def check_against_oracle(b, r, csrs, which=None):
    voff = b.voff.numpy()
    gtri = r.graph_tri.cpu().numpy()
    orow = r.o.rowptr.cpu().numpy()
    ocol = r.o.col.cpu().numpy()
    perm = r.o.perm.cpu().numpy()
    tri = r.tri.cpu().numpy()
    for g in (which if which is not None else range(len(csrs))):
        c = csrs[g]
        rp, col = c.numpy()
        ref = oracle.orient(rp, col)
        v0, v1 = int(voff[g]), int(voff[g + 1])
        assert np.array_equal(perm[v0:v1] - v0, ref.perm), f"graph {g} perm"
        e0, e1 = int(orow[v0]), int(orow[v1])
        assert np.array_equal(orow[v0:v1 + 1] - e0, ref.orow), f"graph {g} rowptr"
        assert np.array_equal(ocol[e0:e1] - v0, ref.ocol), f"graph {g} col"
        t_ref = oracle.list_triangles(ref)
        assert gtri[g + 1] - gtri[g] == len(t_ref), f"graph {g} T"
        assert np.array_equal(tri[gtri[g]:gtri[g + 1]] - v0, t_ref), f"graph {g} list"


def test_batch_matches_oracle_per_graph():
    need_gpu()
    csrs = mixed(41)
    b = make_batch(csrs)
    say(f"[gpu] batch of {b.count}: n={b.n} nnz={b.nnz}")
    probe = aot.batch_run(b, cap=0)
    torch.cuda.synchronize()
    T = int(probe.graph_tri[-1].item())
    r = aot.batch_run(b, cap=T)
    torch.cuda.synchronize()
    check_against_oracle(b, r, csrs)
    assert torch.equal(r.tri_off, probe.tri_off)


def test_batch_schedules_give_the_same_bytes():
    need_gpu()
    csrs = mixed(42, count=18)
    b = make_batch(csrs)
    base = aot.batch_run(b, cap=0)
    torch.cuda.synchronize()
    T = int(base.graph_tri[-1].item())
    ref = aot.batch_run(b, cap=T)
    torch.cuda.synchronize()
    schedules = [aot.Schedule(table=learn.exploration_table(i)) for i in range(5)]
    schedules += [aot.Schedule(heavy_min=h) for h in (1, 4, 16, 128, 1 << 30)]
    schedules += [aot.Schedule(light_rounds=k) for k in (1, 3, 64)]
    schedules += [aot.Schedule(heavy_min=8, table=learn.exploration_table(3), light_rounds=2)]
    for sc in schedules:
        r = aot.batch_run(b, cap=T, schedule=sc)
        torch.cuda.synchronize()
        assert torch.equal(r.tri, ref.tri), sc
        assert torch.equal(r.tri_off, ref.tri_off), sc
        assert torch.equal(r.graph_tri, ref.graph_tri), sc
        assert torch.equal(r.o.col, ref.o.col) and torch.equal(r.o.perm, ref.o.perm)


def test_batch_matches_per_graph_launches():
    need_gpu()
    csrs = [c.to("cuda") for c in mixed(43, count=15)]
    b = make_batch(csrs)
    base = aot.batch_run(b, cap=0)
    torch.cuda.synchronize()
    T = int(base.graph_tri[-1].item())
    r = aot.batch_run(b, cap=T)
    torch.cuda.synchronize()
    gtri = r.graph_tri.cpu()
    for g, c in enumerate(csrs):
        o = aot.orient(c.rowptr, c.col)
        cnt = aot.count(o)
        t = aot.list_triangles(o, cnt)
        v0 = int(b.voff[g])
        assert cnt.T == int(gtri[g + 1] - gtri[g])
        assert torch.equal(r.tri[int(gtri[g]):int(gtri[g + 1])] - v0, t), f"graph {g}"
        e0 = int(r.o.rowptr[v0])
        assert torch.equal(r.tri_off[e0:e0 + o.m + 1] - r.tri_off[e0], cnt.tri_off)


def test_batch_windows_past_capacity():
    need_gpu()
    csrs = mixed(44, count=12)
    b = make_batch(csrs)
    base = aot.batch_run(b, cap=0)
    torch.cuda.synchronize()
    T = int(base.graph_tri[-1].item())
    full = aot.batch_run(b, cap=T)
    cap = T // 3
    part = aot.batch_run(b, cap=cap)
    torch.cuda.synchronize()
    assert torch.equal(part.tri[:cap], full.tri[:cap])
    c = part.counted()
    assert c.T == T
    for first, k in ((cap, T - cap), (T // 2, 1), (T - 5, 100)):
        w = aot.list_triangles(part.o, c, first=first, count=k)
        assert torch.equal(w, full.tri[first:first + k])


def test_batch_graph_replays_match_eager():
    """Captured once, replayed several times with the program's own eager
    work and synchronisations in between; every replay equals the eager
    pass."""
    need_gpu()
    csrs = mixed(45, count=20)
    b = make_batch(csrs)
    base = aot.batch_run(b, cap=0)
    torch.cuda.synchronize()
    T = int(base.graph_tri[-1].item())
    eager = aot.batch_run(b, cap=T)
    torch.cuda.synchronize()
    g = aot.BatchGraph(b, cap=T, schedule=aot.Schedule(light_rounds=2))
    try:
        for rep in range(4):
            g.run.tri.fill_(-1)
            g.run.tri_off.fill_(-1)
            g.run.graph_tri.fill_(-1)
            g.run.o.col.fill_(-1)
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            assert torch.equal(g.run.tri, eager.tri), f"replay {rep}"
            assert torch.equal(g.run.tri_off, eager.tri_off), f"replay {rep}"
            assert torch.equal(g.run.graph_tri, eager.graph_tri), f"replay {rep}"
            assert torch.equal(g.run.o.col, eager.o.col), f"replay {rep}"
            # eager work of the program between replays
            other = aot.batch_run(b, cap=T // 2)
            torch.cuda.synchronize()
            assert torch.equal(other.tri[:T // 2], eager.tri[:T // 2])
    finally:
        g.close()


def test_batch_rejects_bad_offsets():
    need_gpu()
    csrs = mixed(46, count=4)
    b = make_batch(csrs)
    bad = aot.Batch(b.voff.clone(), b.voff_dev, b.rowptr, b.col)
    bad.voff[-1] += 1
    with pytest.raises(aot.AotError) as e:
        aot.batch_workspace(bad)
    assert e.value.status == -1
    bad = aot.Batch(b.voff.clone(), b.voff_dev, b.rowptr, b.col)
    bad.voff[2] = bad.voff[1] - 1
    with pytest.raises(aot.AotError):
        aot.batch_workspace(bad)


@pytest.mark.timeout(900)
def test_full_batch_of_512_matches_oracle():
    """The measured batch itself: 512 graphs, n log-uniform in [1e3, 2e5],
    ER / R-MAT / RGG (seeds mixed from 4).  Its list (about 3e9 triangles) is
    digested on both sides over arena ids: the oracle runs CF on the arena as
    one graph (a disjoint union: the same triangles, Section 2.1), and the
    batch's digest, the triangles through every arena vertex and every
    graph's triangle count must equal it."""
    need_gpu()
    import time
    t0 = time.time()
    csrs = [inputs.batch_member(s, device="cuda") for s in inputs.batch_spec(512, 4)]
    b = make_batch(csrs)
    del csrs
    run = aot.batch_run(b, 0)
    torch.cuda.synchronize()
    gtri = run.graph_tri.cpu().numpy()
    c = run.counted()
    (t, s, x), vc = aot.digest(run.o, c)
    say(f"[gpu] batch512: n={b.n} m={b.nnz // 2} T={t} at {time.time() - t0:.1f}s")
    rp, col = b.rowptr.cpu().numpy(), b.col.cpu().numpy()
    ref = oracle.orient_threaded(rp, col, threads=16)
    del col
    rt, (rf1, rf2), rtv = oracle.list_digest_threaded(ref, threads=16)
    say(f"[gpu] batch512: oracle digest at {time.time() - t0:.1f}s")
    assert (t, s, x) == (rt, rf1, rf2) and t == int(gtri[-1])
    vcn = vc.cpu().numpy().astype(np.uint64)
    assert np.array_equal(vcn, rtv)
    voff = b.voff.numpy()
    cs = np.concatenate([[0], np.cumsum(rtv.astype(np.int64))])
    per = (cs[voff[1:]] - cs[voff[:-1]]) // 3
    assert np.array_equal(np.diff(gtri), per)
    say(f"[gpu] batch512: digest, {b.n} vertex counts and 512 graph counts equal the oracle's")
