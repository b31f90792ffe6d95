"""Seeded synthetic graph generators (input preparation only).

Every graph the tests, the smoke check and the benchmark feed to the library
comes from here, and the same arrays are handed to the CPU oracle, so both
sides always see identical input.  Nothing in this module orients, ranks,
intersects or counts: it only draws edges and builds the undirected simple
CSR the method starts from (the paper treats every input as an undirected
simple graph, Section 4, "Datasets").

Randomness is counter-based: a value is a pure function of (seed, stream,
index), computed with integer arithmetic that never leaves int64 range, so a
graph is bit-identical whether it is drawn on the CPU or on a GPU device with
torch, and independent of chunking.

Output format (``Csr``): ``rowptr`` int64[n+1], ``col`` int32[nnz]; every row
sorted ascending, no self-loops, no duplicates, symmetric (nnz = 2m).
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

_M16 = 0xFFFF
_M32 = 0xFFFFFFFF


@dataclass
class Csr:
    n: int
    rowptr: torch.Tensor  # int64 [n+1]
    col: torch.Tensor     # int32 [nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    @property
    def m(self) -> int:
        return self.nnz // 2

    def to(self, device) -> "Csr":
        return Csr(self.n, self.rowptr.to(device), self.col.to(device), self.name)

    def numpy(self):
        return self.rowptr.cpu().numpy(), self.col.cpu().numpy()


# ---------------------------------------------------------------------------
# counter-based 32-bit hashing in int64 lanes (no signed overflow anywhere)
# ---------------------------------------------------------------------------

def _mul32(a: torch.Tensor, c: int) -> torch.Tensor:
    """(a * c) mod 2^32 for 0 <= a, c < 2^32, via 16-bit halves (< 2^49)."""
    lo = (a & _M16) * c
    hi = ((a >> 16) * c) & _M16
    return (lo + (hi << 16)) & _M32


def _fmix32(h: torch.Tensor) -> torch.Tensor:
    """MurmurHash3's 32-bit finaliser (a bijection on 32-bit words)."""
    h = h ^ (h >> 16)
    h = _mul32(h, 0x85EBCA6B)
    h = h ^ (h >> 13)
    h = _mul32(h, 0xC2B2AE35)
    return h ^ (h >> 16)


def _key(seed: int, stream: int) -> int:
    t = torch.tensor([(seed * 0x9E3779B1 + 0x7F4A7C15) & _M32], dtype=torch.int64)
    t = _fmix32(t ^ ((stream * 0x85EBCA77 + 0x27D4EB2F) & _M32))
    return int(_fmix32(t)[0])


def rand32(seed: int, stream: int, idx: torch.Tensor) -> torch.Tensor:
    """Uniform 32-bit words (held in int64) for counters ``idx`` (int64, >= 0)."""
    k = _key(seed, stream)
    h = _fmix32((idx & _M32) ^ k)
    h = _fmix32(h ^ ((idx >> 32) & _M32) ^ 0x165667B1)
    return h


def mix_seed(*parts: int) -> int:
    h = 0x12345678
    for p in parts:
        h = _key(h, p)
    return h


# ---------------------------------------------------------------------------
# edge list -> undirected simple CSR
# ---------------------------------------------------------------------------

def csr_from_pairs(n: int, u: torch.Tensor, v: torch.Tensor, name: str = "") -> Csr:
    """Symmetrise, drop self-loops and duplicates, and build a sorted CSR."""
    u = u.to(torch.int64)
    v = v.to(torch.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    a = torch.minimum(u, v)
    b = torch.maximum(u, v)
    key = torch.unique(a * n + b)            # sorted, deduplicated undirected pairs
    a = key // n
    b = key - a * n
    rows = torch.cat([a, b])
    cols = torch.cat([b, a])
    order = torch.sort(rows * n + cols, stable=True).values
    rows = order // n
    cols = order - rows * n
    counts = torch.bincount(rows, minlength=n)
    rowptr = torch.zeros(n + 1, dtype=torch.int64, device=u.device)
    rowptr[1:] = torch.cumsum(counts, 0)
    return Csr(n, rowptr, cols.to(torch.int32), name)


def csr_from_pairs_partitioned(n: int, u, v, name: str = "", parts: int = 32,
                               consume: bool = False) -> Csr:
    """The same CSR as csr_from_pairs, built one range of rows at a time so
    that no sort ever holds more than about 2 * pairs / parts keys (graphs
    with billions of entries).  u, v: tensors (int32 or int64), or equally
    chunked lists of them, so that no single operation sees all pairs.  With
    consume=True and lists, the lists are emptied once every range is built,
    so the pairs are freed before the rows are joined."""
    us = list(u) if isinstance(u, (list, tuple)) else [u]
    vs = list(v) if isinstance(v, (list, tuple)) else [v]
    dev = us[0].device if us else torch.device("cpu")
    counts = torch.zeros(n, dtype=torch.int64, device=dev)
    cols = []
    bounds = [n * p // parts for p in range(parts + 1)]
    for p in range(parts):
        lo, hi = bounds[p], bounds[p + 1]
        if hi <= lo:
            continue
        keys = []
        for cu, cv in zip(us, vs):
            for x, y in ((cu, cv), (cv, cu)):
                sel = (x >= lo) & (x < hi) & (x != y)
                keys.append((x[sel].to(torch.int64) - lo) * n + y[sel].to(torch.int64))
                del sel
        key = torch.unique(torch.cat(keys)) if keys else torch.zeros(0, dtype=torch.int64,
                                                                     device=dev)
        del keys
        rows = key // n                                  # sorted, deduplicated (row, col)
        counts[lo:hi] = torch.bincount(rows, minlength=hi - lo)
        cols.append((key - rows * n).to(torch.int32))
        del key, rows
    if consume:
        for lst in (u, v):
            if isinstance(lst, list):
                lst.clear()
        us.clear()
        vs.clear()
    rowptr = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    rowptr[1:] = torch.cumsum(counts, 0)
    col = torch.cat(cols) if cols else torch.zeros(0, dtype=torch.int32, device=dev)
    return Csr(n, rowptr, col, name)


def csr_from_edges_np(n: int, edges) -> Csr:
    """Small hand-written graphs: ``edges`` is an iterable of (u, v) pairs."""
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    return csr_from_pairs(n, torch.from_numpy(e[:, 0].copy()), torch.from_numpy(e[:, 1].copy()))


def _random_permutation(seed: int, n: int, device) -> torch.Tensor:
    keys = rand32(seed, 0x5EED, torch.arange(n, dtype=torch.int64, device=device))
    return torch.sort(keys * n + torch.arange(n, dtype=torch.int64, device=device)).indices


# ---------------------------------------------------------------------------
# families
# ---------------------------------------------------------------------------

def erdos_renyi(n: int, p: float, seed: int, device="cpu") -> Csr:
    """G(n, p): an independent Bernoulli(p) draw for every pair i < j."""
    thr = int(round(p * 2**32))
    i = torch.arange(n, dtype=torch.int64, device=device)
    us, vs = [], []
    rows_per_chunk = max(1, (1 << 24) // max(n, 1))
    for r0 in range(0, n, rows_per_chunk):
        r1 = min(n, r0 + rows_per_chunk)
        ii = i[r0:r1, None].expand(r1 - r0, n)
        jj = i[None, :].expand(r1 - r0, n)
        upper = jj > ii
        h = rand32(seed, 1, ii * n + jj)
        sel = upper & (h < thr)
        us.append(ii[sel])
        vs.append(jj[sel])
    return csr_from_pairs(n, torch.cat(us), torch.cat(vs), f"er(n={n},p={p},seed={seed})")


def erdos_renyi_m(n: int, mean_degree: float, seed: int, device="cpu") -> Csr:
    """ER with about n*d/2 uniformly drawn pairs (duplicates and loops dropped)."""
    m = int(round(n * mean_degree / 2))
    idx = torch.arange(m, dtype=torch.int64, device=device)
    u = rand32(seed, 2, idx) % n
    v = rand32(seed, 3, idx) % n
    return csr_from_pairs(n, u, v, f"er_m(n={n},d={mean_degree},seed={seed})")


def rmat(scale: int, edge_factor: int, seed: int, a=0.57, b=0.19, c=0.19,
         device="cpu", chunk: int = 1 << 24, parts: int | None = None) -> Csr:
    """R-MAT: edge_factor * 2^scale tuples, one quadrant draw per bit level
    (16-bit resolution, no per-level noise), then a seeded vertex relabelling.
    From 2^27 tuples on (or when parts is given) the CSR is built by row
    ranges (csr_from_pairs_partitioned): the same graph, less memory."""
    n = 1 << scale
    ntup = edge_factor * n
    ta = int(round(a * 65536))
    tab = int(round((a + b) * 65536))
    tabc = int(round((a + b + c) * 65536))
    perm = _random_permutation(seed, n, device)
    us, vs = [], []
    for t0 in range(0, ntup, chunk):
        t = torch.arange(t0, min(ntup, t0 + chunk), dtype=torch.int64, device=device)
        u = torch.zeros_like(t)
        v = torch.zeros_like(t)
        for lvl in range(scale):
            if lvl % 2 == 0:
                word = rand32(seed, 16 + lvl // 2, t)
                x = word & _M16
            else:
                x = word >> 16
            ubit = (x >= tab).to(torch.int64)
            vbit = ((x >= ta) & (x < tab) | (x >= tabc)).to(torch.int64)
            u = u | (ubit << lvl)
            v = v | (vbit << lvl)
        us.append(perm[u].to(torch.int32))
        vs.append(perm[v].to(torch.int32))
        del t, u, v
    name = f"rmat(scale={scale},ef={edge_factor},seed={seed})"
    if parts is None and ntup < (1 << 27):
        return csr_from_pairs(n, torch.cat(us), torch.cat(vs), name)
    return csr_from_pairs_partitioned(n, us, vs, name, parts or max(8, ntup >> 26),
                                      consume=True)


def chung_lu(n: int, mean_degree: float, gamma: float, max_degree: float, seed: int,
             device="cpu", chunk: int = 1 << 24) -> Csr:
    """Chung-Lu power law: expected degrees w_i = min(cap, c (i+1)^(-1/(gamma-1))),
    c set by bisection so that mean(w) = mean_degree; sum(w)/2 endpoint pairs are
    drawn with probability proportional to w (loops and duplicates dropped)."""
    i = np.arange(n, dtype=np.float64)
    base = (i + 1.0) ** (-1.0 / (gamma - 1.0))
    lo, hi = 0.0, 60.0                      # bisection on log(c)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if np.minimum(max_degree, math.exp(mid) * base).mean() < mean_degree:
            lo = mid
        else:
            hi = mid
    w = np.minimum(max_degree, math.exp(hi) * base)
    scale = float(2**46) / w.sum()
    wi = np.floor(w * scale).astype(np.int64)
    cdf = torch.from_numpy(np.cumsum(wi)).to(device)
    total = int(cdf[-1])
    npairs = int(round(w.sum() / 2))
    perm = _random_permutation(seed, n, device)
    us, vs = [], []
    for t0 in range(0, npairs, chunk):
        t = torch.arange(t0, min(npairs, t0 + chunk), dtype=torch.int64, device=device)
        ends = []
        for s in (0, 1):
            r = (rand32(seed, 40 + 2 * s, t) << 14) ^ (rand32(seed, 41 + 2 * s, t) & 0x3FFF)
            r = torch.clamp(r, max=total - 1)
            ends.append(torch.searchsorted(cdf, r, right=True))
        us.append(perm[ends[0]])
        vs.append(perm[ends[1]])
    return csr_from_pairs(n, torch.cat(us), torch.cat(vs),
                          f"chung_lu(n={n},d={mean_degree},g={gamma},seed={seed})")


def random_geometric(n: int, mean_degree: float, seed: int, device="cpu") -> Csr:
    """2-D random geometric graph: n uniform points in the unit square, an edge
    when the distance is below r = sqrt(d / (pi n)) (no wrap-around)."""
    r = math.sqrt(mean_degree / (math.pi * n))
    idx = torch.arange(n, dtype=torch.int64, device=device)
    x = rand32(seed, 60, idx).to(torch.float64) / 2**32
    y = rand32(seed, 61, idx).to(torch.float64) / 2**32
    g = max(1, int(1.0 / r))
    cx = torch.clamp((x * g).to(torch.int64), max=g - 1)
    cy = torch.clamp((y * g).to(torch.int64), max=g - 1)
    cell = cx * g + cy
    order = torch.sort(cell * n + idx).indices
    cell_sorted = cell[order]
    counts = torch.bincount(cell_sorted, minlength=g * g)
    start = torch.zeros(g * g + 1, dtype=torch.int64, device=device)
    start[1:] = torch.cumsum(counts, 0)
    us, vs = [], []
    r2 = r * r
    for dx, dy in ((0, 0), (1, -1), (1, 0), (1, 1), (0, 1)):
        nx, ny = cx + dx, cy + dy
        ok = (nx >= 0) & (nx < g) & (ny >= 0) & (ny < g)
        src = idx[ok]
        ncell = nx[ok] * g + ny[ok]
        cnt = counts[ncell]
        src_rep = torch.repeat_interleave(src, cnt)
        first = torch.repeat_interleave(start[ncell], cnt)
        off = torch.arange(int(cnt.sum()), dtype=torch.int64, device=device)
        off = off - torch.repeat_interleave(torch.cumsum(cnt, 0) - cnt, cnt)
        dst = order[first + off]
        d2 = (x[src_rep] - x[dst]) ** 2 + (y[src_rep] - y[dst]) ** 2
        keep = (d2 < r2) & (src_rep != dst)
        if dx == 0 and dy == 0:
            keep &= src_rep < dst
        us.append(src_rep[keep])
        vs.append(dst[keep])
    return csr_from_pairs(n, torch.cat(us), torch.cat(vs),
                          f"rgg(n={n},d={mean_degree},seed={seed})")


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------

def workload(name: str, seed: int | None = None, device="cpu") -> Csr:
    """The synthetic stand-ins for the paper's real graphs (Table 2):
    er2000 (ER n=2000 p=0.01), rmat20 (scale 20, edge factor 16),
    chunglu4m (n=4M, mean degree 40, exponent 2.1, cap 100k),
    rmat26 (scale 26, edge factor 32); rmatS / rmatSxE: R-MAT of scale S and
    edge factor 16 / E (smaller variants and proxies)."""
    if name == "er2000":
        return erdos_renyi(2000, 0.01, 1 if seed is None else seed, device)
    if name == "rmat20":
        return rmat(20, 16, 2 if seed is None else seed, device=device)
    if name == "chunglu4m":
        return chung_lu(4_000_000, 40.0, 2.1, 100_000.0, 3 if seed is None else seed, device)
    if name == "rmat26":
        return rmat(26, 32, 5 if seed is None else seed, device=device)
    if name.startswith("rmat"):           # rmatS (edge factor 16) or rmatSxE
        spec = name[4:].split("x")
        scale, ef = int(spec[0]), int(spec[1]) if len(spec) > 1 else 16
        return rmat(scale, ef, 2 if seed is None else seed, device=device)
    raise ValueError(f"unknown workload {name!r}")


def batch_spec(count: int = 512, seed: int = 4):
    """Per-member recipe of the uneven batch: n log-uniform in [1e3, 2e5]; family
    uniform over ER (mean degree U[8, 64]), R-MAT (edge factor U{8..32},
    scale = round(log2 n)) and 2-D RGG (mean degree 20)."""
    out = []
    for j in range(count):
        s = mix_seed(seed, j)
        t = torch.arange(4, dtype=torch.int64)
        r = rand32(s, 7, t).double() / 2**32
        n = int(round(math.exp(math.log(1000) + r[0].item() * (math.log(200000) - math.log(1000)))))
        fam = min(2, int(r[1].item() * 3))
        if fam == 0:
            out.append(("er", n, 8.0 + 56.0 * r[2].item(), s))
        elif fam == 1:
            out.append(("rmat", int(round(math.log2(n))), 8 + min(24, int(r[3].item() * 25)), s))
        else:
            out.append(("rgg", n, 20.0, s))
    return out


def batch_member(spec, device="cpu") -> Csr:
    fam, a, b, s = spec
    if fam == "er":
        return erdos_renyi_m(a, b, s, device)
    if fam == "rmat":
        return rmat(a, b, s, device=device)
    return random_geometric(a, b, s, device)


def arena(csrs, device=None):
    """The block-diagonal union of several CSRs (a batch's arena): graph g's
    vertices become [voff[g], voff[g+1]).  Returns (voff int64 [count+1] on
    the host, rowptr, col) with rowptr/col on `device` (default: the first
    graph's)."""
    device = device if device is not None else (csrs[0].rowptr.device if csrs else "cpu")
    ns = [c.n for c in csrs]
    nnzs = [c.nnz for c in csrs]
    voff = torch.zeros(len(csrs) + 1, dtype=torch.int64)
    voff[1:] = torch.cumsum(torch.tensor(ns, dtype=torch.int64), 0)
    eoff = [0]
    for z in nnzs:
        eoff.append(eoff[-1] + z)
    rows = [c.rowptr[:-1].to(device) + eoff[g] for g, c in enumerate(csrs)]
    rows.append(torch.tensor([eoff[-1]], dtype=torch.int64, device=device))
    cols = [c.col.to(device) + int(voff[g]) for g, c in enumerate(csrs)]
    rowptr = torch.cat(rows)
    col = torch.cat(cols).to(torch.int32) if cols else torch.zeros(0, dtype=torch.int32, device=device)
    return voff, rowptr, col
