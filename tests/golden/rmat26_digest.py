"""Writes tests/golden/rmat26_digest.json: what the CPU oracle computes for the
R-MAT scale-26 workload (edge factor 32, seed 5), whose triangle list (about
2.3e11 triangles) is too large to store.  Calls only oracle/ (and the seeded
generator, which holds none of the method's arithmetic):

  * the input's size and SHA-256 of its rowptr and col arrays (so a GPU test
    knows it holds the same graph);
  * the probe count, the sum over directed edges of min(deg+(u), deg+(v));
  * T, F1 = sum and F2 = xor of the triple hashes over the whole list (CF,
    Algorithm 1, over rank ranges on host threads);
  * t[v], the triangles through every vertex: SHA-256 of the uint64 array
    (little-endian), its sum (3T) and the values at sampled vertices.

    python tests/golden/rmat26_digest.py [threads [workload]]

(another workload name writes <workload>_digest.json instead, for trying the
script on a small graph)

Takes about 20 GB of host memory beyond the graph and, on 8 cores, about an
hour."""

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2006_11494_amd import inputs  # noqa: E402

T0 = time.time()


def log(*a):
    print(f"[{time.time() - T0:7.1f}s]", *a, file=sys.stderr, flush=True)


def sha(a: np.ndarray) -> str:
    h = hashlib.sha256()
    flat = np.ascontiguousarray(a).view(np.uint8).reshape(-1)
    for i in range(0, flat.size, 1 << 28):
        h.update(flat[i:i + (1 << 28)])
    return h.hexdigest()


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 8)
    name = sys.argv[2] if len(sys.argv) > 2 else "rmat26"
    import torch
    torch.set_num_threads(threads)
    log(f"generating {name} on the CPU")
    csr = inputs.workload(name)
    rp, col = csr.numpy()
    graph = csr.name
    del csr
    log(f"n={rp.size - 1} nnz={col.size}")
    rec = {"workload": name, "graph": graph, "n": int(rp.size - 1),
           "nnz": int(col.size), "m": int(col.size // 2),
           "rowptr_sha256": sha(rp.astype("<i8")), "col_sha256": sha(col.astype("<i4"))}
    log("hashed the input; orienting")
    o = oracle.orient_threaded(rp, col, threads=threads, log=log)
    del col
    rec["probes"] = oracle.sum_min_threaded(o, threads=threads)
    log(f"probes {rec['probes']}; listing digest")
    t, (f1, f2), tv = oracle.list_digest_threaded(o, threads=threads, log=log)
    assert int(tv.sum(dtype=np.uint64)) == 3 * t
    rng = np.random.default_rng(2626)
    deg = np.diff(rp)
    top = np.argsort(deg)[-64:]
    vs = np.unique(np.concatenate([rng.integers(0, o.n, 4000), top])).astype(np.int64)
    rec.update({"T": int(t), "F1": int(f1), "F2": int(f2),
                "vertex_counts_sha256": sha(tv.astype("<u8")),
                "vertex_counts_sum": int(tv.sum(dtype=np.uint64)),
                "sample_vertices": vs.tolist(), "sample_counts": tv[vs].astype(np.int64).tolist(),
                "oracle": "CF (Algorithm 1) over rank ranges, orc_list_digest",
                "threads": threads, "seconds": round(time.time() - T0, 1)})
    with open(os.path.join(HERE, f"{name}_digest.json"), "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    log(f"T={t} F1={f1} F2={f2}; written")


if __name__ == "__main__":
    main()
