"""Write the oracle's per-graph results for the 4,096-graph mixed batch.

Calls only the CPU oracle (oracle/) on graphs from
paper_2306_08623_amd.inputs.batch_graphs; the GPU batch test recomputes the
same digests from the HIP path's per-graph outputs.
Run: python tests/golden/make_batch_golden.py [count] [workers]
"""
from __future__ import annotations

import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, HERE)

from make_golden import result_hashes  # noqa: E402

BASE_SEED = 4_000_000


def result_digest(rcliques, counts, coreness, parent, level) -> str:
    """12 hex digits over the five result arrays (layout of result_hashes)."""
    h = result_hashes(rcliques, counts, coreness, parent, level)
    joined = "".join(h[k] for k in ("rcliques", "counts", "coreness", "parent", "level"))
    return hashlib.sha256(joined.encode()).hexdigest()[:12]


def _one(i: int):
    import oracle
    from paper_2306_08623_amd import inputs as I
    g, r, s = I.batch_graph(i, BASE_SEED)
    t0 = time.time()
    d = oracle.decompose(g, r, s)
    dt = time.time() - t0
    dig = result_digest(d.rcliques, d.count, d.coreness, d.parent, d.level)
    return [d.n_r, d.n_s, d.k, d.n_int, g.sha256()[:12], dig], dt


def main(count: int, workers: int) -> None:
    import oracle
    oracle.build()
    t0 = time.time()
    with mp.get_context("spawn").Pool(workers) as pool:
        out = pool.map(_one, range(count), chunksize=4)
    rows = [o[0] for o in out]
    cpu = sum(o[1] for o in out)
    doc = {
        "source": "written by tests/golden/make_batch_golden.py from the CPU oracle",
        "workload": "inputs.batch_graph(i, 4000000) for i < count: n log-uniform in "
                    "[64, 65536], Erdos-Renyi (avg degree 8) or Chung-Lu (exponent 2.3, "
                    "mean degree 8) + 1..10 planted cliques of size 6..24, (2,3)/(3,4) mixed",
        "count": count, "base_seed": BASE_SEED,
        "columns": ["n_r", "n_s", "k", "n_int", "csr_sha256_12", "result_digest_12"],
        "oracle_cpu_seconds": round(cpu, 1),
        "graphs": rows,
    }
    path = os.path.join(HERE, f"batch{count}.json")
    with open(path, "w") as f:
        f.write(json.dumps(doc, separators=(",", ":")))
    print("wrote", path, f"(wall {time.time() - t0:.0f} s, oracle cpu {cpu:.0f} s)")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 4096,
         int(sys.argv[2]) if len(sys.argv) > 2 else 7)
