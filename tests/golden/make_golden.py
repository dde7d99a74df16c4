"""Write the oracle's full-size results as hashes under tests/golden/.

Calls only the CPU oracle (oracle/) on the seeded workloads from
paper_2306_08623_amd.inputs; the GPU parity tests recompute the same hashes
from the HIP path's outputs. Run: python tests/golden/make_golden.py rmat18 2 3
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2306_08623_amd import inputs as I  # noqa: E402

WORKLOADS = {
    "rmat18": (I.workload_rmat18, "R-MAT scale 18, edge factor 16, (a,b,c,d)=(.57,.19,.19,.05), seed 2"),
    "er2k": (I.workload_er2k, "G(2000, 0.01) + 20 planted cliques of size 5..30, seed 1"),
    "chunglu4m": (I.workload_chung_lu_4m,
                  "Chung-Lu n=4,000,000, exponent 2.1, max expected degree 20,000, ~40M edges, "
                  "+ 1,000 communities of size 20..200 at density 0.6, seed 3"),
}


def digest(a: np.ndarray, dtype) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).tobytes()).hexdigest()


def result_hashes(rcliques, counts, coreness, parent, level) -> dict:
    """The hash layout shared by the golden files and the GPU tests."""
    return {
        "rcliques": digest(rcliques, np.uint32),
        "counts": digest(counts, np.uint32),
        "coreness": digest(coreness, np.uint32),
        "parent": digest(parent, np.uint64),
        "level": digest(level, np.uint32),
    }


def main(name: str, r: int, s: int) -> None:
    gen, desc = WORKLOADS[name]
    g = gen()
    print(f"{name}: n={g.n} m={g.m}, oracle ({r},{s}) started", flush=True)
    t0 = time.time()
    d = oracle.decompose(g, r, s)
    dt = time.time() - t0
    out = {
        "source": "written by tests/golden/make_golden.py from the CPU oracle",
        "workload": desc, "csr_sha256": g.sha256(), "n": g.n, "m": g.m, "r": r, "s": s,
        "n_r": d.n_r, "n_s": d.n_s, "k": d.k, "n_int": d.n_int,
        "oracle_seconds": round(dt, 1),
        "oracle_phase_seconds": {"count": round(d.t_count, 1), "peel": round(d.t_peel, 1),
                                 "tree": round(d.t_tree, 1)},
        "sha256": result_hashes(d.rcliques, d.count, d.coreness, d.parent, d.level),
    }
    path = os.path.join(HERE, f"{name}_{r}{s}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, f"({dt:.0f} s)")


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]), int(sys.argv[3]))
