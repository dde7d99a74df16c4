"""Autotuner of the persistent peel's grid size (the nd_schedule table).

The peel runs every round of a decomposition in one persistent launch whose
workgroups meet at grid barriers two or three times per round. The grid size
changes no result, only the cost: a barrier over fewer workgroups is cheaper,
and more workgroups give large rounds more lanes. Graphs (and batch unions)
with many small rounds prefer small grids; large graphs prefer the whole
device.

For each kind (a batch group's disjoint union, or a single graph), each
(r,s) and a few size classes, this times the candidate grids on the device
(median of `reps` runs, inputs resident in device memory, validation off)
and keeps the fastest. A class covers n_r up to the geometric midpoint
between its measured n_r and the next class's; the largest class of a kind
and pair covers everything above it. The table goes to schedules.json next
to this file, which nucleus.Context loads by default.

    python -m paper_2306_08623_amd.autotune [--out PATH] [--count 4096] [--reps 3]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

CANDIDATES = [64, 128, 256, 512, 768, 0]   # 0: the device's resident capacity
BATCH_PAIRS = [(2, 3), (3, 4)]
SINGLE = [((3, 4), [10, 12, 14, 16]), ((2, 3), [10, 12, 14, 16])]   # R-MAT scales
U64_MAX = (1 << 64) - 1


def _say(msg: str):
    print(f"[autotune] {msg}", file=sys.stderr, flush=True)


def _device_descs(graphs):
    import torch
    from . import nucleus
    keep, descs = [], (nucleus.GraphDesc * len(graphs))()
    for i, (g, r, s) in enumerate(graphs):
        rp = torch.from_numpy(g.row_ptr.astype(np.int64)).cuda()
        col = torch.from_numpy(g.col.astype(np.int32)).cuda() if g.col.size else \
            torch.zeros(1, dtype=torch.int32, device="cuda")
        keep.append((rp, col))
        descs[i] = nucleus.GraphDesc(g.n, r, s, g.nnz, rp.data_ptr(), col.data_ptr())
    torch.cuda.synchronize()
    return keep, descs


def _time_batch(descs, count, peel_blocks, reps):
    import torch
    from . import nucleus
    results = (nucleus.GraphResult * count)()
    with nucleus.Context(device=0, validate=False, peel_blocks=peel_blocks,
                         schedule="none") as ctx:
        ctx.nd_batch_decompose(descs, results, nucleus.ND_MEM_DEVICE)   # warm-up
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.nd_batch_decompose(descs, results, nucleus.ND_MEM_DEVICE)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
    n_r = sum(results[i].n_r for i in range(count))
    return float(np.median(times)), int(n_r)


def _time_single(g, r, s, peel_blocks, reps):
    import torch
    from . import nucleus
    with nucleus.Context(device=0, validate=False, peel_blocks=peel_blocks,
                         schedule="none") as ctx:
        ctx.load_csr(g)
        ctx.nd_set_rs(r, s)
        ctx._check(ctx.lib.nd_decompose(ctx.h))                             # warm-up
        ctx._check(ctx.lib.nd_sync(ctx.h))
        times = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx._check(ctx.lib.nd_decompose(ctx.h))
            ctx._check(ctx.lib.nd_sync(ctx.h))
            times.append(time.perf_counter() - t0)
        n_r = ctx.nd_get_info()["n_r"]
    return float(np.median(times)), int(n_r)


def _classes_to_entries(kind, r, s, classes):
    """classes: [(n_r, best_blocks)] ascending in n_r."""
    out = []
    for j, (nr, best) in enumerate(classes):
        hi = U64_MAX if j + 1 == len(classes) else int(np.sqrt(float(max(nr, 1)) *
                                                               float(max(classes[j + 1][0], 1))))
        out.append({"kind": kind, "r": r, "s": s, "n_r_max": hi, "peel_blocks": best})
    return out


def tune(count: int = 4096, reps: int = 3) -> dict:
    import torch
    from . import inputs as I
    from . import nucleus
    entries, log = [], []
    t0 = time.perf_counter()
    graphs = I.batch_graphs(count)
    _say(f"generated {count} batch graphs in {time.perf_counter() - t0:.1f} s")
    for r, s in BATCH_PAIRS:
        members = [x for x in graphs if (x[1], x[2]) == (r, s)]
        classes = []
        for frac in (16, 4, 1):
            sub = members[: max(1, len(members) // frac)]
            keep, descs = _device_descs(sub)
            best = None
            for nb in CANDIDATES:
                t, n_r = _time_batch(descs, len(sub), nb, reps)
                log.append({"kind": "batch", "r": r, "s": s, "graphs": len(sub), "n_r": n_r,
                            "peel_blocks": nb, "seconds": t})
                _say(f"batch ({r},{s}) {len(sub)} graphs n_r={n_r} peel_blocks={nb}: {t:.4f} s")
                if best is None or t < best[0]:
                    best = (t, nb, n_r)
            classes.append((best[2], best[1]))
            del keep
            torch.cuda.empty_cache()
        entries += _classes_to_entries(nucleus.ND_SCHED_BATCH, r, s, classes)
    for (r, s), scales in SINGLE:
        classes = []
        for sc in scales:
            g = I.rmat(sc, 16, 2)
            best = None
            for nb in CANDIDATES:
                t, n_r = _time_single(g, r, s, nb, reps)
                log.append({"kind": "single", "r": r, "s": s, "graph": f"rmat{sc}", "n_r": n_r,
                            "peel_blocks": nb, "seconds": t})
                _say(f"single ({r},{s}) rmat{sc} n_r={n_r} peel_blocks={nb}: {t:.4f} s")
                if best is None or t < best[0]:
                    best = (t, nb, n_r)
            classes.append((best[2], best[1]))
        # above the largest tuned size the default (the whole device) applies
        ent = _classes_to_entries(nucleus.ND_SCHED_SINGLE, r, s, classes)
        ent[-1]["n_r_max"] = classes[-1][0]
        entries += ent
    return {"device": torch.cuda.get_device_name(0), "candidates": CANDIDATES, "reps": reps,
            "batch_graphs": count, "entries": entries, "timings": log}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                  "schedules.json"))
    ap.add_argument("--count", type=int, default=4096)
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args()
    table = tune(a.count, a.reps)
    with open(a.out, "w") as f:
        json.dump(table, f, indent=1)
    _say(f"wrote {len(table['entries'])} entries to {a.out}")


if __name__ == "__main__":
    main()
