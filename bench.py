#!/usr/bin/env python3
"""Benchmark: exact (3,4) nucleus decomposition + hierarchy on one MI355X.

Workload (the largest (3,4) configuration): a Chung-Lu power-law graph with
n = 4,000,000, degree exponent 2.1, ~40M sampled edges, maximum expected
degree 20,000, plus 1,000 disjoint communities of 20-200 vertices at edge
density 0.6, seed 3; (r,s) = (3,4). A step is one full decomposition from
the CSR already resident in HBM: orientation, triangle tables, 4-clique
counting, the peel rounds with hierarchy linking, and the canonical tree.
R-MAT scale 18 (edge factor 16, (a,b,c,d) = (.57,.19,.19,.05), seed 2) is
measured the same way as a secondary object of the line.

Metric: s-cliques traversed per second, where a decomposition traverses
n_s + C(s,r) * n_s s-cliques (each s-clique once while counting, and once per
member r-clique while peeling). The same numerator is used for the CPU
oracle baseline, which runs on a smaller graph of the same generator.

The same line carries a "batch" object: the 4,096-graph mixed batch
(n log-uniform in [64, 65536], Erdos-Renyi or Chung-Lu with planted cliques,
(2,3)/(3,4) mixed), decomposed with inputs already in HBM once as one
nd_batch_decompose call and once graph by graph (nd_load_csr from device
memory + nd_decompose), in graphs per second.

Prints one JSON line (see the keys below).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from math import comb

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic bytes of the dominant kernels: peel+link kernel, bytes per
# (r-clique, s-clique) visit and per peeled r-clique; counting kernel, bytes
# per listed s-clique. A visit resolves the ids of the s-clique's other
# r-cliques (4 B per edge id from a CSR slot, 8 B per triangle id: list
# entry + its triangle) and touches each one's state (a 4 B peel state and
# an 8 B count read-modify-write): (3,4) 3 x (8 + 12) = 60 B, (2,3)
# 2 x (4 + 12) = 32 B, (2,4) 5 x (4 + 12) = 80 B, (1,2) 16 B, (1,3) 2 x 16,
# (1,4) 3 x 16 (a vertex id instead of an r-clique id). A peeled r-clique
# adds its frontier slot (write + read), core number and peel round, and its
# probe range offsets. A counted 4-clique costs four triangle-id lookups and
# four count updates (8 B each).
PEEL_BYTES_PER_VISIT = {(1, 2): 16, (2, 3): 32, (3, 4): 60, (2, 4): 80, (1, 3): 32, (1, 4): 48}
PEEL_BYTES_PER_RCLIQUE = {(1, 2): 20, (2, 3): 24, (3, 4): 28, (2, 4): 28, (1, 3): 20, (1, 4): 20}
COUNT_BYTES_PER_SCLIQUE = {(1, 2): 0, (2, 3): 36, (3, 4): 64, (2, 4): 72, (1, 3): 36, (1, 4): 48}


def byte_model(r: int, s: int) -> tuple[int, int, int]:
    """(peel bytes per visit, per peeled r-clique, count bytes per s-clique).
    s = 5..7 keep their s-cliques: a visit reads its incidence entry (4 B)
    and the s-clique's C(s,r) r-clique ids (4 B each), then touches the
    C(s,r) - 1 others' state (12 B each); a peeled r-clique also reads its
    two incidence offsets (8 B more); counting writes the ids and the
    incidence entry of every (r-clique, s-clique) pair and increments its
    count (16 B per pair)."""
    if (r, s) in PEEL_BYTES_PER_VISIT:
        return PEEL_BYTES_PER_VISIT[(r, s)], PEEL_BYTES_PER_RCLIQUE[(r, s)], \
            COUNT_BYTES_PER_SCLIQUE[(r, s)]
    c = comb(s, r)
    return 4 + 4 * c + 12 * (c - 1), 36, 16 * c

DESCS = {
    "chunglu4m": "Chung-Lu n=4,000,000, exponent 2.1, ~40M edges, max expected degree 20,000, "
                 "+ 1,000 communities of size 20..200 at density 0.6, seed 3",
    "rmat18": "R-MAT scale 18, edge factor 16, (a,b,c,d)=(.57,.19,.19,.05), seed 2",
    "er2k": "G(2000, 0.01) + 20 planted cliques of size 5..30, seed 1",
}


def profile_path(kernel: str, workload_name: str, r: int, s: int) -> str:
    return os.path.join(ROOT, "profiles", f"{kernel}_{workload_name}_{r}{s}.txt")


def measured_traffic(kernel: str, workload_name: str, r: int, s: int):
    """HBM bytes per launch from the committed rocprofv3 --pmc summary of
    this kernel on this workload (FETCH_SIZE + WRITE_SIZE, scaled by the
    copy-kernel calibration), or None if it was not profiled or the kernel's
    source changed since the counters were taken."""
    import hashlib
    path = profile_path("k_peel", workload_name, r, s)
    if not os.path.exists(path):
        return None
    text = open(path).read()
    src = os.path.join(ROOT, "paper_2306_08623_amd", "csrc")
    files = {"k_peel": ("nd_peel_kern.h", "nd_internal.h"),
             "k_count_s4": ("nd_count.hip", "nd_internal.h")}.get(kernel)
    if files is None:
        return None
    h = hashlib.sha256(b"".join(open(os.path.join(src, f), "rb").read()
                                for f in files)).hexdigest()
    key = f"traffic_bytes_per_launch {kernel}<{r},{s}> {workload_name} source {h}:"
    for line in text.splitlines():
        if line.startswith(key):
            return int(line.split(":")[1])
    return None


def workload(name: str):
    from paper_2306_08623_amd import inputs as I
    if name == "chunglu4m":
        return I.workload_chung_lu_4m(), DESCS[name]
    if name == "rmat18":
        return I.workload_rmat18(), DESCS[name]
    if name == "er2k":
        return I.workload_er2k(), DESCS[name]
    if name.startswith("rmat"):
        sc = int(name[4:])
        return I.rmat(sc, 16, 2), f"R-MAT scale {sc}, edge factor 16, seed 2"
    raise SystemExit(f"unknown workload {name}")


def cpu_sample(name: str, scale: int):
    """A smaller graph of the benched workload's generator, for the oracle."""
    from paper_2306_08623_amd import inputs as I
    if name == "chunglu4m":
        # same exponent, mean degree and community recipe; n, the maximum
        # expected degree and the number of communities shrink by 2^scale
        n = 4_000_000 >> scale
        wmax = 20_000.0 / (1 << scale)
        comms = max(1, 1000 >> scale)
        g = I.chung_lu(n, 2.1, 20.0, wmax, 3, target_edges=10 * n, n_communities=comms,
                       comm_lo=20, comm_hi=200, comm_density=0.6)
        return g, (f"Chung-Lu n={n}, exponent 2.1, mean degree 20, max expected degree {wmax:.0f}, "
                   f"+ {comms} communities of size 20..200 at density 0.6, seed 3 (the "
                   f"benched generator with n, max degree and communities / {1 << scale})")
    sc = scale if not name.startswith("rmat") else int(name[4:]) - scale
    return I.rmat(sc, 16, 2), f"R-MAT scale {sc}, edge factor 16, seed 2 (same generator)"


def golden_oracle_runs(name: str) -> list:
    """Full-size oracle runs of this workload recorded by the golden files
    (tests/golden/make_golden.py, one host core): same-workload context."""
    import glob
    out = []
    for path in sorted(glob.glob(os.path.join(ROOT, "tests", "golden", f"{name}_*.json"))):
        try:
            d = json.load(open(path))
            trav = d["n_s"] + comb(d["s"], d["r"]) * d["n_s"]
            out.append({"r": d["r"], "s": d["s"], "oracle_seconds": d["oracle_seconds"],
                        "traversals_per_s": trav / d["oracle_seconds"], "cores": 1,
                        "file": os.path.relpath(path, ROOT)})
        except (KeyError, ValueError, OSError, ZeroDivisionError):
            continue
    return out


def cpu_baseline(name: str, r: int, s: int, scale: int) -> dict:
    """The oracle, single-threaded, on a smaller graph of the same generator
    (a bounded sample of the workload): traversals per second."""
    import oracle
    g, what = cpu_sample(name, scale)
    t0 = time.perf_counter()
    d = oracle.decompose(g, r, s)
    dt = time.perf_counter() - t0
    trav = d.n_s + comb(s, r) * d.n_s
    return {
        "value": trav / dt,
        "unit": "s-cliques traversed/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"full ({r},{s}) decomposition of {what}: n={g.n}, m={g.m}, "
                   f"n_r={d.n_r}, n_s={d.n_s}, {dt:.1f} s on one host core"),
        "seconds": dt,
        "full_size_runs": golden_oracle_runs(name),
    }


def _oracle_batch_item(i: int) -> int:
    import oracle
    from paper_2306_08623_amd import inputs as I
    g, r, s = I.batch_graph(i)
    return oracle.decompose(g, r, s).n_s


def cpu_batch_baseline(sample: int) -> dict:
    """The oracle over the first `sample` graphs of the mixed batch, one
    process per host core (graphs are independent), in graphs/s."""
    import multiprocessing as mp
    workers = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(workers) as pool:
        pool.map(_oracle_batch_item, range(sample), chunksize=4)
    dt = time.perf_counter() - t0
    return {"value": sample / dt, "unit": "graphs/s", "cores": workers, "kind": "oracle",
            "sample": f"full decompositions of batch graphs 0..{sample - 1}, {workers} processes, "
                      f"{dt:.1f} s including process start and graph generation"}


def bench_batch(count: int, reps: int) -> dict:
    """Batched vs one-by-one decomposition of the mixed batch, inputs
    resident in HBM, validation off in both (the inputs are validated once,
    untimed, by a first batched call with validation on)."""
    import numpy as np
    import torch

    from paper_2306_08623_amd import inputs as I
    from paper_2306_08623_amd import nucleus

    t0 = time.perf_counter()
    graphs = I.batch_graphs(count)
    print(f"[bench] batch: generated {count} graphs in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    dev = []
    descs = (nucleus.GraphDesc * count)()
    for i, (g, r, s) in enumerate(graphs):
        rp = torch.from_numpy(g.row_ptr.astype(np.int64)).cuda()
        col = torch.from_numpy(g.col.astype(np.int32)).cuda() if g.col.size else \
            torch.zeros(1, dtype=torch.int32, device="cuda")
        dev.append((g.n, rp, col, r, s, g.nnz))
        descs[i] = nucleus.GraphDesc(g.n, r, s, g.nnz, rp.data_ptr(), col.data_ptr())
    torch.cuda.synchronize()
    results = (nucleus.GraphResult * count)()
    with nucleus.Context(device=0, validate=True) as vctx:
        vctx.nd_batch_decompose(descs, results, nucleus.ND_MEM_DEVICE)
        total_ns = sum(results[i].n_s for i in range(count))
        total_nr = sum(results[i].n_r for i in range(count))
    ctx = nucleus.Context(device=0, validate=False)
    ctx.nd_batch_decompose(descs, results, nucleus.ND_MEM_DEVICE)      # warm-up
    torch.cuda.synchronize()
    tb = time.perf_counter()
    for rep in range(reps):
        ctx.nd_batch_decompose(descs, results, nucleus.ND_MEM_DEVICE)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - tb) / reps
    binfo = ctx.nd_get_info()
    print(f"[bench] batch: batched {t_batch:.3f} s per batch (tuned schedules: "
          f"{len(nucleus.load_schedules())} entries)", file=sys.stderr, flush=True)
    # the same batch with the default grid (no schedule table)
    with nucleus.Context(device=0, validate=False, schedule="none") as uctx:
        uctx.nd_batch_decompose(descs, results, nucleus.ND_MEM_DEVICE)   # warm-up
        torch.cuda.synchronize()
        tu = time.perf_counter()
        for rep in range(reps):
            uctx.nd_batch_decompose(descs, results, nucleus.ND_MEM_DEVICE)
        torch.cuda.synchronize()
        t_untuned = (time.perf_counter() - tu) / reps
    print(f"[bench] batch: untuned {t_untuned:.3f} s per batch", file=sys.stderr, flush=True)
    lib = ctx.lib
    # one by one: same context kind, same device-resident inputs
    for (n, rp, col, r, s, nnz) in dev[:8]:                             # warm-up
        ctx._check(lib.nd_load_csr(ctx.h, n, nnz, rp.data_ptr(), col.data_ptr(),
                                   nucleus.ND_MEM_DEVICE))
        ctx._check(lib.nd_set_rs(ctx.h, r, s))
        ctx._check(lib.nd_decompose(ctx.h))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for j, (n, rp, col, r, s, nnz) in enumerate(dev):
        ctx._check(lib.nd_load_csr(ctx.h, n, nnz, rp.data_ptr(), col.data_ptr(),
                                   nucleus.ND_MEM_DEVICE))
        ctx._check(lib.nd_set_rs(ctx.h, r, s))
        ctx._check(lib.nd_decompose(ctx.h))
        if j % 1024 == 1023:
            print(f"[bench] batch: one-by-one {j + 1} graphs, "
                  f"{time.perf_counter() - t1:.1f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_one = time.perf_counter() - t1
    ctx.close()
    cpu = cpu_batch_baseline(min(count, 512))
    print(f"[bench] batch: oracle {cpu['value']:.1f} graphs/s on {cpu['cores']} processes",
          file=sys.stderr, flush=True)
    return {
        "graphs": count,
        "cpu_oracle": cpu,
        "workload": "inputs.batch_graph(i, 4000000), i < %d: n log-uniform in [64, 65536], "
                    "Erdos-Renyi (avg degree 8) or Chung-Lu (exponent 2.3) + 1..10 planted "
                    "cliques of size 6..24, (2,3)/(3,4) alternating in pairs" % count,
        "total_n": int(sum(g.n for g, _, _ in graphs)),
        "total_m": int(sum(g.m for g, _, _ in graphs)),
        "total_n_r": int(total_nr), "total_n_s": int(total_ns),
        "batched_graphs_per_s": count / t_batch,
        "batched_untuned_graphs_per_s": count / t_untuned,
        "schedule_entries": len(nucleus.load_schedules()),
        "one_by_one_graphs_per_s": count / t_one,
        "speedup": t_one / t_batch,
        "batched_s": t_batch, "one_by_one_s": t_one, "reps": reps,
        "batched_phases_ms": {"prep": round(binfo["ms_prep"], 2),
                              "count": round(binfo["ms_count"], 2),
                              "peel": round(binfo["ms_peel"], 2),
                              "tree": round(binfo["ms_tree"], 2)},
    }


def bench_serve(pool_size: int, count: int, rates: list[float], workers: int) -> dict:
    """Serving: Poisson arrivals of requests drawn from a pool of seeded
    Chung-Lu / R-MAT graphs (1K-2M edges, (r,s) from {(1,2),(2,3),(3,4)}).
    For every rate: p50/p99 latency (submit to results ready on the device,
    server clock; and submit to results downloaded to the host, host clock)
    and completed graphs/s. Capacity (all requests submitted at once) is
    compared with a one-request-at-a-time server on the same requests."""
    import threading

    import numpy as np

    from paper_2306_08623_amd import inputs as I
    from paper_2306_08623_amd import nucleus

    t0 = time.perf_counter()
    pool = I.serve_graphs(pool_size)
    print(f"[bench] serve: generated {pool_size} requests in {time.perf_counter() - t0:.1f} s "
          f"(sum m = {sum(g.m for g, _, _ in pool)})", file=sys.stderr, flush=True)

    def run(rate: float | None, n_req: int, n_workers: int, max_batch: int) -> dict:
        rng = np.random.default_rng(12345)
        gaps = rng.exponential(1.0 / rate, size=n_req) if rate else np.zeros(n_req)
        arrive = np.cumsum(gaps)
        with nucleus.Server(device=0, workers=n_workers, max_batch=max_batch) as srv:
            tickets = [0] * n_req
            lag = np.zeros(n_req)
            t_submit_host = np.zeros(n_req)
            submitted = [threading.Event() for _ in range(n_req)]

            errors = []

            def submitter():
                start = time.perf_counter()
                try:
                    for i in range(n_req):
                        wait = start + arrive[i] - time.perf_counter()
                        if wait > 0:
                            time.sleep(wait)
                        lag[i] = time.perf_counter() - start - arrive[i]
                        g, r, s = pool[i % len(pool)]
                        t_submit_host[i] = time.perf_counter()
                        tickets[i] = srv.submit(g, r, s)
                        submitted[i].set()
                except Exception as e:          # surfaced by the collector below
                    errors.append(e)
                    for ev in submitted:
                        ev.set()

            th = threading.Thread(target=submitter)
            th.start()
            # collect results as they complete (any order): poll the
            # outstanding tickets, download each finished one to the host
            infos = [None] * n_req
            t_sub = np.zeros(n_req)
            t_got = np.zeros(n_req)
            pending = []
            nxt = 0
            while nxt < n_req or pending:
                while nxt < n_req and submitted[nxt].is_set():
                    if errors:
                        raise errors[0]
                    t_sub[nxt] = t_submit_host[nxt]
                    pending.append(nxt)
                    nxt += 1
                progressed = False
                for i in list(pending):
                    info = srv.poll(tickets[i])
                    if not info["done"]:
                        continue
                    if info["status"] != nucleus.ND_OK:
                        raise RuntimeError(f"request {i} failed: {info}")
                    srv.get(tickets[i], pool[i % len(pool)][1])   # results to the host
                    t_got[i] = time.perf_counter()
                    srv.release(tickets[i])
                    infos[i] = info
                    pending.remove(i)
                    progressed = True
                if errors:
                    raise errors[0]
                if not progressed:
                    time.sleep(0.0005)
            th.join()
            st = srv.stats()
        lat = np.array([x["t_done_ms"] - x["t_submit_ms"] for x in infos])
        e2e = (t_got - t_sub) * 1e3
        t_first = min(x["t_submit_ms"] for x in infos)
        t_last = max(x["t_done_ms"] for x in infos)
        return {
            "rate_req_s": rate, "requests": n_req,
            "graphs_per_s": n_req / ((t_last - t_first) * 1e-3),
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "p50_with_download_ms": float(np.percentile(e2e, 50)),
            "p99_with_download_ms": float(np.percentile(e2e, 99)),
            "mean_batch": float(np.mean([x["batch_size"] for x in infos])),
            "submit_lag_p99_ms": float(np.percentile(lag, 99) * 1e3),
            "batches": st["batches"], "overlapped": st["overlapped"],
            "device_overlap_ms": round(st["device_overlap_ms"], 3),
            "device_busy_ms": round(st["device_busy_ms"], 3),
        }

    out = {"workload": f"inputs.serve_graph(i, 5000000), i < {pool_size}: m log-uniform in "
                       "[1K, 2M], Chung-Lu (exponent 2.3, mean degree 8) or R-MAT (edge factor "
                       "8), (r,s) uniform over (1,2),(2,3),(3,4); Poisson arrivals (seed 12345)",
           "pool": pool_size, "workers": workers, "sweep": []}
    run(None, min(8, count), workers, 0)                                   # warm-up
    for rate in rates:
        res = run(rate, count, workers, 0)
        out["sweep"].append(res)
        print(f"[bench] serve: rate {rate}/s -> {res['graphs_per_s']:.1f} graphs/s, "
              f"p50 {res['p50_ms']:.1f} ms, p99 {res['p99_ms']:.1f} ms", file=sys.stderr,
              flush=True)
    cap = run(None, count, workers, 0)
    one = run(None, count, 1, 1)
    out["capacity_graphs_per_s"] = cap["graphs_per_s"]
    out["one_at_a_time_graphs_per_s"] = one["graphs_per_s"]
    out["capacity_speedup"] = cap["graphs_per_s"] / one["graphs_per_s"]
    print(f"[bench] serve: capacity {cap['graphs_per_s']:.1f} graphs/s vs one at a time "
          f"{one['graphs_per_s']:.1f}", file=sys.stderr, flush=True)
    return out


def measure(name: str, r: int, s: int, steps: int, warmup: int, peel_blocks: int) -> dict:
    """Decompose one workload `steps` times after `warmup` untimed runs, the
    CSR already in HBM; throughput, phases, counters and the roofline of the
    dominant kernel (its duration from HIP events on the library's stream)."""
    import torch

    from paper_2306_08623_amd import nucleus

    g, desc = workload(name)
    print(f"[bench] {desc}: n={g.n} m={g.m} (r,s)=({r},{s})", file=sys.stderr, flush=True)
    ctx = nucleus.Context(device=0, peel_blocks=peel_blocks)
    torch.cuda.synchronize()
    tu = time.perf_counter()
    ctx.load_csr(g)              # host -> HBM once (with validation); not in value
    ctx.nd_sync()
    upload_s = time.perf_counter() - tu
    ctx.nd_set_rs(r, s)
    retries = 0
    for i in range(warmup):
        tw = time.perf_counter()
        ctx.nd_decompose()
        retries += ctx.nd_get_info()["grid_retries"]
        print(f"[bench] warmup {i}: {time.perf_counter() - tw:.3f} s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for i in range(steps):
        ctx.nd_decompose()
        infos.append(ctx.nd_get_info())
        print(f"[bench] step {i}: {time.perf_counter() - t0:.3f} s cumulative", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.close()
    retries += sum(i["grid_retries"] for i in infos)
    if retries:
        print(f"[bench] WARNING: {retries} persistent launches were relaunched on a smaller "
              "grid (not fully resident)", file=sys.stderr, flush=True)
    info = infos[-1]
    n_s = info["n_s"]
    trav = n_s + comb(s, r) * n_s

    # roofline of the dominant kernel, timed with HIP events on the
    # library's stream around each launch
    peel_ms = sum(i["ms_peel_kernel"] for i in infos) / len(infos)
    count_ms = sum(i["ms_count_kernel"] for i in infos) / len(infos)
    b_visit, b_rclique, b_sclique = byte_model(r, s)
    peel_bytes = b_visit * info["visits"] + b_rclique * info["n_r"]
    count_bytes = b_sclique * n_s
    if peel_ms >= count_ms:
        kname, kms, kbytes = "k_peel", peel_ms, peel_bytes
    else:
        kname, kms, kbytes = "k_count_s4" if s == 4 else "k_count_s3", count_ms, count_bytes
    achieved = kbytes / (kms * 1e-3) / 1e9 if kms > 0 else 0.0
    traffic = measured_traffic(kname, name, r, s)
    roof = {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 2),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
            "traffic": traffic, "bytes_per_launch": kbytes, "kernel_ms": round(kms, 4)}
    if traffic:
        roof["traffic_GBps"] = round(traffic / (kms * 1e-3) / 1e9, 1)
        roof["traffic_over_model"] = round(traffic / kbytes, 2)
    return {
        "value": trav * steps / wall,
        "ms_per_step": 1000.0 * wall / steps,
        "steps": steps, "warmup": warmup,
        "config": {"workload": f"{desc}; (r,s)=({r},{s})", "n": g.n, "m": g.m,
                   "n_r": info["n_r"], "n_s": n_s, "k": info["k"], "rounds": info["rounds"],
                   "n_int": info["n_int"]},
        "host_upload_ms": round(upload_s * 1e3, 3),
        "value_with_host_upload": trav / (wall / steps + upload_s),
        "phases_ms": {"prep": round(info["ms_prep"], 3), "count": round(info["ms_count"], 3),
                      "peel": round(info["ms_peel"], 3), "tree": round(info["ms_tree"], 3)},
        "counters": {k: info[k] for k in ("visits", "decrements", "links", "link_calls", "unites",
                                           "bucket_scans", "max_outdeg", "orient_rounds")},
        "grid_retries": retries,
        "device_bytes": info["device_bytes"],
        "roofline": roof,
    }


def bench_cut_and_approx(name: str, r: int, s: int, delta: float, cpu_scale: int) -> dict:
    """The two query-side rows on the benched graph: the hierarchy cut (the
    c-(r,s) nuclei with vertex sets and induced edges) at five levels, and
    the approximate decomposition (Algorithm 2) against the exact one; the
    oracle's components-from-definition and approximate decomposition on the
    same scaled-down sample as the baseline."""
    import torch

    from paper_2306_08623_amd import nucleus

    g, _ = workload(name)
    out = {}
    with nucleus.Context(device=0) as ctx:
        ctx.load_csr(g)
        ctx.nd_set_rs(r, s)
        ctx.nd_decompose()
        info = ctx.nd_get_info()
        k = info["k"]
        cuts = []
        for c in sorted({1, max(1, k // 4), max(1, k // 2), max(1, 3 * k // 4), max(1, k)}):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            nn, nv = ctx.nd_cut(c)
            dt = time.perf_counter() - t0
            cuts.append({"c": c, "nuclei": nn, "vertices": nv, "ms": round(dt * 1e3, 3)})
        out["cut"] = {"levels": cuts, "k": k}
        print(f"[bench] cut: {cuts}", file=sys.stderr, flush=True)
        exact_rounds = info["rounds"]
        ctx.nd_set_approx(delta)
        ctx.nd_decompose()                      # warm-up of the approximate mode
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.nd_decompose()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ai = ctx.nd_get_info()
        ctx.nd_set_approx(0.0)
        out["approx"] = {"delta": delta, "ms": round(dt * 1e3, 3), "rounds": ai["rounds"],
                         "exact_rounds": exact_rounds, "k": ai["k"], "exact_k": k,
                         "round_cap": ai["round_cap"],
                         "phases_ms": {"prep": round(ai["ms_prep"], 3),
                                       "count": round(ai["ms_count"], 3),
                                       "peel": round(ai["ms_peel"], 3),
                                       "tree": round(ai["ms_tree"], 3)}}
        print(f"[bench] approx delta={delta}: {dt:.3f} s, {ai['rounds']} rounds "
              f"(exact {exact_rounds})", file=sys.stderr, flush=True)
    if cpu_scale:
        import oracle
        gs, what = cpu_sample(name, cpu_scale)
        d = oracle.decompose(gs, r, s)
        c = max(1, int(d.k) // 2)
        x = oracle.nuclei(gs, r, s, d.coreness, c)
        t0 = time.perf_counter()
        a = oracle.approx_decompose(gs, r, s, delta)
        ta = time.perf_counter() - t0
        out["cut"]["cpu_oracle"] = {"c": c, "nuclei": x["n_nuclei"], "seconds": x["seconds"],
                                    "cores": 1, "kind": "oracle",
                                    "sample": f"components of core >= c, no tree, on {what}"}
        out["approx"]["cpu_oracle"] = {"seconds": round(ta, 3), "exact_seconds":
                                       round(d.t_count + d.t_peel + d.t_tree, 3), "cores": 1,
                                       "kind": "oracle", "sample": what}
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="chunglu4m")
    ap.add_argument("--rs", default="3,4")
    ap.add_argument("--secondary", default="rmat18",
                    help="a second workload measured the same way ('' to skip)")
    ap.add_argument("--secondary-steps", type=int, default=3)
    ap.add_argument("--cpu-scale", type=int, default=7,
                    help="the oracle baseline runs on the workload's generator at a size "
                         "reduced by 2^scale (R-MAT: scale lower by this much) (0: skip)")
    ap.add_argument("--peel-blocks", type=int, default=0)
    ap.add_argument("--queries", type=int, default=1,
                    help="hierarchy cut and approximate decomposition objects (0: skip)")
    ap.add_argument("--delta", type=float, default=0.5)
    ap.add_argument("--batch", type=int, default=4096,
                    help="graphs in the batched-vs-one-by-one comparison (0: skip)")
    ap.add_argument("--batch-reps", type=int, default=2)
    ap.add_argument("--serve", type=int, default=64,
                    help="requests per rate in the serving sweep (0: skip)")
    ap.add_argument("--serve-pool", type=int, default=64)
    ap.add_argument("--serve-rates", default="10,20,50,100,200,500,1000,2000")
    ap.add_argument("--serve-workers", type=int, default=2)
    ap.add_argument("--verbose", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the decomposition of one graph is not "
              "sharded across GPUs.", file=sys.stderr)
        return 2
    r, s = (int(x) for x in args.rs.split(","))

    import torch

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    head = measure(args.workload, r, s, args.steps, args.warmup, args.peel_blocks)
    out = {
        "metric": f"({r},{s})-nucleus s-cliques traversed/s",
        "value": head["value"],
        "unit": "s-cliques traversed/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
    }
    for key in ("config", "host_upload_ms", "value_with_host_upload", "phases_ms", "counters",
                "grid_retries", "device_bytes", "roofline"):
        out[key] = head[key]
    if args.secondary:
        out["secondary"] = measure(args.secondary, r, s, args.secondary_steps, 1,
                                   args.peel_blocks)
    if args.queries:
        out.update(bench_cut_and_approx(args.workload, r, s, args.delta, args.cpu_scale))
    if args.batch:
        out["batch"] = bench_batch(args.batch, args.batch_reps)
    if args.serve:
        out["serve"] = bench_serve(args.serve_pool, args.serve,
                                   [float(x) for x in args.serve_rates.split(",")],
                                   args.serve_workers)
    if args.cpu_scale:
        out["cpu_baseline"] = cpu_baseline(args.workload, r, s, args.cpu_scale)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
