"""Seeded synthetic graph generators and CSR construction.

This module only produces input graphs. It holds none of the nucleus
decomposition arithmetic (no clique enumeration, counting or peeling), so the
GPU path, the CPU oracle and the tests can all draw their inputs from it.

Every generator takes an explicit integer seed and uses numpy's PCG64 bit
generator, so a (generator, parameters, seed) triple always yields the same
graph. The paper's inputs are simple undirected graphs (Section 3,
"Graph Notation and Definitions"); every generator here ends in
:func:`to_csr`, which symmetrises, drops self-loops, removes duplicate edges
and sorts each row, giving a CSR with ``row_ptr`` as uint64[n+1] and ``col``
as uint32[2m].

The paper measures on SNAP graphs (Table 1). Those datasets are not available,
so these generators stand in for them:

* ``er_planted``   Erdos-Renyi G(n, p) plus planted cliques.
* ``rmat``         R-MAT with Graph500-style vertex-id permutation.
* ``chung_lu``     power-law expected-degree graphs, optionally with planted
                   dense communities.
"""
from __future__ import annotations

import hashlib
import os
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class CSR:
    """Undirected simple graph in symmetric CSR form.

    ``row_ptr``: uint64[n+1]; ``col``: uint32[row_ptr[n]] with each row sorted
    ascending, no self-loops and no duplicates; ``col`` is symmetric.
    """

    n: int
    row_ptr: np.ndarray
    col: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.uint64(self.n).tobytes())
        h.update(np.ascontiguousarray(self.row_ptr, dtype=np.uint64).tobytes())
        h.update(np.ascontiguousarray(self.col, dtype=np.uint32).tobytes())
        return h.hexdigest()

    def edges(self) -> np.ndarray:
        """Undirected edges (u < v) as an int64[m, 2] array, lexicographic."""
        deg = np.diff(self.row_ptr.astype(np.int64))
        src = np.repeat(np.arange(self.n, dtype=np.int64), deg)
        dst = self.col.astype(np.int64)
        keep = src < dst
        return np.stack([src[keep], dst[keep]], axis=1)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def to_csr(n: int, src: np.ndarray, dst: np.ndarray) -> CSR:
    """Build a simple undirected CSR from an arbitrary (possibly directed,
    duplicated, self-looped) edge list over vertices ``0..n-1``."""
    if n < 0 or n > 0xFFFFFFFF:
        raise ValueError("n out of range for uint32 vertex ids")
    src = np.asarray(src, dtype=np.int64).ravel()
    dst = np.asarray(dst, dtype=np.int64).ravel()
    if src.shape != dst.shape:
        raise ValueError("src/dst length mismatch")
    if src.size and (src.min() < 0 or dst.min() < 0 or src.max() >= n or dst.max() >= n):
        raise ValueError("vertex id out of range")
    keep = src != dst
    src, dst = src[keep], dst[keep]
    u = np.minimum(src, dst).astype(np.uint64)
    v = np.maximum(src, dst).astype(np.uint64)
    key = np.unique((u << np.uint64(32)) | v)
    u = (key >> np.uint64(32)).astype(np.int64)
    v = (key & np.uint64(0xFFFFFFFF)).astype(np.int64)
    # both directions, ordered by (row, column): one sort of packed keys
    both = np.concatenate([(u.astype(np.uint64) << np.uint64(32)) | v.astype(np.uint64),
                           (v.astype(np.uint64) << np.uint64(32)) | u.astype(np.uint64)])
    both.sort()
    a = (both >> np.uint64(32)).astype(np.int64)
    b = both & np.uint64(0xFFFFFFFF)
    del both
    counts = np.bincount(a, minlength=n) if n else np.zeros(0, dtype=np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.uint64)
    if n:
        row_ptr[1:] = np.cumsum(counts, dtype=np.uint64)
    return CSR(n=n, row_ptr=row_ptr, col=b.astype(np.uint32))


def from_edges(n: int, edges) -> CSR:
    """CSR from a python list / array of (u, v) pairs."""
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    return to_csr(n, e[:, 0], e[:, 1])


def empty(n: int) -> CSR:
    return to_csr(n, np.zeros(0, np.int64), np.zeros(0, np.int64))


# ---------------------------------------------------------------------------
# Small structured graphs used by tests (closed forms)
# ---------------------------------------------------------------------------

def complete(n: int) -> CSR:
    iu = np.triu_indices(n, 1)
    return to_csr(n, iu[0], iu[1])


def disjoint_union(*graphs: CSR) -> CSR:
    srcs, dsts, off = [], [], 0
    for g in graphs:
        e = g.edges()
        srcs.append(e[:, 0] + off)
        dsts.append(e[:, 1] + off)
        off += g.n
    if not srcs:
        return empty(0)
    return to_csr(off, np.concatenate(srcs), np.concatenate(dsts))


def cycle(n: int) -> CSR:
    i = np.arange(n)
    return to_csr(n, i, (i + 1) % n)


def star(n: int) -> CSR:
    i = np.arange(1, n)
    return to_csr(n, np.zeros_like(i), i)


def two_k5_bridge() -> CSR:
    """Two K5 sharing vertex 0, plus one extra edge between vertex 1 (in the
    first K5) and vertex 5 (in the second K5)."""
    a = [0, 1, 2, 3, 4]
    b = [0, 5, 6, 7, 8]
    e = []
    for grp in (a, b):
        for i in range(5):
            for j in range(i + 1, 5):
                e.append((grp[i], grp[j]))
    e.append((1, 5))
    return from_edges(9, e)


# ---------------------------------------------------------------------------
# Random generators
# ---------------------------------------------------------------------------

def _sample_pairs(rng: np.random.Generator, n: int, count: int) -> tuple[np.ndarray, np.ndarray]:
    """``count`` distinct unordered pairs {u, v}, u != v, uniform over all
    C(n, 2) pairs (rejection of repeats)."""
    total = n * (n - 1) // 2
    if count > total:
        raise ValueError("more pairs requested than exist")
    have = np.zeros(0, dtype=np.uint64)
    while have.size < count:
        need = count - have.size
        k = int(need * 1.1) + 16
        u = rng.integers(0, n, size=k, dtype=np.int64)
        v = rng.integers(0, n, size=k, dtype=np.int64)
        ok = u != v
        u, v = u[ok], v[ok]
        lo = np.minimum(u, v).astype(np.uint64)
        hi = np.maximum(u, v).astype(np.uint64)
        key = (lo << np.uint64(32)) | hi
        # keep first occurrence order-independent: unique then random subset
        merged = np.unique(np.concatenate([have, key]))
        if merged.size > count:
            extra = np.setdiff1d(merged, have, assume_unique=True)
            pick = rng.choice(extra.size, size=count - have.size, replace=False)
            merged = np.sort(np.concatenate([have, extra[pick]]))
        have = merged
    return (have >> np.uint64(32)).astype(np.int64), (have & np.uint64(0xFFFFFFFF)).astype(np.int64)


def erdos_renyi_edges(rng: np.random.Generator, n: int, p: float) -> tuple[np.ndarray, np.ndarray]:
    """G(n, p): the edge count is Binomial(C(n,2), p) and the edge set is a
    uniform subset of that size, which is exactly the G(n, p) law."""
    total = n * (n - 1) // 2
    if total == 0 or p <= 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    cnt = int(rng.binomial(total, min(p, 1.0)))
    return _sample_pairs(rng, n, cnt)


def planted_clique_edges(rng: np.random.Generator, n: int, count: int,
                         size_lo: int, size_hi: int) -> tuple[np.ndarray, np.ndarray]:
    """``count`` cliques, each on a uniformly random vertex subset whose size
    is uniform on [size_lo, size_hi]; cliques may overlap."""
    srcs, dsts = [], []
    for _ in range(count):
        q = int(rng.integers(size_lo, size_hi + 1))
        q = min(q, n)
        vs = rng.choice(n, size=q, replace=False).astype(np.int64)
        iu = np.triu_indices(q, 1)
        srcs.append(vs[iu[0]])
        dsts.append(vs[iu[1]])
    if not srcs:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(srcs), np.concatenate(dsts)


def er_planted(n: int, p: float, n_cliques: int, size_lo: int, size_hi: int, seed: int) -> CSR:
    rng = _rng(seed)
    s1, d1 = erdos_renyi_edges(rng, n, p)
    s2, d2 = planted_clique_edges(rng, n, n_cliques, size_lo, size_hi)
    return to_csr(n, np.concatenate([s1, s2]), np.concatenate([d1, d2]))


def rmat_edges(rng: np.random.Generator, scale: int, n_edges: int,
               a: float = 0.57, b: float = 0.19, c: float = 0.19,
               permute: bool = True) -> tuple[np.ndarray, np.ndarray]:
    """R-MAT edge samples: at each of ``scale`` levels pick a quadrant with
    probabilities (a, b, c, 1-a-b-c); then (Graph500 convention) relabel the
    vertices with a seeded random permutation."""
    n = 1 << scale
    src = np.zeros(n_edges, dtype=np.int64)
    dst = np.zeros(n_edges, dtype=np.int64)
    ab = a + b
    abc = a + b + c
    chunk = 1 << 22
    for lo in range(0, n_edges, chunk):
        hi = min(n_edges, lo + chunk)
        k = hi - lo
        s = np.zeros(k, dtype=np.int64)
        d = np.zeros(k, dtype=np.int64)
        for _ in range(scale):
            r = rng.random(k)
            sbit = (r >= ab).astype(np.int64)
            dbit = (((r >= a) & (r < ab)) | (r >= abc)).astype(np.int64)
            s = (s << 1) | sbit
            d = (d << 1) | dbit
        src[lo:hi] = s
        dst[lo:hi] = d
    if permute:
        perm = rng.permutation(n).astype(np.int64)
        src = perm[src]
        dst = perm[dst]
    return src, dst


def rmat(scale: int, edge_factor: int, seed: int, a: float = 0.57, b: float = 0.19,
         c: float = 0.19) -> CSR:
    rng = _rng(seed)
    n = 1 << scale
    s, d = rmat_edges(rng, scale, edge_factor * n, a, b, c)
    return to_csr(n, s, d)


def chung_lu_weights(n: int, gamma: float, mean_degree: float, w_max: float) -> np.ndarray:
    """Power-law expected-degree weights w_i = w_max * ((i + i0) / i0)^(-1/(gamma-1))
    (so w_0 = w_max and the tail falls off with exponent gamma), with the
    offset i0 chosen by bisection so the mean weight equals ``mean_degree``;
    the mean grows with i0, from 0 towards w_max (clamped at the ends)."""
    if n == 0:
        return np.zeros(0)
    expo = -1.0 / (gamma - 1.0)
    i = np.arange(n, dtype=np.float64)

    def mean_w(i0: float) -> float:
        return float(np.mean(w_max * ((i + i0) / i0) ** expo))

    lo, hi = 1e-9, 1e12
    if mean_w(hi) < mean_degree:
        i0 = hi
    elif mean_w(lo) > mean_degree:
        i0 = lo
    else:
        for _ in range(200):
            mid = np.sqrt(lo * hi)
            if mean_w(mid) > mean_degree:
                hi = mid
            else:
                lo = mid
        i0 = np.sqrt(lo * hi)
    return w_max * ((i + i0) / i0) ** expo


def _inverse_cdf(cdf: np.ndarray, x: np.ndarray) -> np.ndarray:
    """searchsorted(cdf, x, side="right") for unsorted x, answered in sorted
    order (far fewer cache misses on large inputs), same result."""
    order = np.argsort(x)
    out = np.empty(x.size, dtype=np.int64)
    out[order] = np.searchsorted(cdf, x[order], side="right")
    return out


def chung_lu_edges(rng: np.random.Generator, n: int, gamma: float, mean_degree: float,
                   w_max: float, target_edges: int | None = None) -> tuple[np.ndarray, np.ndarray]:
    """Sample endpoints proportionally to the weights (weights assigned to a
    random permutation of ids), redrawing until ``target_edges`` distinct
    undirected non-loop edges exist (default: n * mean_degree / 2)."""
    if n < 2:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    w = chung_lu_weights(n, gamma, mean_degree, w_max)
    w = w[rng.permutation(n)]
    prob = w / w.sum()
    cdf = np.cumsum(prob)
    cdf[-1] = 1.0
    if target_edges is None:
        target_edges = int(round(n * mean_degree / 2))
    target_edges = min(target_edges, n * (n - 1) // 2)
    have = np.zeros(0, dtype=np.uint64)
    rounds = 0
    while have.size < target_edges and rounds < 64:
        rounds += 1
        need = target_edges - have.size
        k = int(need * 1.05) + 64
        u = _inverse_cdf(cdf, rng.random(k))
        v = _inverse_cdf(cdf, rng.random(k))
        u = np.minimum(u, n - 1)
        v = np.minimum(v, n - 1)
        ok = u != v
        lo = np.minimum(u[ok], v[ok]).astype(np.uint64)
        hi = np.maximum(u[ok], v[ok]).astype(np.uint64)
        key = (lo << np.uint64(32)) | hi
        merged = np.unique(np.concatenate([have, key]))
        if merged.size > target_edges:
            extra = np.setdiff1d(merged, have, assume_unique=True)
            pick = rng.choice(extra.size, size=target_edges - have.size, replace=False)
            merged = np.sort(np.concatenate([have, extra[pick]]))
        have = merged
    return (have >> np.uint64(32)).astype(np.int64), (have & np.uint64(0xFFFFFFFF)).astype(np.int64)


def community_edges(rng: np.random.Generator, n: int, count: int, size_lo: int,
                    size_hi: int, density: float) -> tuple[np.ndarray, np.ndarray]:
    """``count`` vertex-disjoint communities (random vertex sets), sizes uniform
    on [size_lo, size_hi], each internal pair present with prob ``density``."""
    sizes = rng.integers(size_lo, size_hi + 1, size=count)
    total = int(sizes.sum())
    if total > n:
        raise ValueError("communities do not fit")
    verts = rng.choice(n, size=total, replace=False).astype(np.int64)
    srcs, dsts, off = [], [], 0
    for q in sizes:
        q = int(q)
        vs = verts[off:off + q]
        off += q
        iu = np.triu_indices(q, 1)
        keep = rng.random(iu[0].size) < density
        srcs.append(vs[iu[0][keep]])
        dsts.append(vs[iu[1][keep]])
    if not srcs:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(srcs), np.concatenate(dsts)


def chung_lu(n: int, gamma: float, mean_degree: float, w_max: float, seed: int,
             target_edges: int | None = None, n_cliques: int = 0, clique_lo: int = 6,
             clique_hi: int = 24, n_communities: int = 0, comm_lo: int = 20,
             comm_hi: int = 200, comm_density: float = 0.6) -> CSR:
    rng = _rng(seed)
    s, d = chung_lu_edges(rng, n, gamma, mean_degree, w_max, target_edges)
    parts_s, parts_d = [s], [d]
    if n_cliques:
        s2, d2 = planted_clique_edges(rng, n, n_cliques, clique_lo, clique_hi)
        parts_s.append(s2)
        parts_d.append(d2)
    if n_communities:
        s3, d3 = community_edges(rng, n, n_communities, comm_lo, comm_hi, comm_density)
        parts_s.append(s3)
        parts_d.append(d3)
    return to_csr(n, np.concatenate(parts_s), np.concatenate(parts_d))


def gnp(n: int, p: float, seed: int) -> CSR:
    rng = _rng(seed)
    s, d = erdos_renyi_edges(rng, n, p)
    return to_csr(n, s, d)


# ---------------------------------------------------------------------------
# The named workloads
# ---------------------------------------------------------------------------

def workload_er2k(seed: int = 1) -> CSR:
    """G(2000, 0.01) plus 20 planted cliques of sizes uniform in [5, 30]."""
    return er_planted(2000, 0.01, 20, 5, 30, seed)


def workload_rmat18(seed: int = 2) -> CSR:
    """R-MAT scale 18, edge factor 16, (a,b,c,d) = (.57,.19,.19,.05)."""
    return rmat(18, 16, seed)


def workload_chung_lu_4m(seed: int = 3) -> CSR:
    """Chung-Lu n=4,000,000, exponent 2.1, ~40M edges, max expected degree
    20,000, plus 1,000 disjoint communities of sizes 20..200 at density 0.6."""
    return chung_lu(4_000_000, 2.1, 20.0, 20_000.0, seed, target_edges=40_000_000,
                    n_communities=1000, comm_lo=20, comm_hi=200, comm_density=0.6)


def batch_graph(i: int, base_seed: int = 4_000_000) -> tuple[CSR, int, int]:
    """Graph ``i`` of the mixed batch: n log-uniform in [64, 65536]; half
    Erdos-Renyi with average degree 8, half Chung-Lu (exponent 2.3, mean
    degree 8); 1-10 planted cliques of sizes 6-24; (r, s) alternating
    (2,3) / (3,4)."""
    rng = _rng(base_seed + i)
    n = int(round(np.exp(rng.uniform(np.log(64), np.log(65536)))))
    n = max(64, min(65536, n))
    n_cl = int(rng.integers(1, 11))
    sub_seed = int(rng.integers(0, 2**62))
    if i % 2 == 0:
        g = er_planted(n, 8.0 / (n - 1), n_cl, 6, 24, sub_seed)
    else:
        w_max = min(n - 1.0, n ** (1.0 / (2.3 - 1.0)))
        g = chung_lu(n, 2.3, 8.0, w_max, sub_seed, n_cliques=n_cl, clique_lo=6,
                     clique_hi=24)
    r, s = ((2, 3), (3, 4))[(i // 2) % 2]
    return g, r, s


def _batch_item(args):
    i, base_seed = args
    return batch_graph(i, base_seed)


def batch_graphs(count: int = 4096, base_seed: int = 4_000_000,
                 workers: int = 0) -> list[tuple[CSR, int, int]]:
    """Graphs 0..count-1 of the mixed batch, made in ``workers`` spawned
    processes (0: up to 16). The result does not depend on ``workers``."""
    if workers <= 0:
        workers = min(16, os.cpu_count() or 1)
    if workers <= 1 or count < 64:
        return [batch_graph(i, base_seed) for i in range(count)]
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(workers) as pool:
        return pool.map(_batch_item, [(i, base_seed) for i in range(count)], chunksize=8)


def serve_graph(i: int, base_seed: int = 5_000_000, m_lo: int = 1_000,
                m_hi: int = 2_000_000) -> tuple[CSR, int, int]:
    """Request ``i`` of the serving stream: m log-uniform in [m_lo, m_hi];
    50/50 Chung-Lu (exponent 2.3, mean degree 8) or R-MAT (edge factor 8);
    (r, s) uniform over {(1,2), (2,3), (3,4)}."""
    rng = _rng(base_seed + i)
    m = int(round(np.exp(rng.uniform(np.log(m_lo), np.log(m_hi)))))
    r, s = ((1, 2), (2, 3), (3, 4))[int(rng.integers(0, 3))]
    sub_seed = int(rng.integers(0, 2**62))
    if rng.random() < 0.5:
        n = max(16, m // 4)
        w_max = min(n - 1.0, n ** (1.0 / (2.3 - 1.0)))
        g = chung_lu(n, 2.3, 8.0, w_max, sub_seed, target_edges=m)
    else:
        scale = max(4, int(round(np.log2(max(2, m / 8)))))
        g = rmat(scale, 8, sub_seed)
    return g, r, s


def _serve_item(args):
    i, base_seed = args
    return serve_graph(i, base_seed)


def serve_graphs(count: int, base_seed: int = 5_000_000,
                 workers: int = 0) -> list[tuple[CSR, int, int]]:
    """Requests 0..count-1 of the serving stream, made in ``workers`` spawned
    processes (0: up to 16). The result does not depend on ``workers``."""
    if workers <= 0:
        workers = min(16, os.cpu_count() or 1)
    if workers <= 1 or count < 8:
        return [serve_graph(i, base_seed) for i in range(count)]
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(workers) as pool:
        return pool.map(_serve_item, [(i, base_seed) for i in range(count)], chunksize=1)


# ---------------------------------------------------------------------------
# Binary CSR files (for the C++ profiling driver)
# ---------------------------------------------------------------------------

def save_csr(csr: CSR, path: str) -> None:
    """uint32 n, uint64 nnz, uint64 row_ptr[n+1], uint32 col[nnz], little endian."""
    with open(path, "wb") as f:
        f.write(np.uint32(csr.n).tobytes())
        f.write(np.uint64(csr.nnz).tobytes())
        f.write(np.ascontiguousarray(csr.row_ptr, dtype="<u8").tobytes())
        f.write(np.ascontiguousarray(csr.col, dtype="<u4").tobytes())


def load_csr(path: str) -> CSR:
    with open(path, "rb") as f:
        n = int(np.frombuffer(f.read(4), dtype="<u4")[0])
        nnz = int(np.frombuffer(f.read(8), dtype="<u8")[0])
        rp = np.frombuffer(f.read(8 * (n + 1)), dtype="<u8").astype(np.uint64)
        col = np.frombuffer(f.read(4 * nnz), dtype="<u4").astype(np.uint32)
    return CSR(n=n, row_ptr=rp, col=col)
