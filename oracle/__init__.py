"""ctypes wrapper of the sequential CPU oracle (``ndo.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU baseline of
the benchmark may import this package; the product library and its Python
binding never do. It shares no code with the GPU path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from math import comb

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ndo.c")
_LIB = os.path.join(_HERE, "libndo.so")

NDO_OK = 0
NDO_E_INVALID_ARG = 1
NDO_E_BAD_GRAPH = 2
NDO_E_OOM = 3
NONE = np.uint64(0xFFFFFFFFFFFFFFFF)


class _Result(C.Structure):
    _fields_ = [
        ("n", C.c_uint32), ("r", C.c_uint32), ("s", C.c_uint32),
        ("n_r", C.c_uint64), ("n_s", C.c_uint64),
        ("rcliques", C.POINTER(C.c_uint32)),
        ("count", C.POINTER(C.c_uint64)),
        ("coreness", C.POINTER(C.c_uint64)),
        ("peel_order", C.POINTER(C.c_uint64)),
        ("k", C.c_uint64),
        ("n_int", C.c_uint64),
        ("parent", C.POINTER(C.c_uint64)),
        ("level", C.POINTER(C.c_uint64)),
        ("t_count", C.c_double), ("t_peel", C.c_double), ("t_tree", C.c_double),
    ]


class _Cut(C.Structure):
    _fields_ = [
        ("n_r", C.c_uint64), ("n_nuclei", C.c_uint64),
        ("leaf_nucleus", C.POINTER(C.c_uint64)),
        ("min_leaf", C.POINTER(C.c_uint64)),
        ("level", C.POINTER(C.c_uint64)),
        ("n_rcliques", C.POINTER(C.c_uint64)),
        ("n_vertices", C.POINTER(C.c_uint64)),
        ("n_edges", C.POINTER(C.c_uint64)),
        ("vert_off", C.POINTER(C.c_uint64)),
        ("verts", C.POINTER(C.c_uint32)),
        ("t_cut", C.c_double),
    ]


def build(force: bool = False) -> str:
    """Compile ``libndo.so`` with gcc (portable flags, single-threaded)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-Wall", "-fPIC", "-shared",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = C.CDLL(_LIB)
        u64p = C.POINTER(C.c_uint64)
        u32p = C.POINTER(C.c_uint32)
        lib.ndo_validate_csr.argtypes = [C.c_uint32, u64p, u32p]
        lib.ndo_validate_csr.restype = C.c_int
        lib.ndo_decompose.argtypes = [C.c_uint32, u64p, u32p, C.c_uint32, C.c_uint32,
                                      C.POINTER(_Result)]
        lib.ndo_decompose.restype = C.c_int
        lib.ndo_count.argtypes = lib.ndo_decompose.argtypes
        lib.ndo_count.restype = C.c_int
        lib.ndo_free.argtypes = [C.POINTER(_Result)]
        lib.ndo_free.restype = None
        lib.ndo_open.argtypes = [C.c_uint32, u64p, u32p, C.c_uint32, C.c_uint32,
                                 C.POINTER(C.c_void_p)]
        lib.ndo_open.restype = C.c_int
        lib.ndo_approx_decompose.argtypes = [C.c_uint32, u64p, u32p, C.c_uint32, C.c_uint32,
                                             C.c_double, C.POINTER(_Result)]
        lib.ndo_approx_decompose.restype = C.c_int
        lib.ndo_nuclei.argtypes = [C.c_uint32, u64p, u32p, C.c_uint32, C.c_uint32, u64p,
                                   C.c_uint64, C.POINTER(_Cut)]
        lib.ndo_nuclei.restype = C.c_int
        lib.ndo_cut_free.argtypes = [C.POINTER(_Cut)]
        lib.ndo_cut_free.restype = None
        lib.ndo_graph_n_r.argtypes = [C.c_void_p]
        lib.ndo_graph_n_r.restype = C.c_uint64
        lib.ndo_graph_rcliques.argtypes = [C.c_void_p, u32p]
        lib.ndo_graph_rcliques.restype = None
        lib.ndo_incident.argtypes = [C.c_void_p, C.c_uint64, u64p, C.c_uint64]
        lib.ndo_incident.restype = C.c_uint64
        lib.ndo_close.argtypes = [C.c_void_p]
        lib.ndo_close.restype = None
        _lib = lib
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error code {code}")
        self.code = code


@dataclass
class Decomposition:
    n: int
    r: int
    s: int
    n_r: int
    n_s: int
    rcliques: np.ndarray      # uint32 [n_r, r]
    count: np.ndarray         # uint64 [n_r]
    coreness: np.ndarray | None = None    # uint64 [n_r]
    peel_order: np.ndarray | None = None  # uint64 [n_r]
    k: int = 0
    n_int: int = 0
    parent: np.ndarray | None = None      # uint64 [n_r + n_int]
    level: np.ndarray | None = None       # uint64 [n_int]
    t_count: float = 0.0
    t_peel: float = 0.0
    t_tree: float = 0.0


def _arr(ptr, n, dtype):
    if n == 0:
        return np.zeros(0, dtype=dtype)
    return np.ctypeslib.as_array(ptr, shape=(n,)).astype(dtype, copy=True)


def _csr_args(csr):
    rp = np.ascontiguousarray(csr.row_ptr, dtype=np.uint64)
    col = np.ascontiguousarray(csr.col, dtype=np.uint32)
    if col.size == 0:
        col = np.zeros(1, dtype=np.uint32)
    return rp, col


def validate(csr) -> int:
    lib = _load()
    rp, col = _csr_args(csr)
    return lib.ndo_validate_csr(csr.n, rp.ctypes.data_as(C.POINTER(C.c_uint64)),
                                col.ctypes.data_as(C.POINTER(C.c_uint32)))


def _run(fn_name: str, csr, r: int, s: int, full: bool, *extra) -> Decomposition:
    lib = _load()
    rp, col = _csr_args(csr)
    res = _Result()
    st = getattr(lib, fn_name)(csr.n, rp.ctypes.data_as(C.POINTER(C.c_uint64)),
                               col.ctypes.data_as(C.POINTER(C.c_uint32)), r, s, *extra,
                               C.byref(res))
    if st != NDO_OK:
        raise OracleError(st)
    try:
        n_r = int(res.n_r)
        d = Decomposition(
            n=int(res.n), r=int(res.r), s=int(res.s), n_r=n_r, n_s=int(res.n_s),
            rcliques=_arr(res.rcliques, n_r * r, np.uint32).reshape(n_r, r),
            count=_arr(res.count, n_r, np.uint64),
            t_count=float(res.t_count))
        if full:
            n_int = int(res.n_int)
            d.coreness = _arr(res.coreness, n_r, np.uint64)
            d.peel_order = _arr(res.peel_order, n_r, np.uint64)
            d.k = int(res.k)
            d.n_int = n_int
            d.parent = _arr(res.parent, n_r + n_int, np.uint64)
            d.level = _arr(res.level, n_int, np.uint64)
            d.t_peel = float(res.t_peel)
            d.t_tree = float(res.t_tree)
        return d
    finally:
        lib.ndo_free(C.byref(res))


class Graph:
    """Per-r-clique queries (the oracle's own listing and s-clique scan) for
    graphs too large for a full decomposition."""

    def __init__(self, csr, r: int, s: int):
        lib = _load()
        rp, col = _csr_args(csr)
        self._keep = (rp, col)
        h = C.c_void_p()
        st = lib.ndo_open(csr.n, rp.ctypes.data_as(C.POINTER(C.c_uint64)),
                          col.ctypes.data_as(C.POINTER(C.c_uint32)), r, s, C.byref(h))
        if st != NDO_OK:
            raise OracleError(st)
        self.h = h
        self.r, self.s = r, s
        self.n_r = int(lib.ndo_graph_n_r(h))
        self.others_per_s = comb(s, r) - 1

    def rcliques(self) -> np.ndarray:
        out = np.zeros((self.n_r, self.r), dtype=np.uint32)
        if self.n_r:
            _load().ndo_graph_rcliques(self.h, out.ctypes.data_as(C.POINTER(C.c_uint32)))
        return out

    def incident(self, rid: int) -> np.ndarray:
        """[n_S, C(s,r)-1] ids of the other r-cliques of every s-clique
        containing r-clique ``rid``."""
        lib = _load()
        n_s = int(lib.ndo_incident(self.h, rid, None, 0))
        out = np.zeros(max(1, n_s * self.others_per_s), dtype=np.uint64)
        lib.ndo_incident(self.h, rid, out.ctypes.data_as(C.POINTER(C.c_uint64)), out.size)
        return out[: n_s * self.others_per_s].reshape(n_s, self.others_per_s)

    def close(self):
        if getattr(self, "h", None):
            _load().ndo_close(self.h)
            self.h = None

    def __del__(self):
        self.close()


def decompose(csr, r: int, s: int) -> Decomposition:
    """Full oracle: r-cliques, counts, coreness, canonical tree."""
    return _run("ndo_decompose", csr, r, s, True)


def approx_decompose(csr, r: int, s: int, delta: float) -> Decomposition:
    """Approximate core numbers (Algorithm 2, round-synchronous, geometric
    buckets of parameter delta) and the canonical tree of those values."""
    return _run("ndo_approx_decompose", csr, r, s, True, C.c_double(delta))


def count(csr, r: int, s: int) -> Decomposition:
    """Only r-clique listing and per-r-clique s-clique counts."""
    return _run("ndo_count", csr, r, s, False)


def nuclei(csr, r: int, s: int, coreness, c: int) -> dict:
    """The c-(r,s) nuclei from the definition (components of the r-cliques of
    core >= c under s-clique adjacency, no tree): per nucleus, numbered by
    its smallest r-clique id, that id, its level (smallest core inside), its
    r-clique count, sorted vertex set and the edges of G among those
    vertices; plus every r-clique's nucleus (-1 = none) and the seconds the
    query took."""
    lib = _load()
    rp, col = _csr_args(csr)
    core = np.ascontiguousarray(coreness, dtype=np.uint64)
    if core.size == 0:
        core = np.zeros(1, dtype=np.uint64)
    res = _Cut()
    st = lib.ndo_nuclei(csr.n, rp.ctypes.data_as(C.POINTER(C.c_uint64)),
                        col.ctypes.data_as(C.POINTER(C.c_uint32)), r, s,
                        core.ctypes.data_as(C.POINTER(C.c_uint64)), c, C.byref(res))
    if st != NDO_OK:
        raise OracleError(st)
    try:
        nn, n_r = int(res.n_nuclei), int(res.n_r)
        off = _arr(res.vert_off, nn + 1, np.uint64) if nn else np.zeros(1, np.uint64)
        leaf = _arr(res.leaf_nucleus, n_r, np.uint64).astype(np.int64)
        return {
            "n_nuclei": nn,
            "leaf_nucleus": leaf,
            "min_leaf": _arr(res.min_leaf, nn, np.uint64),
            "level": _arr(res.level, nn, np.uint64),
            "n_rcliques": _arr(res.n_rcliques, nn, np.uint64),
            "n_vertices": _arr(res.n_vertices, nn, np.uint64),
            "n_edges": _arr(res.n_edges, nn, np.uint64),
            "vert_off": off,
            "verts": _arr(res.verts, int(off[-1]), np.uint32),
            "seconds": float(res.t_cut),
        }
    finally:
        lib.ndo_cut_free(C.byref(res))
