"""Python binding of the gfx950 nucleus decomposition library (``libnucleus.so``).

Argument marshalling only: every step of the decomposition runs in the HIP
kernels of the library. The names mirror the C ABI in ``include/nucleus.h``.
PyTorch is used, when present, only to hand device memory (CUDA tensors) and
the current HIP stream to the library.

The library must have been built (``python -m paper_2306_08623_amd.build`` or
``__graft_entry__.build()``); importing a context without it raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

try:  # load PyTorch's HIP runtime first: the library runs on that one
    import torch  # noqa: F401
except ImportError:  # pragma: no cover - torch is part of the image
    torch = None

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnucleus.so")

ND_OK = 0
ND_E_INVALID_ARG = 1
ND_E_BAD_GRAPH = 2
ND_E_UNSUPPORTED = 3
ND_E_OOM = 4
ND_E_OVERFLOW = 5
ND_E_DEVICE = 6
ND_E_WATCHDOG = 7
ND_E_STATE = 8
ND_E_CANCELLED = 9

ND_MEM_HOST = 0
ND_MEM_DEVICE = 1

ND_FLAG_PROGRESS = 1
ND_FLAG_HIER_EL = 2
ND_FLAG_HIER_TE = 4
ND_FLAG_COUNT_GLOBAL = 8

NONE64 = np.uint64(0xFFFFFFFFFFFFFFFF)

# Every function the C ABI exports (kept in sync with include/nucleus.h).
EXPORTS = [
    "nd_create", "nd_destroy", "nd_load_csr", "nd_set_rs", "nd_decompose", "nd_sync",
    "nd_get_info", "nd_get_rcliques", "nd_get_counts", "nd_get_coreness", "nd_get_peel_rounds",
    "nd_get_tree", "nd_batch_decompose", "nd_batch_get", "nd_estimate_footprint",
    "nd_server_create", "nd_server_destroy", "nd_server_submit", "nd_server_poll",
    "nd_server_wait", "nd_server_get", "nd_server_release", "nd_server_cancel",
    "nd_server_get_stats", "nd_server_last_error", "nd_decompose_noalloc",
    "nd_cut", "nd_get_cut", "nd_set_approx", "nd_set_schedule",
    "nd_status_str", "nd_last_error",
]

# fixed device scratch of nd_decompose_noalloc, per GPU (include/nucleus.h)
ND_NOALLOC_SCRATCH_BYTES = 64 << 20


class Options(C.Structure):
    _fields_ = [
        ("device", C.c_int),
        ("hip_stream", C.c_void_p),
        ("validate", C.c_int),
        ("mem_limit", C.c_uint64),
        ("peel_blocks", C.c_uint32),
        ("work_chunk", C.c_uint32),
        ("watchdog", C.c_uint64),
        ("flags", C.c_uint32),
        ("alloc", C.c_void_p),
        ("free", C.c_void_p),
        ("alloc_user", C.c_void_p),
    ]


class Info(C.Structure):
    _fields_ = [
        ("n", C.c_uint32), ("r", C.c_uint32), ("s", C.c_uint32),
        ("m", C.c_uint64),
        ("n_r", C.c_uint64),
        ("n_s", C.c_uint64),
        ("k", C.c_uint32),
        ("rounds", C.c_uint32),
        ("n_int", C.c_uint64),
        ("visits", C.c_uint64),
        ("decrements", C.c_uint64),
        ("links", C.c_uint64),
        ("link_calls", C.c_uint64),
        ("unites", C.c_uint64),
        ("bucket_scans", C.c_uint64),
        ("max_outdeg", C.c_uint32),
        ("orient_rounds", C.c_uint32),
        ("ms_prep", C.c_float),
        ("ms_count", C.c_float),
        ("ms_peel", C.c_float),
        ("ms_tree", C.c_float),
        ("ms_count_kernel", C.c_float),
        ("ms_peel_kernel", C.c_float),
        ("device_bytes", C.c_uint64),
        ("hier_te", C.c_uint32),
        ("ms_hier", C.c_float),
        ("hier_visits", C.c_uint64),
        ("grid_retries", C.c_uint32),
        ("cascades", C.c_uint64),
        ("cas_retries", C.c_uint64),
        ("device_peak", C.c_uint64),
        ("approx_delta", C.c_double),
        ("round_cap", C.c_uint32),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class Nucleus(C.Structure):
    _fields_ = [
        ("node", C.c_uint64), ("min_leaf", C.c_uint64), ("n_rcliques", C.c_uint64),
        ("n_vertices", C.c_uint64), ("n_edges", C.c_uint64), ("vert_off", C.c_uint64),
        ("level", C.c_uint32), ("reserved", C.c_uint32),
    ]


NUCLEUS_DTYPE = np.dtype([("node", "<u8"), ("min_leaf", "<u8"), ("n_rcliques", "<u8"),
                          ("n_vertices", "<u8"), ("n_edges", "<u8"), ("vert_off", "<u8"),
                          ("level", "<u4"), ("reserved", "<u4")])


class Schedule(C.Structure):
    _fields_ = [("r", C.c_uint32), ("s", C.c_uint32), ("n_r_max", C.c_uint64),
                ("peel_blocks", C.c_uint32), ("kind", C.c_uint32)]


ND_SCHED_SINGLE = 0
ND_SCHED_BATCH = 1
SCHEDULES_PATH = os.path.join(_HERE, "schedules.json")


def load_schedules(path: str = SCHEDULES_PATH) -> list[dict]:
    """The autotuned schedule table (entries {kind, r, s, n_r_max,
    peel_blocks}), or [] if none has been written."""
    import json
    if not os.path.exists(path):
        return []
    with open(path) as f:
        return json.load(f)["entries"]


class GraphDesc(C.Structure):
    _fields_ = [
        ("n", C.c_uint32), ("r", C.c_uint32), ("s", C.c_uint32),
        ("nnz", C.c_uint64),
        ("row_ptr", C.c_void_p),
        ("col", C.c_void_p),
    ]


class GraphResult(C.Structure):
    _fields_ = [
        ("status", C.c_int),
        ("k", C.c_uint32),
        ("n_r", C.c_uint64),
        ("n_s", C.c_uint64),
        ("n_int", C.c_uint64),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class ServerOptions(C.Structure):
    _fields_ = [
        ("device", C.c_int),
        ("workers", C.c_uint32),
        ("max_batch", C.c_uint32),
        ("mem_budget", C.c_uint64),
        ("validate", C.c_int),
    ]


class RequestInfo(C.Structure):
    _fields_ = [
        ("status", C.c_int),
        ("done", C.c_int),
        ("k", C.c_uint32),
        ("n_r", C.c_uint64), ("n_s", C.c_uint64), ("n_int", C.c_uint64),
        ("workspace", C.c_uint64),
        ("result_bytes", C.c_uint64),
        ("t_submit_ms", C.c_double),
        ("t_start_ms", C.c_double),
        ("t_done_ms", C.c_double),
        ("batch_size", C.c_uint32),
        ("worker", C.c_uint32),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class ServerStats(C.Structure):
    _fields_ = [(name, C.c_uint64) for name in (
        "submitted", "completed", "failed", "cancelled", "batches", "max_batch_seen",
        "waiting", "running", "result_bytes", "workspace_share", "result_share", "overlapped")] + \
        [(name, C.c_double) for name in ("device_batch_ms", "device_busy_ms", "device_overlap_ms")]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


# nd_options.alloc / nd_options.free (include/nucleus.h)
ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)


def torch_allocator(device: int):
    """(alloc, free) callbacks that take the library's device workspace from
    PyTorch's caching allocator on ``device``, ordered on the stream the
    library passes (so torch accounts for the memory and reuses it)."""
    def alloc(nbytes, stream, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device, int(stream or 0))
        except Exception:   # reported by the library as ND_E_OOM
            return None

    def free(ptr, nbytes, stream, user):
        try:
            torch.cuda.caching_allocator_delete(int(ptr))
        except Exception:   # interpreter shutdown: torch is already gone
            pass
    return ALLOC_FN(alloc), FREE_FN(free)


class NucleusError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"nucleus error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Load ``libnucleus.so``; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build the HIP library first "
            "(python -m paper_2306_08623_amd.build)")
    lib = C.CDLL(path)
    vp = C.c_void_p
    u64p = C.POINTER(C.c_uint64)
    u32p = C.POINTER(C.c_uint32)
    lib.nd_create.argtypes = [C.POINTER(vp), C.POINTER(Options)]
    lib.nd_create.restype = C.c_int
    lib.nd_destroy.argtypes = [vp]
    lib.nd_destroy.restype = None
    lib.nd_load_csr.argtypes = [vp, C.c_uint32, C.c_uint64, vp, vp, C.c_int]
    lib.nd_load_csr.restype = C.c_int
    lib.nd_set_schedule.argtypes = [vp, C.POINTER(Schedule), C.c_uint32]
    lib.nd_set_schedule.restype = C.c_int
    lib.nd_set_rs.argtypes = [vp, C.c_uint32, C.c_uint32]
    lib.nd_set_rs.restype = C.c_int
    lib.nd_decompose.argtypes = [vp]
    lib.nd_decompose.restype = C.c_int
    lib.nd_sync.argtypes = [vp]
    lib.nd_sync.restype = C.c_int
    lib.nd_get_info.argtypes = [vp, C.POINTER(Info)]
    lib.nd_get_info.restype = C.c_int
    for name in ("nd_get_rcliques", "nd_get_counts", "nd_get_coreness", "nd_get_peel_rounds"):
        getattr(lib, name).argtypes = [vp, vp, C.c_int]
        getattr(lib, name).restype = C.c_int
    lib.nd_get_tree.argtypes = [vp, vp, vp, C.c_int]
    lib.nd_get_tree.restype = C.c_int
    lib.nd_batch_decompose.argtypes = [vp, C.c_uint32, C.POINTER(GraphDesc), C.c_int,
                                       C.POINTER(GraphResult)]
    lib.nd_batch_decompose.restype = C.c_int
    lib.nd_batch_get.argtypes = [vp, C.c_uint32, vp, vp, vp, vp, vp, C.c_int]
    lib.nd_batch_get.restype = C.c_int
    lib.nd_estimate_footprint.argtypes = [C.POINTER(GraphDesc), C.c_int, C.POINTER(C.c_uint64),
                                          C.POINTER(C.c_uint64)]
    lib.nd_estimate_footprint.restype = C.c_int
    lib.nd_server_create.argtypes = [C.POINTER(vp), C.POINTER(ServerOptions)]
    lib.nd_server_create.restype = C.c_int
    lib.nd_server_destroy.argtypes = [vp]
    lib.nd_server_destroy.restype = None
    lib.nd_server_submit.argtypes = [vp, C.POINTER(GraphDesc), C.c_int, C.POINTER(C.c_uint64)]
    lib.nd_server_submit.restype = C.c_int
    lib.nd_server_poll.argtypes = [vp, C.c_uint64, C.POINTER(RequestInfo)]
    lib.nd_server_poll.restype = C.c_int
    lib.nd_server_wait.argtypes = [vp, C.c_uint64, C.c_double, C.POINTER(RequestInfo)]
    lib.nd_server_wait.restype = C.c_int
    lib.nd_server_get.argtypes = [vp, C.c_uint64, vp, vp, vp, vp, vp, C.c_int]
    lib.nd_server_get.restype = C.c_int
    lib.nd_server_release.argtypes = [vp, C.c_uint64]
    lib.nd_server_release.restype = C.c_int
    lib.nd_server_cancel.argtypes = [vp, C.c_uint64]
    lib.nd_server_cancel.restype = C.c_int
    lib.nd_server_get_stats.argtypes = [vp, C.POINTER(ServerStats)]
    lib.nd_server_get_stats.restype = C.c_int
    lib.nd_server_last_error.argtypes = [vp]
    lib.nd_server_last_error.restype = C.c_char_p
    lib.nd_decompose_noalloc.argtypes = [C.c_int, vp, C.c_uint32, C.c_uint64, vp, vp,
                                         C.c_uint32, C.c_uint32, C.c_uint64, vp, vp, vp,
                                         C.POINTER(Info)]
    lib.nd_decompose_noalloc.restype = C.c_int
    lib.nd_set_approx.argtypes = [vp, C.c_double]
    lib.nd_set_approx.restype = C.c_int
    lib.nd_cut.argtypes = [vp, C.c_uint32, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]
    lib.nd_cut.restype = C.c_int
    lib.nd_get_cut.argtypes = [vp, vp, vp, vp, C.c_int]
    lib.nd_get_cut.restype = C.c_int
    lib.nd_status_str.argtypes = [C.c_int]
    lib.nd_status_str.restype = C.c_char_p
    lib.nd_last_error.argtypes = [vp]
    lib.nd_last_error.restype = C.c_char_p
    del u64p, u32p
    _lib = lib
    return lib


def _ptr(a) -> tuple[int, int]:
    """(address, memory kind) of a numpy array or a torch tensor."""
    if isinstance(a, np.ndarray):
        return a.ctypes.data, ND_MEM_HOST
    if hasattr(a, "data_ptr") and hasattr(a, "is_cuda"):
        return a.data_ptr(), (ND_MEM_DEVICE if a.is_cuda else ND_MEM_HOST)
    raise TypeError(f"unsupported array type {type(a)}")


def _current_stream(device: int):
    if torch is None or not torch.cuda.is_available():
        return None
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


@dataclass
class Result:
    r: int
    s: int
    info: dict
    rcliques: np.ndarray   # uint32 [n_r, r]
    counts: np.ndarray     # uint32 [n_r]
    coreness: np.ndarray   # uint32 [n_r]
    parent: np.ndarray     # uint64 [n_r + n_int]
    level: np.ndarray      # uint32 [n_int]


class Context:
    """One library context (device buffers, stream, last result)."""

    def __init__(self, device: int = 0, stream=None, validate: bool = True, mem_limit: int = 0,
                 peel_blocks: int = 0, work_chunk: int = 0, watchdog: int = 0,
                 use_torch_stream: bool = True, progress: bool = False,
                 hierarchy: str = "auto", allocator: str = "hip", count_global: bool = False,
                 schedule="tuned"):
        """allocator: "hip" (the library's own hipMalloc) or "torch" (PyTorch's
        caching allocator through the nd_options callbacks). schedule:
        "tuned" (the autotuned table in schedules.json, if present), "none",
        or a list of entries {kind, r, s, n_r_max, peel_blocks}."""
        self.lib = load_library()
        opt = Options()
        opt.device = device
        if stream is None and use_torch_stream:
            stream = _current_stream(device)
        opt.hip_stream = stream if stream is None or isinstance(stream, C.c_void_p) else C.c_void_p(stream)
        opt.validate = 1 if validate else 0
        opt.mem_limit = mem_limit
        opt.peel_blocks = peel_blocks
        opt.work_chunk = work_chunk
        opt.watchdog = watchdog
        opt.flags = (ND_FLAG_PROGRESS if progress else 0) | \
            {"auto": 0, "el": ND_FLAG_HIER_EL, "te": ND_FLAG_HIER_TE}[hierarchy] | \
            (ND_FLAG_COUNT_GLOBAL if count_global else 0)
        self._alloc_cbs = None
        if allocator == "torch":
            if torch is None or not torch.cuda.is_available():
                raise RuntimeError("allocator='torch' needs PyTorch with a GPU")
            self._alloc_cbs = torch_allocator(device)
            opt.alloc = C.cast(self._alloc_cbs[0], C.c_void_p)
            opt.free = C.cast(self._alloc_cbs[1], C.c_void_p)
        elif allocator != "hip":
            raise ValueError(f"unknown allocator {allocator!r}")
        h = C.c_void_p()
        st = self.lib.nd_create(C.byref(h), C.byref(opt))
        if st != ND_OK:
            msg = self.lib.nd_last_error(None).decode() or self.lib.nd_status_str(st).decode()
            raise NucleusError(st, msg)
        self.h = h
        self.r = self.s = 0
        entries = load_schedules() if schedule == "tuned" else \
            ([] if schedule == "none" else list(schedule))
        if entries:
            self.set_schedule(entries)

    def set_schedule(self, entries: list[dict]):
        """nd_set_schedule with a list of {kind, r, s, n_r_max, peel_blocks}."""
        tab = (Schedule * max(1, len(entries)))()
        for i, e in enumerate(entries):
            tab[i] = Schedule(int(e["r"]), int(e["s"]), int(e["n_r_max"]),
                              int(e["peel_blocks"]), int(e.get("kind", ND_SCHED_SINGLE)))
        self._check(self.lib.nd_set_schedule(self.h, tab, len(entries)))

    # -- error handling ----------------------------------------------------
    def _check(self, st: int):
        if st != ND_OK:
            msg = self.lib.nd_last_error(self.h).decode() or self.lib.nd_status_str(st).decode()
            raise NucleusError(st, msg)

    def close(self):
        if getattr(self, "h", None):
            self.lib.nd_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- C ABI mirrors -----------------------------------------------------
    def nd_load_csr(self, n: int, row_ptr, col):
        rp_ptr, kind = _ptr(row_ptr)
        col_ptr, kind2 = _ptr(col)
        if kind != kind2:
            raise ValueError("row_ptr and col must live in the same memory")
        nnz = int(row_ptr[-1]) if kind == ND_MEM_HOST else int(col.numel())
        self._keep = (row_ptr, col)
        self._check(self.lib.nd_load_csr(self.h, n, nnz, rp_ptr, col_ptr, kind))

    def load_csr(self, csr):
        rp = np.ascontiguousarray(csr.row_ptr, dtype=np.uint64)
        col = np.ascontiguousarray(csr.col, dtype=np.uint32)
        if col.size == 0:
            col = np.zeros(1, dtype=np.uint32)
            self._keep = (rp, col)
            self._check(self.lib.nd_load_csr(self.h, csr.n, 0, rp.ctypes.data, col.ctypes.data,
                                             ND_MEM_HOST))
            return
        self._keep = (rp, col)
        self._check(self.lib.nd_load_csr(self.h, csr.n, int(rp[-1]), rp.ctypes.data,
                                         col.ctypes.data, ND_MEM_HOST))

    def nd_set_rs(self, r: int, s: int):
        self._check(self.lib.nd_set_rs(self.h, r, s))
        self.r, self.s = r, s

    def nd_decompose(self):
        self._check(self.lib.nd_decompose(self.h))

    def nd_sync(self):
        self._check(self.lib.nd_sync(self.h))

    def nd_get_info(self) -> dict:
        info = Info()
        self._check(self.lib.nd_get_info(self.h, C.byref(info)))
        return info.as_dict()

    def nd_get_rcliques(self) -> np.ndarray:
        info = self.nd_get_info()
        out = np.zeros((info["n_r"], info["r"]), dtype=np.uint32)
        self._check(self.lib.nd_get_rcliques(self.h, out.ctypes.data if out.size else None,
                                             ND_MEM_HOST))
        return out

    def nd_get_counts(self) -> np.ndarray:
        n_r = self.nd_get_info()["n_r"]
        out = np.zeros(n_r, dtype=np.uint32)
        self._check(self.lib.nd_get_counts(self.h, out.ctypes.data if out.size else None,
                                           ND_MEM_HOST))
        return out

    def nd_get_coreness(self, out=None):
        n_r = self.nd_get_info()["n_r"]
        if out is None:
            out = np.zeros(n_r, dtype=np.uint32)
        p, kind = _ptr(out)
        self._check(self.lib.nd_get_coreness(self.h, p if n_r else None, kind))
        return out

    def nd_get_peel_rounds(self) -> np.ndarray:
        n_r = self.nd_get_info()["n_r"]
        out = np.zeros(n_r, dtype=np.uint32)
        self._check(self.lib.nd_get_peel_rounds(self.h, out.ctypes.data if out.size else None,
                                                ND_MEM_HOST))
        return out

    def nd_get_tree(self) -> tuple[np.ndarray, np.ndarray]:
        info = self.nd_get_info()
        n_r, n_int = info["n_r"], info["n_int"]
        parent = np.zeros(n_r + n_int, dtype=np.uint64)
        level = np.zeros(n_int, dtype=np.uint32)
        self._check(self.lib.nd_get_tree(self.h, parent.ctypes.data if parent.size else None,
                                         level.ctypes.data if level.size else None, ND_MEM_HOST))
        return parent, level

    def nd_set_approx(self, delta: float):
        """delta > 0: approximate decomposition (Algorithm 2); 0: exact."""
        self._check(self.lib.nd_set_approx(self.h, float(delta)))

    def decompose_approx(self, csr, r: int, s: int, delta: float) -> Result:
        """Approximate core numbers and their hierarchy; the context returns
        to exact peeling afterwards."""
        self.nd_set_approx(delta)
        try:
            return self.decompose(csr, r, s)
        finally:
            self.nd_set_approx(0.0)

    def nd_cut(self, c: int) -> tuple[int, int]:
        """Cut the last decomposition's tree at level c: (nuclei, vertices)."""
        nn, nv = C.c_uint64(), C.c_uint64()
        self._check(self.lib.nd_cut(self.h, c, C.byref(nn), C.byref(nv)))
        return nn.value, nv.value

    def cut(self, c: int) -> dict:
        """The c-(r,s) nuclei: a structured array (node, min_leaf, n_rcliques,
        n_vertices, n_edges, vert_off, level), their vertex lists and every
        r-clique's nucleus (-1 = none), read back to the host."""
        nn, nv = self.nd_cut(c)
        n_r = self.nd_get_info()["n_r"]
        nuc = np.zeros(nn, dtype=NUCLEUS_DTYPE)
        verts = np.zeros(nv, dtype=np.uint32)
        leaf = np.zeros(n_r, dtype=np.uint32)

        def p(a):
            return a.ctypes.data if a.size else None
        self._check(self.lib.nd_get_cut(self.h, p(nuc), p(verts), p(leaf), ND_MEM_HOST))
        leaf_i = leaf.astype(np.int64)
        leaf_i[leaf == 0xFFFFFFFF] = -1
        return {"nuclei": nuc, "verts": verts, "leaf_nucleus": leaf_i}

    def nd_batch_decompose(self, descs, results, where: int = ND_MEM_HOST):
        """descs / results: ctypes arrays of GraphDesc / GraphResult."""
        self._check(self.lib.nd_batch_decompose(self.h, len(descs), descs, where, results))

    def nd_batch_get(self, i: int, res: GraphResult, r: int) -> Result:
        n_r, n_int = res.n_r, res.n_int
        rcl = np.zeros((n_r, r), dtype=np.uint32)
        counts = np.zeros(n_r, dtype=np.uint32)
        core = np.zeros(n_r, dtype=np.uint32)
        parent = np.zeros(n_r + n_int, dtype=np.uint64)
        level = np.zeros(n_int, dtype=np.uint32)

        def p(a):
            return a.ctypes.data if a.size else None
        self._check(self.lib.nd_batch_get(self.h, i, p(rcl), p(counts), p(core), p(parent),
                                          p(level), ND_MEM_HOST))
        return Result(r=r, s=0, info=res.as_dict(), rcliques=rcl, counts=counts, coreness=core,
                      parent=parent, level=level)

    def decompose_batch(self, graphs, where: int = ND_MEM_HOST) -> list[Result]:
        """graphs: sequence of (csr, r, s) with host CSR arrays, or, for
        ``where=ND_MEM_DEVICE``, of (n, row_ptr, col, r, s) with device
        tensors. Returns every graph's Result, read back to the host."""
        G = len(graphs)
        descs = (GraphDesc * max(G, 1))()
        results = (GraphResult * max(G, 1))()
        keep = []
        rs = []
        for i, g in enumerate(graphs):
            if where == ND_MEM_HOST:
                csr, r, s = g
                rp = np.ascontiguousarray(csr.row_ptr, dtype=np.uint64)
                col = np.ascontiguousarray(csr.col, dtype=np.uint32)
                if col.size == 0:
                    col = np.zeros(1, dtype=np.uint32)
                keep.append((rp, col))
                descs[i] = GraphDesc(csr.n, r, s, int(rp[-1]), rp.ctypes.data, col.ctypes.data)
            else:
                n, rp, col, r, s = g
                keep.append((rp, col))
                descs[i] = GraphDesc(n, r, s, int(col.numel()), rp.data_ptr(), col.data_ptr())
            rs.append((r, s))
        self._check(self.lib.nd_batch_decompose(self.h, G, descs, where, results))
        out = []
        for i in range(G):
            res = self.nd_batch_get(i, results[i], rs[i][0])
            res.s = rs[i][1]
            out.append(res)
        return out

    # -- convenience --------------------------------------------------------
    def decompose(self, csr, r: int, s: int) -> Result:
        self.load_csr(csr)
        self.nd_set_rs(r, s)
        self.nd_decompose()
        return self.result()

    def result(self) -> Result:
        info = self.nd_get_info()
        parent, level = self.nd_get_tree()
        return Result(r=info["r"], s=info["s"], info=info, rcliques=self.nd_get_rcliques(),
                      counts=self.nd_get_counts(), coreness=self.nd_get_coreness(),
                      parent=parent, level=level)


def decompose(csr, r: int, s: int, device: int = 0, **opts) -> Result:
    with Context(device=device, **opts) as ctx:
        return ctx.decompose(csr, r, s)


def decompose_noalloc(n: int, row_ptr, col, r: int, s: int, coreness, parent, level,
                      device: int = 0, stream=None) -> dict:
    """nd_decompose_noalloc: device tensors in (CSR) and out (coreness
    uint32[cap], parent uint64[2 cap], level uint32[cap]); the library
    allocates no device memory. Returns the run's nd_info."""
    lib = load_library()
    if stream is None:
        stream = _current_stream(device)
    cap = int(coreness.numel())
    if int(parent.numel()) < 2 * cap or int(level.numel()) < cap:
        raise ValueError("parent needs 2 * cap entries and level cap entries")
    info = Info()
    st = lib.nd_decompose_noalloc(device, stream, n, int(col.numel()), row_ptr.data_ptr(),
                                  col.data_ptr(), r, s, cap, coreness.data_ptr(),
                                  parent.data_ptr(), level.data_ptr(), C.byref(info))
    if st != ND_OK:
        msg = lib.nd_last_error(None).decode() or lib.nd_status_str(st).decode()
        raise NucleusError(st, msg)
    return info.as_dict()


def _host_desc(csr, r: int, s: int):
    rp = np.ascontiguousarray(csr.row_ptr, dtype=np.uint64)
    col = np.ascontiguousarray(csr.col, dtype=np.uint32)
    if col.size == 0:
        col = np.zeros(1, dtype=np.uint32)
    return GraphDesc(csr.n, r, s, int(rp[-1]), rp.ctypes.data, col.ctypes.data), (rp, col)


def estimate_footprint(csr, r: int, s: int) -> tuple[int, int]:
    """(workspace bytes, result bytes) the library estimates for one graph."""
    lib = load_library()
    d, keep = _host_desc(csr, r, s)
    ws, res = C.c_uint64(), C.c_uint64()
    st = lib.nd_estimate_footprint(C.byref(d), ND_MEM_HOST, C.byref(ws), C.byref(res))
    if st != ND_OK:
        raise NucleusError(st, lib.nd_status_str(st).decode())
    del keep
    return ws.value, res.value


class Server:
    """Request loop with continuous batching (nd_server_*)."""

    def __init__(self, device: int = 0, workers: int = 0, max_batch: int = 0,
                 mem_budget: int = 0, validate: bool = True):
        self.lib = load_library()
        opt = ServerOptions(device, workers, max_batch, mem_budget, 1 if validate else 0)
        h = C.c_void_p()
        st = self.lib.nd_server_create(C.byref(h), C.byref(opt))
        if st != ND_OK:
            raise NucleusError(st, self.lib.nd_status_str(st).decode())
        self.h = h

    def _check(self, st: int):
        if st != ND_OK:
            msg = self.lib.nd_server_last_error(self.h).decode() or \
                self.lib.nd_status_str(st).decode()
            raise NucleusError(st, msg)

    def close(self):
        if getattr(self, "h", None):
            self.lib.nd_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, csr, r: int, s: int) -> int:
        d, keep = _host_desc(csr, r, s)
        t = C.c_uint64()
        self._check(self.lib.nd_server_submit(self.h, C.byref(d), ND_MEM_HOST, C.byref(t)))
        del keep
        return t.value

    def submit_device(self, n: int, row_ptr, col, r: int, s: int, nnz: int | None = None) -> int:
        """row_ptr / col: device tensors; nnz defaults to col.numel()."""
        nnz = int(col.numel()) if nnz is None else int(nnz)
        d = GraphDesc(n, r, s, nnz, row_ptr.data_ptr(), col.data_ptr())
        t = C.c_uint64()
        self._check(self.lib.nd_server_submit(self.h, C.byref(d), ND_MEM_DEVICE, C.byref(t)))
        return t.value

    def poll(self, ticket: int) -> dict:
        info = RequestInfo()
        self._check(self.lib.nd_server_poll(self.h, ticket, C.byref(info)))
        return info.as_dict()

    def wait(self, ticket: int, timeout_ms: float = -1.0) -> dict:
        info = RequestInfo()
        self._check(self.lib.nd_server_wait(self.h, ticket, timeout_ms, C.byref(info)))
        return info.as_dict()

    def get(self, ticket: int, r: int) -> Result:
        info = self.wait(ticket)
        n_r, n_int = info["n_r"], info["n_int"]
        rcl = np.zeros((n_r, r), dtype=np.uint32)
        counts = np.zeros(n_r, dtype=np.uint32)
        core = np.zeros(n_r, dtype=np.uint32)
        parent = np.zeros(n_r + n_int, dtype=np.uint64)
        level = np.zeros(n_int, dtype=np.uint32)

        def p(a):
            return a.ctypes.data if a.size else None
        self._check(self.lib.nd_server_get(self.h, ticket, p(rcl), p(counts), p(core),
                                           p(parent), p(level), ND_MEM_HOST))
        return Result(r=r, s=0, info=info, rcliques=rcl, counts=counts, coreness=core,
                      parent=parent, level=level)

    def release(self, ticket: int):
        self._check(self.lib.nd_server_release(self.h, ticket))

    def cancel(self, ticket: int):
        self._check(self.lib.nd_server_cancel(self.h, ticket))

    def stats(self) -> dict:
        out = ServerStats()
        self._check(self.lib.nd_server_get_stats(self.h, C.byref(out)))
        return out.as_dict()
