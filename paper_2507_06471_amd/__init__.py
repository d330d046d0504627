"""Python binding of the MI355X Louvain library (``liblv.so``, C ABI in include/lv.h).

Argument marshalling only: every step of the method runs in the HIP library.
The ``lv_*`` functions mirror the C entry points one to one; ``Graph``,
``louvain``, ``lpa`` and ``modularity`` are small conveniences over them.
Device buffers may be passed as torch CUDA tensors (PyTorch is used for device
memory and streams only); host buffers as numpy arrays.

There is no fallback: if ``liblv.so`` is missing or fails to load, every call
raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblv.so")

LV_OK = 0
STATUS_NAMES = {
    0: "LV_OK", 1: "LV_E_ARG", 2: "LV_E_CSR", 3: "LV_E_ASYMMETRIC", 4: "LV_E_WEIGHT",
    5: "LV_E_OVERFLOW", 6: "LV_E_NOMEM", 7: "LV_E_HIP", 8: "LV_E_BUSY", 9: "LV_E_TOO_LARGE",
    10: "LV_E_CANCELLED", 11: "LV_E_STATE", 12: "LV_E_NOT_FOUND",
}
LV_MEM_HOST, LV_MEM_DEVICE = 0, 1
LV_VALIDATE = 1
LV_KEEP_ORDER = 2
LV_EDGES_NO_LOOPS = 4
LV_EDGES_SIMPLE = 8
LV_NO_ENTRY_CACHE = 16
LV_TIMING = 1
LV_KEEP_GRAPHS = 2
LV_NO_HIPGRAPH = 4
LV_AUTOTUNE = 8
LV_PRUNE = 16
LV_ASYNC = 32
LV_NO_CACHE = 64
KERNEL_SLOTS = 26
# kernel slot -> name (slot = 2*(class-1) + first-sweep flag; then the bucketed
# hub scatter pass, whose partition workgroups are timed as "hub"; the commit
# with pair refresh and sweep control; the entry cache's refresh; the fused
# persistent kernel of the classes below the hub class)
KERNEL_NAMES = [f"{c}{'/first' if f else ''}"
                for c in ("l4", "l8", "l32", "l128", "l256", "l512", "l1k", "l2k", "l3k", "l8k", "hub")
                for f in (0, 1)] + ["hub/scatter", "commit", "cache/refresh", "fused"]

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_vp = ctypes.c_void_p


class lv_tuning(ctypes.Structure):
    _fields_ = [("sub_max", ctypes.c_int32), ("wave_max", ctypes.c_int32),
                ("block_max", ctypes.c_int32), ("part_keys", ctypes.c_int32),
                ("part_slots", ctypes.c_int32), ("hub_mode", ctypes.c_int32),
                ("hub_chunk", ctypes.c_int32), ("order_min", ctypes.c_int32),
                ("agg_sort", ctypes.c_int32), ("cache_pct", ctypes.c_int32), ("fused", ctypes.c_int32),
                ("table_pct", ctypes.c_int32)]


class lv_params(ctypes.Structure):
    _fields_ = [("max_sweeps", ctypes.c_int32), ("max_levels", ctypes.c_int32),
                ("lpa_threshold", ctypes.c_int64), ("flags", ctypes.c_uint32),
                ("tuning", ctypes.POINTER(lv_tuning))]


class lv_level_info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_next", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("sweeps", ctypes.c_int32), ("accepted", ctypes.c_int32),
                ("q_start", ctypes.c_int64), ("q_end", ctypes.c_int64),
                ("move_ms", ctypes.c_double), ("sweep_ms", ctypes.c_double),
                ("renumber_ms", ctypes.c_double), ("aggregate_ms", ctypes.c_double),
                ("move_launches", ctypes.c_int64), ("move_bytes", ctypes.c_int64),
                ("kern_ms", ctypes.c_double * KERNEL_SLOTS), ("kern_launches", ctypes.c_int64 * KERNEL_SLOTS),
                ("kern_bytes", ctypes.c_int64 * KERNEL_SLOTS), ("cached_sweeps", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("refreshed_entries", ctypes.c_int64)]

    def as_dict(self) -> dict:
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if name.startswith("kern_") else v
        return out


class lv_server_config(ctypes.Structure):
    _fields_ = [("mem_budget", ctypes.c_int64), ("max_jobs", ctypes.c_int32), ("max_sweeps", ctypes.c_int32),
                ("max_levels", ctypes.c_int32), ("flags", ctypes.c_uint32), ("tuning", ctypes.POINTER(lv_tuning))]


class lv_job_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("steps", ctypes.c_int32), ("q_int", ctypes.c_int64), ("m", ctypes.c_int64), ("q", ctypes.c_double),
                ("entries", ctypes.c_int64), ("queue_ms", ctypes.c_double), ("total_ms", ctypes.c_double)]


class lv_server_stats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in ("submitted", "completed", "steps", "max_batch", "entries", "queued",
                                              "in_flight", "mem_in_use", "mem_budget")]


JOB_QUEUED, JOB_RUNNING, JOB_DONE = 0, 1, 2

# name -> (restype, argtypes); every entry point declared in include/lv.h
SIGNATURES = {
    "lv_params_default": (None, [ctypes.POINTER(lv_params)]),
    "lv_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "lv_last_error": (ctypes.c_char_p, []),
    "lv_graph_create_csr": (ctypes.c_int, [ctypes.c_int32, _vp, _vp, _vp, ctypes.c_int, ctypes.c_uint32, _vp,
                                           ctypes.POINTER(_vp)]),
    "lv_graph_create_batch": (ctypes.c_int, [ctypes.c_int32, _vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_uint32,
                                             _vp, ctypes.POINTER(_vp)]),
    "lv_graph_destroy": (ctypes.c_int, [_vp]),
    "lv_autotune": (ctypes.c_int, [_vp, ctypes.POINTER(lv_params), ctypes.POINTER(lv_tuning),
                                   ctypes.POINTER(ctypes.c_double)]),
    "lv_graph_count": (ctypes.c_int, [_vp, _i32p]),
    "lv_graph_info": (ctypes.c_int, [_vp, _i32p, _i64p, _i64p]),
    "lv_louvain": (ctypes.c_int, [_vp, ctypes.POINTER(lv_params), ctypes.POINTER(_vp)]),
    "lv_result_num_levels": (ctypes.c_int, [_vp, _i32p, _i32p]),
    "lv_result_level_info": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(lv_level_info)]),
    "lv_result_level_moves": (ctypes.c_int, [_vp, ctypes.c_int32, _i64p, ctypes.c_int32]),
    "lv_result_level_labels": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, ctypes.c_int]),
    "lv_result_level_graph": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _vp, _vp, _i64p, ctypes.c_int]),
    "lv_result_final_labels": (ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    "lv_result_modularity": (ctypes.c_int, [_vp, _i64p, _i64p, ctypes.POINTER(ctypes.c_double)]),
    "lv_result_destroy": (ctypes.c_int, [_vp]),
    "lv_result_graph_num_levels": (ctypes.c_int, [_vp, ctypes.c_int32, _i32p, _i32p]),
    "lv_result_graph_level_info": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32,
                                                  ctypes.POINTER(lv_level_info)]),
    "lv_result_graph_level_moves": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, _i64p, ctypes.c_int32]),
    "lv_result_graph_level_labels": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, _vp, ctypes.c_int]),
    "lv_result_graph_final_labels": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, ctypes.c_int]),
    "lv_result_graph_modularity": (ctypes.c_int, [_vp, ctypes.c_int32, _i64p, _i64p,
                                                  ctypes.POINTER(ctypes.c_double)]),
    "lv_lpa": (ctypes.c_int, [_vp, ctypes.POINTER(lv_params), _vp, ctypes.c_int,
                              ctypes.POINTER(lv_level_info), _i64p, ctypes.c_int32]),
    "lv_result_final_labels_all": (ctypes.c_int, [_vp, _vp, ctypes.c_int]),
    "lv_result_modularity_all": (ctypes.c_int, [_vp, _i64p, _i64p, ctypes.POINTER(ctypes.c_double)]),
    "lv_lpa_batch": (ctypes.c_int, [_vp, ctypes.POINTER(lv_params), _vp, ctypes.c_int, _i32p, _i64p, _i64p,
                                    _i64p, ctypes.c_int32]),
    "lv_server_create": (ctypes.c_int, [ctypes.POINTER(lv_server_config), ctypes.POINTER(_vp)]),
    "lv_server_submit": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _vp, _vp, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_uint64)]),
    "lv_server_poll": (ctypes.c_int, [_vp, ctypes.c_uint64, _i32p]),
    "lv_server_wait": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.c_int64]),
    "lv_server_result": (ctypes.c_int, [_vp, ctypes.c_uint64, _vp, ctypes.c_int, ctypes.POINTER(lv_job_info)]),
    "lv_server_cancel": (ctypes.c_int, [_vp, ctypes.c_uint64]),
    "lv_server_stats_get": (ctypes.c_int, [_vp, ctypes.POINTER(lv_server_stats)]),
    "lv_server_destroy": (ctypes.c_int, [_vp]),
    "lv_modularity": (ctypes.c_int, [_vp, _vp, ctypes.c_int, _i64p, _i64p, ctypes.POINTER(ctypes.c_double)]),
    "lv_graph_create_edges": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, _vp, _vp, _vp, ctypes.c_int,
                                             ctypes.c_uint32, _vp, ctypes.POINTER(_vp)]),
    "lv_graph_csr": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i64p, ctypes.c_int]),
    "lv_probe_gather": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "lv_probe_copy": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "lv_modularity_noalloc": (ctypes.c_int, [_vp, _vp, _i64p, _i64p, ctypes.POINTER(ctypes.c_double)]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblv.so and declare its signatures.  Raises if it is missing.

    When PyTorch is installed it is imported first: its wheel ships its own HIP
    runtime under the same soname (libamdhip64.so.7), and loading torch first
    makes liblv bind to that one, so a process never holds two HIP runtimes
    (the second one would not see the GPU).  LV_NO_TORCH=1 skips this.
    """
    global _lib
    if _lib is None:
        if os.environ.get("LV_NO_TORCH") != "1":
            try:
                import torch  # noqa: F401
            except ImportError:
                pass
        if not os.path.exists(path):
            raise ImportError(f"{path} is not built; run paper_2507_06471_amd/build.py "
                              "(or __graft_entry__.build())")
        lib = ctypes.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class LvError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load_library()
        detail = lib.lv_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)} ({detail})")
        self.status = status


def _check(status: int, where: str):
    if status != LV_OK:
        raise LvError(status, where)


def _ptr(buf):
    """(address, memkind) of a numpy array or torch tensor (None -> (None, host))."""
    if buf is None:
        return None, LV_MEM_HOST
    if isinstance(buf, np.ndarray):
        assert buf.dtype == np.int32 and buf.flags.c_contiguous, "int32 contiguous arrays only"
        return buf.ctypes.data, LV_MEM_HOST
    # torch tensor
    import torch

    assert buf.dtype == torch.int32 and buf.is_contiguous(), "int32 contiguous tensors only"
    return buf.data_ptr(), (LV_MEM_DEVICE if buf.is_cuda else LV_MEM_HOST)


def make_params(max_sweeps: int = 20, max_levels: int = 32, lpa_threshold: int = 0, flags: int = 0,
                tuning: Optional[dict] = None):
    p = lv_params()
    load_library().lv_params_default(ctypes.byref(p))
    p.max_sweeps, p.max_levels, p.lpa_threshold, p.flags = max_sweeps, max_levels, lpa_threshold, flags
    keep = None
    if tuning:
        keep = lv_tuning(**tuning)
        p.tuning = ctypes.pointer(keep)
    return p, keep


class Graph:
    """Device-resident graph handle (lv_graph_create_csr / lv_graph_destroy)."""

    def __init__(self, n: int, offsets, indices, weights=None, validate: bool = True, stream: int = 0,
                 keep_order: bool = False, entry_cache: bool = True):
        lib = load_library()
        po, ko = _ptr(offsets)
        pi, ki = _ptr(indices)
        pw, kw = _ptr(weights)
        kinds = {ko, ki} | ({kw} if weights is not None else set())
        if len(kinds) != 1:
            raise ValueError("offsets, indices and weights must live in the same memory")
        h = _vp()
        flags = ((LV_VALIDATE if validate else 0) | (LV_KEEP_ORDER if keep_order else 0)
                 | (0 if entry_cache else LV_NO_ENTRY_CACHE))
        st = lib.lv_graph_create_csr(int(n), po, pi, pw, ko, flags, stream or None, ctypes.byref(h))
        _check(st, "lv_graph_create_csr")
        self._h = h
        self.n = int(n)
        nn, nnz, vol = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib.lv_graph_info(h, ctypes.byref(nn), ctypes.byref(nnz), ctypes.byref(vol)), "lv_graph_info")
        self.nnz = nnz.value
        self.volume = vol.value
        self.count = 1
        self.sizes = [self.n]

    @classmethod
    def batch(cls, graphs, validate: bool = True, keep_order: bool = False, entry_cache: bool = True):
        """Pack several ``graphgen.CSR``-like graphs into one handle
        (lv_graph_create_batch); graph g keeps its own vertex numbering."""
        lib = load_library()
        arrs = []
        for g in graphs:
            off = np.ascontiguousarray(g.offsets, dtype=np.int32)
            idx = np.ascontiguousarray(g.indices, dtype=np.int32)
            w = None if g.weights is None else np.ascontiguousarray(g.weights, dtype=np.int32)
            arrs.append((int(g.n), off, idx, w))
        cnt = len(arrs)
        ns = np.array([a[0] for a in arrs], dtype=np.int32)
        P = ctypes.c_void_p * cnt
        po = P(*[a[1].ctypes.data for a in arrs])
        pi = P(*[a[2].ctypes.data for a in arrs])
        pw = P(*[(a[3].ctypes.data if a[3] is not None else None) for a in arrs])
        h = _vp()
        st = lib.lv_graph_create_batch(cnt, ns.ctypes.data, ctypes.cast(po, _vp), ctypes.cast(pi, _vp),
                                       ctypes.cast(pw, _vp), LV_MEM_HOST,
                                       (LV_VALIDATE if validate else 0) | (LV_KEEP_ORDER if keep_order else 0)
                                       | (0 if entry_cache else LV_NO_ENTRY_CACHE), None, ctypes.byref(h))
        _check(st, "lv_graph_create_batch")
        self = cls.__new__(cls)
        self._h = h
        nn, nnz, vol = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib.lv_graph_info(h, ctypes.byref(nn), ctypes.byref(nnz), ctypes.byref(vol)), "lv_graph_info")
        c = ctypes.c_int32()
        _check(lib.lv_graph_count(h, ctypes.byref(c)), "lv_graph_count")
        self.n, self.nnz, self.volume, self.count = nn.value, nnz.value, None, c.value
        self.sizes = [int(x) for x in ns]
        return self

    @classmethod
    def from_csr(cls, g, validate: bool = True, device: bool = False, keep_order: bool = False,
                 entry_cache: bool = True):
        """From a ``graphgen.CSR``-like object (n, offsets, indices, weights)."""
        off = np.ascontiguousarray(g.offsets, dtype=np.int32)
        idx = np.ascontiguousarray(g.indices, dtype=np.int32)
        w = None if g.weights is None else np.ascontiguousarray(g.weights, dtype=np.int32)
        if device:
            import torch

            off, idx = torch.from_numpy(off).cuda(), torch.from_numpy(idx).cuda()
            w = None if w is None else torch.from_numpy(w).cuda()
            torch.cuda.synchronize()
        return cls(g.n, off, idx, w, validate=validate, keep_order=keep_order, entry_cache=entry_cache)

    @classmethod
    def from_edges(cls, n: int, src, dst, weights=None, drop_loops: bool = False, simple: bool = False,
                   keep_order: bool = False, entry_cache: bool = True):
        """lv_graph_create_edges: an undirected edge list (numpy or torch
        int32, all in the same memory), built into a CSR on the device."""
        lib = load_library()
        if isinstance(src, np.ndarray):
            src = np.ascontiguousarray(src, dtype=np.int32)
            dst = np.ascontiguousarray(dst, dtype=np.int32)
            weights = None if weights is None else np.ascontiguousarray(weights, dtype=np.int32)
        ps, ks = _ptr(src)
        pd, kd = _ptr(dst)
        pw, kw = _ptr(weights)
        kinds = {ks, kd} | ({kw} if weights is not None else set())
        if len(kinds) != 1:
            raise ValueError("src, dst and weights must live in the same memory")
        m = int(src.shape[0])
        flags = ((LV_EDGES_NO_LOOPS if drop_loops else 0) | (LV_EDGES_SIMPLE if simple else 0)
                 | (LV_KEEP_ORDER if keep_order else 0) | (0 if entry_cache else LV_NO_ENTRY_CACHE))
        h = _vp()
        _check(lib.lv_graph_create_edges(int(n), m, ps, pd, pw, ks, flags, None, ctypes.byref(h)),
               "lv_graph_create_edges")
        self = cls.__new__(cls)
        self._h = h
        nn, nnz, vol = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib.lv_graph_info(h, ctypes.byref(nn), ctypes.byref(nnz), ctypes.byref(vol)), "lv_graph_info")
        self.n, self.nnz, self.volume, self.count = nn.value, nnz.value, vol.value, 1
        self.sizes = [self.n]
        return self

    def csr(self):
        """lv_graph_csr: (offsets, indices, weights) in vertex-id order, host numpy."""
        lib = load_library()
        nnz = ctypes.c_int64()
        _check(lib.lv_graph_csr(self._h, None, None, None, ctypes.byref(nnz), LV_MEM_HOST), "lv_graph_csr")
        off = np.empty(self.n + 1, dtype=np.int32)
        idx = np.empty(max(nnz.value, 1), dtype=np.int32)
        w = np.empty(max(nnz.value, 1), dtype=np.int32)
        _check(lib.lv_graph_csr(self._h, off.ctypes.data, idx.ctypes.data, w.ctypes.data, ctypes.byref(nnz),
                                LV_MEM_HOST), "lv_graph_csr")
        return off, idx[:nnz.value], w[:nnz.value]

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            load_library().lv_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


@dataclass
class LevelResult:
    info: dict
    moves: List[int]
    labels: Optional[np.ndarray] = None
    graph: Optional[tuple] = None  # (offsets, indices, weights) when kept


@dataclass
class LouvainResult:
    q_int: int
    M: int
    q: float
    final_labels: np.ndarray
    levels: List[LevelResult] = field(default_factory=list)  # every attempted level

    @property
    def accepted(self) -> List[LevelResult]:
        return [lv for lv in self.levels if lv.info["accepted"]]


@dataclass
class FinalPartition:
    labels: np.ndarray     # packed like the handle: graph g's labels at its vertex offset
    q_int: np.ndarray      # [count]
    M: np.ndarray          # [count]
    q: np.ndarray          # [count]


def louvain_final(graph: Graph, max_sweeps: int = 20, max_levels: int = 32, tuning: Optional[dict] = None,
                  autotuned: bool = False, out=None, prune: bool = False, asynchronous: bool = False,
                  cache: bool = True) -> FinalPartition:
    """lv_louvain, then only the final labels and modularity of every graph
    (two calls, whatever the number of graphs); `out` may be a numpy or
    torch int32 buffer of the handle's total vertex count."""
    lib = load_library()
    p, _keep = make_params(max_sweeps, max_levels, 0, _flags(False, False, True, autotuned, prune, asynchronous, cache),
                           tuning)
    r = _vp()
    _check(lib.lv_louvain(graph.handle, ctypes.byref(p), ctypes.byref(r)), "lv_louvain")
    try:
        labels = np.empty(max(graph.n, 1), dtype=np.int32) if out is None else out
        pl, kind = _ptr(labels)
        _check(lib.lv_result_final_labels_all(r, pl, kind), "lv_result_final_labels_all")
        G = graph.count
        qi = np.zeros(G, dtype=np.int64)
        m = np.zeros(G, dtype=np.int64)
        q = np.zeros(G, dtype=np.float64)
        _check(lib.lv_result_modularity_all(r, qi.ctypes.data_as(_i64p), m.ctypes.data_as(_i64p),
                                            q.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
               "lv_result_modularity_all")
        return FinalPartition(labels[:graph.n] if out is None else labels, qi, m, q)
    finally:
        lib.lv_result_destroy(r)


def _read_graph_result(lib, r, gi: int, n0: int, keep_graphs: bool, level_labels: bool = True,
                       fin_out=None) -> LouvainResult:
    acc, att = ctypes.c_int32(), ctypes.c_int32()
    _check(lib.lv_result_graph_num_levels(r, gi, ctypes.byref(acc), ctypes.byref(att)), "lv_result_graph_num_levels")
    levels = []
    for lvl in range(att.value):
        info = lv_level_info()
        _check(lib.lv_result_graph_level_info(r, gi, lvl, ctypes.byref(info)), "lv_result_graph_level_info")
        mv = np.zeros(max(info.sweeps, 1), dtype=np.int64)
        _check(lib.lv_result_graph_level_moves(r, gi, lvl, mv.ctypes.data_as(_i64p), info.sweeps),
               "lv_result_graph_level_moves")
        lr = LevelResult(info.as_dict(), [int(x) for x in mv[:info.sweeps]])
        if lvl < acc.value and level_labels:
            lab = np.empty(info.n, dtype=np.int32)
            _check(lib.lv_result_graph_level_labels(r, gi, lvl, lab.ctypes.data, LV_MEM_HOST),
                   "lv_result_graph_level_labels")
            lr.labels = lab
            if keep_graphs:
                nnz = ctypes.c_int64()
                _check(lib.lv_result_level_graph(r, lvl, None, None, None, ctypes.byref(nnz), LV_MEM_HOST),
                       "lv_result_level_graph")
                off = np.empty(info.n_next + 1, dtype=np.int32)
                idx = np.empty(max(nnz.value, 1), dtype=np.int32)
                w = np.empty(max(nnz.value, 1), dtype=np.int32)
                _check(lib.lv_result_level_graph(r, lvl, off.ctypes.data, idx.ctypes.data, w.ctypes.data,
                                                 ctypes.byref(nnz), LV_MEM_HOST), "lv_result_level_graph")
                lr.graph = (off, idx[:nnz.value], w[:nnz.value])
        levels.append(lr)
    fin = np.empty(n0, dtype=np.int32) if fin_out is None else fin_out
    pf, kind = _ptr(fin)
    _check(lib.lv_result_graph_final_labels(r, gi, pf, kind), "lv_result_graph_final_labels")
    qi, m, q = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
    _check(lib.lv_result_graph_modularity(r, gi, ctypes.byref(qi), ctypes.byref(m), ctypes.byref(q)),
           "lv_result_graph_modularity")
    return LouvainResult(qi.value, m.value, q.value, fin, levels)


def _flags(timing: bool, keep_graphs: bool = False, hipgraph: bool = True, autotuned: bool = False,
           prune: bool = False, asynchronous: bool = False, cache: bool = True) -> int:
    return ((LV_TIMING if timing else 0) | (LV_KEEP_GRAPHS if keep_graphs else 0) | (0 if hipgraph else LV_NO_HIPGRAPH)
            | (LV_AUTOTUNE if autotuned else 0) | (LV_PRUNE if prune else 0) | (LV_ASYNC if asynchronous else 0)
            | (0 if cache else LV_NO_CACHE))


def louvain(graph: Graph, max_sweeps: int = 20, max_levels: int = 32, timing: bool = False,
            keep_graphs: bool = False, tuning: Optional[dict] = None, hipgraph: bool = True,
            autotuned: bool = False, level_labels: bool = True, prune: bool = False, asynchronous: bool = False,
            out=None, cache: bool = True):
    """lv_louvain + result accessors, copied to host numpy.  A packed handle
    (``Graph.batch``) gives one LouvainResult per graph, in order.  With
    level_labels=False only the final labels are copied (levels keep their
    statistics and move counts).  prune=True sets LV_PRUNE, asynchronous=True
    LV_ASYNC, cache=False LV_NO_CACHE.  `out` (one graph only) takes the final labels instead of a new
    numpy array: a numpy or torch int32 buffer of n entries, host or device."""
    if out is not None and graph.count != 1:
        raise ValueError("out= takes the final labels of a one-graph handle")
    lib = load_library()
    p, _keep = make_params(max_sweeps, max_levels, 0, _flags(timing, keep_graphs, hipgraph, autotuned, prune,
                                                            asynchronous, cache), tuning)
    r = _vp()
    _check(lib.lv_louvain(graph.handle, ctypes.byref(p), ctypes.byref(r)), "lv_louvain")
    try:
        if graph.count == 1:
            return _read_graph_result(lib, r, 0, graph.n, keep_graphs, level_labels, out)
        return [_read_graph_result(lib, r, gi, graph.sizes[gi], False, level_labels) for gi in range(graph.count)]
    finally:
        lib.lv_result_destroy(r)


@dataclass
class LpaResult:
    labels: np.ndarray
    moves: List[int]
    info: dict


def lpa(graph: Graph, max_sweeps: int = 20, threshold: int = 0, timing: bool = False, out=None,
        tuning: Optional[dict] = None, hipgraph: bool = True, autotuned: bool = False, prune: bool = False,
        asynchronous: bool = False, cache: bool = True) -> LpaResult:
    """lv_lpa; labels land in `out` (numpy or torch int32) or a new numpy array."""
    lib = load_library()
    if graph.count != 1:
        return lpa_batch(graph, max_sweeps, threshold, tuning=tuning, hipgraph=hipgraph, autotuned=autotuned,
                         prune=prune, asynchronous=asynchronous, cache=cache)
    p, _keep = make_params(max_sweeps, 32, threshold,
                           _flags(timing, False, hipgraph, autotuned, prune, asynchronous, cache), tuning)
    labels = np.empty(graph.n, dtype=np.int32) if out is None else out
    pl, kind = _ptr(labels)
    info = lv_level_info()
    mv = np.zeros(max_sweeps, dtype=np.int64)
    _check(lib.lv_lpa(graph.handle, ctypes.byref(p), pl, kind, ctypes.byref(info), mv.ctypes.data_as(_i64p),
                      max_sweeps), "lv_lpa")
    return LpaResult(labels, [int(x) for x in mv[:info.sweeps]], info.as_dict())


def lpa_batch(graph: Graph, max_sweeps: int = 20, threshold: int = 0, tuning: Optional[dict] = None,
              hipgraph: bool = True, autotuned: bool = False, prune: bool = False,
              asynchronous: bool = False, cache: bool = True) -> List[LpaResult]:
    """lv_lpa_batch over a packed handle: one LpaResult per graph (local labels)."""
    lib = load_library()
    p, _keep = make_params(max_sweeps, 32, threshold,
                           _flags(False, False, hipgraph, autotuned, prune, asynchronous, cache), tuning)
    G = graph.count
    labels = np.empty(max(graph.n, 1), dtype=np.int32)
    sw = np.zeros(G, dtype=np.int32)
    qi = np.zeros(G, dtype=np.int64)
    m = np.zeros(G, dtype=np.int64)
    mv = np.zeros((G, max_sweeps), dtype=np.int64)
    _check(lib.lv_lpa_batch(graph.handle, ctypes.byref(p), labels.ctypes.data, LV_MEM_HOST, sw.ctypes.data_as(_i32p),
                            qi.ctypes.data_as(_i64p), m.ctypes.data_as(_i64p), mv.ctypes.data_as(_i64p), max_sweeps),
           "lv_lpa_batch")
    out, base = [], 0
    for gi in range(G):
        n = graph.sizes[gi]
        info = {"n": n, "sweeps": int(sw[gi]), "q_end": int(qi[gi]), "M": int(m[gi])}
        out.append(LpaResult(labels[base:base + n].copy(), [int(x) for x in mv[gi, :sw[gi]]], info))
        base += n
    return out


def probe_gather(graph: Graph, reps: int = 5) -> float:
    """lv_probe_gather: the handle's pure-gather ceiling in entries per second."""
    out = ctypes.c_double()
    _check(load_library().lv_probe_gather(graph.handle, int(reps), ctypes.byref(out)), "lv_probe_gather")
    return out.value


def probe_copy(graph: Graph, reps: int = 5) -> float:
    """lv_probe_copy: a STREAM-style copy of the handle's index array, bytes read plus written per second."""
    out = ctypes.c_double()
    _check(load_library().lv_probe_copy(graph.handle, int(reps), ctypes.byref(out)), "lv_probe_copy")
    return out.value


def autotune(graph: Graph, max_sweeps: int = 20):
    """lv_autotune -> (tuning dict, estimated level ms); the handle keeps the
    setting for calls with ``autotuned=True``."""
    lib = load_library()
    p, _keep = make_params(max_sweeps, 32, 0, 0, None)
    t = lv_tuning()
    ms = ctypes.c_double()
    _check(lib.lv_autotune(graph.handle, ctypes.byref(p), ctypes.byref(t), ctypes.byref(ms)), "lv_autotune")
    return {name: getattr(t, name) for name, _ in lv_tuning._fields_}, ms.value


def modularity(graph: Graph, labels):
    """lv_modularity -> (Q_int, M, Q)."""
    lib = load_library()
    pl, kind = _ptr(labels)
    qi, m, q = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
    _check(lib.lv_modularity(graph.handle, pl, kind, ctypes.byref(qi), ctypes.byref(m), ctypes.byref(q)),
           "lv_modularity")
    return qi.value, m.value, q.value


NOALLOC_SCRATCH_BYTES = 64 << 20


def modularity_noalloc(graph: Graph, labels):
    """lv_modularity_noalloc -> (Q_int, M, Q); labels: a device int32 tensor of n entries."""
    lib = load_library()
    pl, kind = _ptr(labels)
    if kind != LV_MEM_DEVICE:
        raise ValueError("lv_modularity_noalloc takes device labels")
    qi, m, q = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
    _check(lib.lv_modularity_noalloc(graph.handle, pl, ctypes.byref(qi), ctypes.byref(m), ctypes.byref(q)),
           "lv_modularity_noalloc")
    return qi.value, m.value, q.value


class Server:
    """Continuous-batching Louvain server (lv_server_*).  Thread-safe: submit
    from any thread; results are collected per ticket."""

    def __init__(self, mem_budget: int = 0, max_jobs: int = 0, max_sweeps: int = 0, max_levels: int = 0,
                 validate: bool = True, tuning: Optional[dict] = None):
        lib = load_library()
        cfg = lv_server_config(mem_budget, max_jobs, max_sweeps, max_levels, LV_VALIDATE if validate else 0)
        self._tuning = None
        if tuning:
            self._tuning = lv_tuning(**tuning)
            cfg.tuning = ctypes.pointer(self._tuning)
        h = _vp()
        _check(lib.lv_server_create(ctypes.byref(cfg), ctypes.byref(h)), "lv_server_create")
        self._h = h

    def submit(self, g, device: bool = False) -> int:
        """Queue a ``graphgen.CSR``-like graph; returns its ticket.  With
        device=True its arrays are first put in device memory (torch), and the
        server copies them device to device."""
        lib = load_library()
        off = np.ascontiguousarray(g.offsets, dtype=np.int32)
        idx = np.ascontiguousarray(g.indices, dtype=np.int32)
        w = None if g.weights is None else np.ascontiguousarray(g.weights, dtype=np.int32)
        kind = LV_MEM_HOST
        if device:
            import torch

            off, idx = torch.from_numpy(off).cuda(), torch.from_numpy(idx).cuda()
            w = None if w is None else torch.from_numpy(w).cuda()
            torch.cuda.synchronize()
            kind = LV_MEM_DEVICE
        po, _ = _ptr(off)
        pi, _ = _ptr(idx)
        pw, _ = _ptr(w)
        t = ctypes.c_uint64()
        _check(lib.lv_server_submit(self._h, int(g.n), po, pi, pw, kind, ctypes.byref(t)), "lv_server_submit")
        return t.value

    def poll(self, ticket: int) -> int:
        st = ctypes.c_int32()
        _check(load_library().lv_server_poll(self._h, ticket, ctypes.byref(st)), "lv_server_poll")
        return st.value

    def wait(self, ticket: int, timeout_ms: int = -1) -> bool:
        st = load_library().lv_server_wait(self._h, ticket, timeout_ms)
        if st == 8:  # LV_E_BUSY: timed out
            return False
        _check(st, "lv_server_wait")
        return True

    def result(self, ticket: int, n: int):
        """(labels, info dict) of a finished job; raises LvError with the job's status."""
        lib = load_library()
        labels = np.empty(max(n, 1), dtype=np.int32)
        info = lv_job_info()
        st = lib.lv_server_result(self._h, ticket, labels.ctypes.data, LV_MEM_HOST, ctypes.byref(info))
        _check(st, "lv_server_result")
        return labels[:n], {name: getattr(info, name) for name, _ in lv_job_info._fields_}

    def cancel(self, ticket: int):
        _check(load_library().lv_server_cancel(self._h, ticket), "lv_server_cancel")

    def stats(self) -> dict:
        st = lv_server_stats()
        _check(load_library().lv_server_stats_get(self._h, ctypes.byref(st)), "lv_server_stats_get")
        return {name: getattr(st, name) for name, _ in lv_server_stats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            load_library().lv_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
