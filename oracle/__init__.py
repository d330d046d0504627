"""CPU oracle for the Louvain local-moving method (and its LPA mode).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the GPU library never does
and shares no code with it.

The arithmetic lives in ``lv_oracle.c`` (plain C, int64, OpenMP over the
vertex loop of a sweep); this module marshals arguments and runs the level
driver of the paper's Algorithm 3 in plain Python:

    repeat: local moving (Alg. 2) -> renumber -> aggregate (Alg. 3, Aggregation)
    until a level leaves modularity where it was (the end condition of
    Section III-B) or max_levels levels were accepted.

Readings of the paper that fix deterministic semantics are stated in
``lv_oracle.c``'s header.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblv_oracle.so")
_SRC = os.path.join(_HERE, "lv_oracle.c")

LOUVAIN, LPA = 0, 1
DOWN, UP = 0, 1

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


def build_library() -> str:
    """Compile liblv_oracle.so with gcc (plain C + OpenMP)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", _LIB_PATH, _SRC]
    subprocess.run(cmd, check=True)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_library()
        _lib = _configure(ctypes.CDLL(_LIB_PATH))
    return _lib


def _configure(lib):
    """Declare the C signatures on a loaded oracle library."""
    i32, i64 = ctypes.c_int32, ctypes.c_int64
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    lib.orc_adjacency.argtypes = [i32, _i32p, _i32p, _i32p, _i32p]
    lib.orc_adjacency.restype = ctypes.c_int
    lib.orc_degrees.argtypes = [i32, _i32p, _i32p, _i64p]
    lib.orc_degrees.restype = i64
    lib.orc_modularity.argtypes = [i32, _i32p, _i32p, _i32p, _i32p, _i64p, _i64p]
    lib.orc_modularity.restype = ctypes.c_int
    lib.orc_decide_vertices.argtypes = [i32, _i32p, _i32p, _i32p, _i64p, i64, _i32p, _i64p,
                                        ctypes.c_int, ctypes.c_int, _i32p, i32, _i32p]
    lib.orc_decide_vertices.restype = ctypes.c_int
    lib.orc_sweep.argtypes = [i32, _i32p, _i32p, _i32p, _i64p, i64, _i32p, _i64p, ctypes.c_int,
                              ctypes.c_int, ctypes.c_void_p, _i32p]
    lib.orc_sweep.restype = i64
    lib.orc_local_move.argtypes = [i32, _i32p, _i32p, _i32p, ctypes.c_int, i32, i64, ctypes.c_int, _i32p,
                                   _i64p]
    lib.orc_local_move.restype = i32
    lib.orc_renumber.argtypes = [i32, _i32p, _i32p]
    lib.orc_renumber.restype = i32
    lib.orc_aggregate.argtypes = [i32, _i32p, _i32p, _i32p, _i32p, i32, _i32p, _i32p, _i32p]
    lib.orc_aggregate.restype = i64
    lib.orc_singleton_qint.argtypes = [i32, _i32p, _i32p, _i32p]
    lib.orc_singleton_qint.restype = i64
    return lib


def _p32(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(_i32p)


def _p64(a: np.ndarray):
    assert a.dtype == np.int64 and a.flags.c_contiguous
    return a.ctypes.data_as(_i64p)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(t: int) -> None:
    _load().orc_set_threads(int(t))


@dataclass
class Adj:
    """Level graph in the oracle's convention: A_vv holds twice the loop weight."""

    n: int
    off: np.ndarray
    idx: np.ndarray
    a: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.off[-1])


def adjacency(g) -> Adj:
    """Caller CSR (``graphgen.CSR``-like: n, offsets, indices, weights|None) -> Adj."""
    lib = _load()
    off = np.ascontiguousarray(g.offsets, dtype=np.int32)
    idx = np.ascontiguousarray(g.indices, dtype=np.int32)
    a = np.empty(len(idx), dtype=np.int32)
    w = None if g.weights is None else np.ascontiguousarray(g.weights, dtype=np.int32)
    rc = lib.orc_adjacency(g.n, _p32(off), _p32(idx), _p32(w) if w is not None else None, _p32(a))
    if rc != 0:
        raise ValueError(f"oracle: invalid graph (code {rc})")
    return Adj(g.n, off, idx, a)


def degrees(adj: Adj):
    k = np.empty(adj.n, dtype=np.int64)
    M = _load().orc_degrees(adj.n, _p32(adj.off), _p32(adj.a), _p64(k))
    return k, int(M)


def modularity_int(adj: Adj, labels) -> tuple:
    """(Q_int, M) for any labels in [0, n)."""
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    q, m = ctypes.c_int64(), ctypes.c_int64()
    rc = _load().orc_modularity(adj.n, _p32(adj.off), _p32(adj.idx), _p32(adj.a), _p32(lab),
                                ctypes.byref(q), ctypes.byref(m))
    if rc != 0:
        raise ValueError("oracle: labels out of range")
    return int(q.value), int(m.value)


def q_float(q_int: int, M: int) -> float:
    """FP64 modularity from the exact integers: Q = Q_int / (M * M)."""
    return float(q_int) / (float(M) * float(M)) if M > 0 else 0.0


def modularity(g, labels) -> tuple:
    """(Q_int, M, Q) of a caller-convention graph and labels."""
    q, m = modularity_int(adjacency(g), labels)
    return q, m, q_float(q, m)


def sweep(adj: Adj, c, sigma, direction: int, mode: int = LOUVAIN, active=None):
    """One synchronous sweep against state (c, sigma); returns (c_next, moves).
    `active` (bool per vertex, None = all) limits which vertices are evaluated."""
    k, M = degrees(adj)
    c = np.ascontiguousarray(c, dtype=np.int32)
    sigma = np.ascontiguousarray(sigma, dtype=np.int64)
    nxt = np.empty(adj.n, dtype=np.int32)
    act = None if active is None else np.ascontiguousarray(active, dtype=np.uint8)
    mv = _load().orc_sweep(adj.n, _p32(adj.off), _p32(adj.idx), _p32(adj.a), _p64(k), M, _p32(c),
                           _p64(sigma), direction, mode, None if act is None else act.ctypes.data, _p32(nxt))
    if mv < 0:
        raise MemoryError("oracle sweep")
    return nxt, int(mv)


def decide_vertices(adj: Adj, verts, c, sigma, direction: int, mode: int = LOUVAIN, k=None, M=None):
    """Decisions of the listed vertices against state (c, sigma)."""
    if k is None:
        k, M = degrees(adj)
    verts = np.ascontiguousarray(verts, dtype=np.int32)
    c = np.ascontiguousarray(c, dtype=np.int32)
    sigma = np.ascontiguousarray(sigma, dtype=np.int64)
    out = np.empty(len(verts), dtype=np.int32)
    rc = _load().orc_decide_vertices(adj.n, _p32(adj.off), _p32(adj.idx), _p32(adj.a), _p64(k), M,
                                     _p32(c), _p64(sigma), direction, mode, _p32(verts), len(verts),
                                     _p32(out))
    if rc != 0:
        raise MemoryError("oracle decide")
    return out


def local_move(adj: Adj, mode: int = LOUVAIN, max_sweeps: int = 20, theta: int = 0, prune: bool = False):
    """One level from singletons; returns (labels c, per-sweep moves).  With
    `prune`, only active vertices are evaluated (rule in lv_oracle.c)."""
    c = np.empty(adj.n, dtype=np.int32)
    moves = np.zeros(max_sweeps, dtype=np.int64)
    s = _load().orc_local_move(adj.n, _p32(adj.off), _p32(adj.idx), _p32(adj.a), mode, max_sweeps,
                               theta, int(bool(prune)), _p32(c), _p64(moves))
    if s < 0:
        raise RuntimeError(f"oracle local_move failed ({-s})")
    return c, moves[:s].copy()


def renumber(c):
    c = np.ascontiguousarray(c, dtype=np.int32)
    lab = np.empty(len(c), dtype=np.int32)
    n2 = _load().orc_renumber(len(c), _p32(c), _p32(lab))
    if n2 < 0:
        raise ValueError("oracle renumber: label out of range")
    return lab, int(n2)


def aggregate(adj: Adj, labels, n2: int) -> Adj:
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    off2 = np.empty(n2 + 1, dtype=np.int32)
    idx2 = np.empty(max(adj.nnz, 1), dtype=np.int32)
    a2 = np.empty(max(adj.nnz, 1), dtype=np.int32)
    e2 = _load().orc_aggregate(adj.n, _p32(adj.off), _p32(adj.idx), _p32(adj.a), _p32(lab), n2,
                               _p32(off2), _p32(idx2), _p32(a2))
    if e2 < 0:
        raise RuntimeError(f"oracle aggregate failed ({-e2})")
    return Adj(n2, off2, idx2[:e2].copy(), a2[:e2].copy())


def graph_from_edges(n: int, src, dst, w=None, drop_loops: bool = False, simple: bool = False):
    """Undirected edge list -> symmetric CSR in the caller's convention.

    Section II-A: G(V, E, w) with E a set of unordered pairs {u, v}, loops
    allowed.  Every listing of a pair, in either orientation, is merged into
    one edge whose weight is the sum of the listings' weights (Section III-B
    sums the weights of edges whose endpoints coincide); with `simple` the
    merged edge has weight 1.  A loop (v, v) is one diagonal entry carrying
    its weight (the weighted degree counts it twice later); `drop_loops`
    removes loops.  Rows come out sorted.  Returns (offsets, indices,
    weights), int32.  Raises ValueError for an endpoint outside [0, n) or a
    weight below 1, OverflowError for a merged weight above 2^31 - 1.
    """
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    w = np.ones(len(src), dtype=np.int64) if w is None else np.asarray(w, dtype=np.int64)
    if len(src) != len(dst) or len(w) != len(src):
        raise ValueError("src, dst and w differ in length")
    if len(src) and (min(src.min(), dst.min()) < 0 or max(src.max(), dst.max()) >= n):
        raise ValueError("edge endpoint outside [0, n)")
    if len(w) and w.min() < 1:
        raise ValueError("edge weight < 1")
    lo, hi = np.minimum(src, dst), np.maximum(src, dst)
    if drop_loops:
        keep = lo != hi
        lo, hi, w = lo[keep], hi[keep], w[keep]
    # one record per unordered pair, its listings' weights summed
    pair = lo * max(n, 1) + hi
    pairs, which = np.unique(pair, return_inverse=True)
    weight = np.zeros(len(pairs), dtype=np.int64)
    np.add.at(weight, which, w)
    if simple:
        weight[:] = 1
    if len(weight) and weight.max() > np.iinfo(np.int32).max:
        raise OverflowError("merged edge weight above 2^31 - 1")
    a, b = pairs // max(n, 1), pairs % max(n, 1)
    # both directions of a non-loop pair, one entry for a loop
    off_diag = a != b
    rows = np.concatenate([a, b[off_diag]])
    cols = np.concatenate([b, a[off_diag]])
    vals = np.concatenate([weight, weight[off_diag]])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.add.at(offsets, rows + 1, 1)
    return np.cumsum(offsets).astype(np.int32), cols.astype(np.int32), vals.astype(np.int32)


def singleton_qint(adj: Adj) -> int:
    return int(_load().orc_singleton_qint(adj.n, _p32(adj.off), _p32(adj.idx), _p32(adj.a)))


@dataclass
class LevelRecord:
    n: int
    nnz: int
    q_start: int
    q_end: int
    sweeps: int
    moves: np.ndarray
    labels: np.ndarray  # renumbered labels of this level's vertices
    n_next: int
    accepted: bool


@dataclass
class LouvainResult:
    M: int
    q_int: int
    q: float
    final_labels: np.ndarray
    levels: List[LevelRecord] = field(default_factory=list)  # every attempted level

    @property
    def accepted(self) -> List[LevelRecord]:
        return [lv for lv in self.levels if lv.accepted]


def louvain(g, max_sweeps: int = 20, max_levels: int = 32, keep_graphs: bool = False, prune: bool = False,
            phase_times: Optional[dict] = None):
    """Multi-level Louvain (Alg. 3) under the oracle's deterministic semantics.

    Level l: Q_start = Q_int of singletons on G_l; local moving; renumber;
    aggregate to G_{l+1}; Q_end = Q_int of singletons on G_{l+1} (equal to
    Q_int(G_l, labels)).  A level with Q_end <= Q_start is discarded and ends
    the run; otherwise it is accepted and G <- G_{l+1}.

    `phase_times` (a dict, optional) accumulates the wall time in seconds of
    the phases the paper times apart (Section V-B): "local_move", "renumber"
    and "aggregate" (the Q_int evaluations go to "other").
    """
    import time

    pt = phase_times if phase_times is not None else {}
    for key in ("local_move", "renumber", "aggregate", "other"):
        pt.setdefault(key, 0.0)
    t = time.perf_counter()
    adj = adjacency(g)
    n0 = adj.n
    _, M = degrees(adj)
    final = np.arange(n0, dtype=np.int32)
    res = LouvainResult(M=M, q_int=singleton_qint(adj), q=0.0, final_labels=final)
    graphs = [adj]
    pt["other"] += time.perf_counter() - t
    while True:
        t0 = time.perf_counter()
        q_start = singleton_qint(adj)
        t1 = time.perf_counter()
        c, moves = local_move(adj, LOUVAIN, max_sweeps, 0, prune)
        t2 = time.perf_counter()
        labels, n2 = renumber(c)
        t3 = time.perf_counter()
        adj2 = aggregate(adj, labels, n2)
        t4 = time.perf_counter()
        q_end = singleton_qint(adj2)
        pt["other"] += (t1 - t0) + (time.perf_counter() - t4)
        pt["local_move"] += t2 - t1
        pt["renumber"] += t3 - t2
        pt["aggregate"] += t4 - t3
        accepted = q_end > q_start
        res.levels.append(LevelRecord(adj.n, adj.nnz, q_start, q_end, len(moves), moves, labels, n2,
                                      accepted))
        if not accepted:
            break
        final = labels[final]
        adj = adj2
        if keep_graphs:
            graphs.append(adj)
        res.q_int = q_end
        if len(res.accepted) >= max_levels:
            break
    res.final_labels = final
    res.q = q_float(res.q_int, M)
    if keep_graphs:
        res.graphs = graphs
    return res


@dataclass
class LpaResult:
    labels: np.ndarray
    moves: np.ndarray
    q_int: int
    M: int
    q: float


def lpa(g, max_sweeps: int = 20, theta: int = 0, prune: bool = False) -> LpaResult:
    """Label propagation (Alg. 1) as one level of synchronous sweeps, then renumber."""
    adj = adjacency(g)
    c, moves = local_move(adj, LPA, max_sweeps, theta, prune)
    labels, _ = renumber(c)
    q, M = modularity_int(adj, labels)
    return LpaResult(labels, moves, q, M, q_float(q, M))
