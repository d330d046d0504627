"""Seeded synthetic graph generators (shared input source, no method arithmetic).

The C library ``libgraphgen.so`` next to this file does the sampling and the
CSR canonicalisation; this module only marshals arguments.  Both the CPU oracle
and the GPU library consume the same ``CSR`` objects, so the two sides always
see identical input bytes.

Graph model: the paper's Section II-A (undirected, weighted, unit weight when
unweighted).  Generated graphs carry no self-loops; tests that need loops build
small graphs by hand with :func:`from_edges`.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_SRC = os.path.join(_HERE, "graphgen.c")

_i32p = ctypes.POINTER(ctypes.c_int32)


def build_library() -> str:
    """Compile libgraphgen.so (plain C + OpenMP)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", _LIB_PATH, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_library()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.gg_free.argtypes = [ctypes.c_void_p]
        lib.gg_set_threads.argtypes = [ctypes.c_int]
        lib.gg_rand.restype = ctypes.c_uint64
        lib.gg_rand.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.gg_stream_key.restype = ctypes.c_uint64
        lib.gg_stream_key.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        out3 = [ctypes.POINTER(_i32p), ctypes.POINTER(_i32p), ctypes.POINTER(ctypes.c_int64)]
        lib.gg_csr_from_edges.argtypes = [ctypes.c_int32, ctypes.c_int64, _i32p, _i32p] + out3
        lib.gg_rmat.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                ctypes.c_double, ctypes.c_double, ctypes.c_uint64] + out3
        lib.gg_rmat_edges.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_uint64, _i32p, _i32p]
        lib.gg_sbm.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                               ctypes.c_uint64] + out3
        lib.gg_pair_weights.argtypes = [ctypes.c_int32, _i32p, _i32p, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_uint64, _i32p]
        lib.gg_lfr.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                               ctypes.c_double, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                               ctypes.c_uint64] + out3 + [ctypes.POINTER(_i32p),
                                                          ctypes.POINTER(ctypes.c_int32)]
        for f in ("gg_csr_from_edges", "gg_rmat", "gg_sbm", "gg_pair_weights", "gg_lfr"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclass
class CSR:
    """Symmetric CSR graph.  ``weights`` None means unit weights.

    A diagonal entry (v, v, w) is a loop of weight w (the paper counts it twice
    in the weighted degree).
    """

    n: int
    offsets: np.ndarray  # int32[n+1]
    indices: np.ndarray  # int32[nnz]
    weights: Optional[np.ndarray] = None  # int32[nnz] or None
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.offsets[-1])

    def weights_or_ones(self) -> np.ndarray:
        if self.weights is None:
            return np.ones(self.nnz, dtype=np.int32)
        return self.weights


def _take(off_p, idx_p, n: int, nnz: int):
    lib = _load()
    off = np.ctypeslib.as_array(off_p, shape=(n + 1,)).copy()
    idx = np.ctypeslib.as_array(idx_p, shape=(max(nnz, 1),))[:nnz].copy()
    lib.gg_free(ctypes.cast(off_p, ctypes.c_void_p))
    lib.gg_free(ctypes.cast(idx_p, ctypes.c_void_p))
    return off, idx


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"graphgen {what} failed with code {rc}")


def rmat(scale: int, edge_factor: float = 16.0, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 2, n: Optional[int] = None, samples: Optional[int] = None) -> CSR:
    """R-MAT graph: ``samples`` (default edge_factor * 2^scale) quadrant descents,
    symmetrised, self-loops and duplicates removed, unit weights."""
    lib = _load()
    nv = (1 << scale) if n is None else int(n)
    ns = int(round(edge_factor * (1 << scale))) if samples is None else int(samples)
    off_p, idx_p, nnz = _i32p(), _i32p(), ctypes.c_int64()
    _check(lib.gg_rmat(scale, nv, ns, a, b, c, seed, ctypes.byref(off_p), ctypes.byref(idx_p),
                       ctypes.byref(nnz)), "rmat")
    off, idx = _take(off_p, idx_p, nv, nnz.value)
    return CSR(nv, off, idx, None, f"rmat{scale}_ef{edge_factor:g}_s{seed}")


def rmat_edges(scale: int, edge_factor: float = 16.0, a: float = 0.57, b: float = 0.19, c: float = 0.19,
               seed: int = 2, n: Optional[int] = None, samples: Optional[int] = None):
    """The raw samples behind ``rmat`` with the same arguments: (u, v) int32
    arrays, one per quadrant descent, loops and repeated pairs included (a
    sample outside [0, n) is recorded as the loop (0, 0))."""
    lib = _load()
    nv = (1 << scale) if n is None else int(n)
    ns = int(round(edge_factor * (1 << scale))) if samples is None else int(samples)
    u = np.empty(max(ns, 1), dtype=np.int32)
    v = np.empty(max(ns, 1), dtype=np.int32)
    _check(lib.gg_rmat_edges(scale, nv, ns, a, b, c, seed, u.ctypes.data_as(_i32p), v.ctypes.data_as(_i32p)),
           "rmat_edges")
    return u[:ns], v[:ns]


def sbm(n: int, block_size: int, p_in: float, p_out: float, seed: int = 1) -> CSR:
    """Planted-partition SBM with equal blocks (last block takes the remainder)."""
    lib = _load()
    off_p, idx_p, nnz = _i32p(), _i32p(), ctypes.c_int64()
    _check(lib.gg_sbm(n, block_size, p_in, p_out, seed, ctypes.byref(off_p), ctypes.byref(idx_p),
                      ctypes.byref(nnz)), "sbm")
    off, idx = _take(off_p, idx_p, n, nnz.value)
    return CSR(n, off, idx, None, f"sbm{n}_b{block_size}_s{seed}")


def pair_weights(g: CSR, lo: int, hi: int, seed: int) -> np.ndarray:
    """Symmetric per-pair weights uniform in [lo, hi]."""
    lib = _load()
    w = np.empty(g.nnz, dtype=np.int32)
    _check(lib.gg_pair_weights(g.n, g.offsets.ctypes.data_as(_i32p), g.indices.ctypes.data_as(_i32p),
                               lo, hi, seed, w.ctypes.data_as(_i32p)), "pair_weights")
    return w


def lfr(n: int, tau1: float = 2.5, mean_deg: float = 20.0, kmax: int = 5000, tau2: float = 1.5,
        smin: int = 50, smax: int = 20000, mu: float = 0.3, wlo: int = 1, whi: int = 8,
        seed: int = 3):
    """LFR-style power-law benchmark; returns (CSR with weights, planted membership)."""
    lib = _load()
    off_p, idx_p, nnz = _i32p(), _i32p(), ctypes.c_int64()
    mem_p, nc = _i32p(), ctypes.c_int32()
    _check(lib.gg_lfr(n, tau1, mean_deg, kmax, tau2, smin, smax, mu, seed, ctypes.byref(off_p),
                      ctypes.byref(idx_p), ctypes.byref(nnz), ctypes.byref(mem_p), ctypes.byref(nc)),
           "lfr")
    off, idx = _take(off_p, idx_p, n, nnz.value)
    memb = np.ctypeslib.as_array(mem_p, shape=(n,)).copy()
    lib.gg_free(ctypes.cast(mem_p, ctypes.c_void_p))
    g = CSR(n, off, idx, None, f"lfr{n}_mu{mu:g}_s{seed}")
    g.weights = pair_weights(g, wlo, whi, seed)
    return g, memb


def from_edges(n: int, u, v, w=None, keep_loops: bool = True) -> CSR:
    """Small hand-built graphs (tests): undirected edge list -> canonical CSR.

    Duplicate pairs have their weights summed; a pair (v, v, w) becomes a loop
    entry of weight w.  Pure numpy; meant for small inputs.
    """
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    w = np.ones(len(u), dtype=np.int64) if w is None else np.asarray(w, dtype=np.int64)
    if len(u) and (u.min() < 0 or v.min() < 0 or u.max() >= n or v.max() >= n):
        raise ValueError("endpoint out of range")
    loop = u == v
    if not keep_loops:
        u, v, w, loop = u[~loop], v[~loop], w[~loop], loop[~loop]
    rows = np.concatenate([u, v[~loop]])
    cols = np.concatenate([v, u[~loop]])
    ws = np.concatenate([w, w[~loop]])
    key = rows * n + cols
    order = np.argsort(key, kind="stable")
    key, ws = key[order], ws[order]
    uk, start = np.unique(key, return_index=True)
    wsum = np.add.reduceat(ws, start) if len(ws) else ws
    r = (uk // n).astype(np.int64)
    cidx = (uk % n).astype(np.int32)
    off = np.zeros(n + 1, dtype=np.int64)
    np.add.at(off, r + 1, 1)
    off = np.cumsum(off).astype(np.int32)
    return CSR(n, off, cidx, wsum.astype(np.int32), "edges")


def stream_key(seed: int, tag: int) -> int:
    return int(_load().gg_stream_key(seed, tag))


def rand_u64(key: int, counter: int) -> int:
    return int(_load().gg_rand(key, counter))


def loguniform_int(lo: int, hi: int, u: float) -> int:
    return int(math.floor(math.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))))


def batch_mix(count: int = 4096, seed: int = 4, n_lo: int = 1024, n_hi: int = 65536, deg_lo: float = 8.0,
              deg_hi: float = 32.0, block: int = 128, intra: float = 0.75):
    """The mixed batch workload: `count` independent graphs alternating SBM and
    R-MAT, vertex counts log-uniform in [n_lo, n_hi], mean degree uniform in
    [deg_lo, deg_hi], unit weights.  SBM: blocks of `block` vertices with a
    fraction `intra` of the expected degree inside the block.  R-MAT: scale
    ceil(log2 n), (0.57, 0.19, 0.19), ids >= n dropped, n * degree / 2 samples.
    Parameters are drawn from a numpy generator seeded with `seed`; graph t
    uses generator seed `seed * 1_000_003 + t`."""
    rng = np.random.default_rng(seed)
    specs = []
    for t in range(count):
        n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
        d = float(rng.uniform(deg_lo, deg_hi))
        specs.append((t, n, d, seed * 1_000_003 + t))

    def make(spec):
        t, n, d, gs = spec
        if t % 2 == 0:
            b = min(block, n)
            p_in = min(1.0, intra * d / max(1, b - 1))
            p_out = min(1.0, (1.0 - intra) * d / max(1, n - b))
            g = sbm(n, b, p_in, p_out, seed=gs)
        else:
            scale = max(1, int(np.ceil(np.log2(n))))
            g = rmat(scale, n=n, samples=int(round(n * d / 2)), seed=gs)
        g.name = f"mix{t}"
        return g

    # the graphs are independent: generate them on host threads, one OpenMP
    # thread each (the C generators release the interpreter lock)
    from concurrent.futures import ThreadPoolExecutor

    workers = max(1, min(16, os.cpu_count() or 1))
    lib = _load()

    def init():
        lib.gg_set_threads(1)

    with ThreadPoolExecutor(workers, initializer=init) as ex:
        return list(ex.map(make, specs))


def serving_pool(count: int = 32, seed: int = 5, n_lo: int = 10_000, n_hi: int = 4_000_000,
                 ef_lo: int = 8, ef_hi: int = 16):
    """Graphs for the serving workload: R-MAT (0.57, 0.19, 0.19), vertex
    counts log-uniform in [n_lo, n_hi], edge factor uniform in {ef_lo..ef_hi}
    (n * ef samples), scale ceil(log2 n) with ids >= n dropped, unit weights.
    Generated on host threads, one OpenMP thread each."""
    rng = np.random.default_rng(seed)
    specs = []
    for t in range(count):
        n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
        ef = int(rng.integers(ef_lo, ef_hi + 1))
        specs.append((t, n, ef, seed * 1_000_003 + t))

    def make(spec):
        t, n, ef, gs = spec
        scale = max(1, int(np.ceil(np.log2(n))))
        g = rmat(scale, n=n, samples=n * ef, seed=gs)
        g.name = f"serve{t}_n{n}_ef{ef}"
        return g

    from concurrent.futures import ThreadPoolExecutor

    lib = _load()
    with ThreadPoolExecutor(max(1, min(16, os.cpu_count() or 1)), initializer=lambda: lib.gg_set_threads(1)) as ex:
        return list(ex.map(make, specs))
