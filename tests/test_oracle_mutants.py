"""The pins must catch plausible mistakes in the oracle.

Each case compiles a copy of the oracle's C source with one planted mistake
(CPU only), swaps it in, and runs a compact version of the pins; at least one
of them has to fail.  The unmodified source has to pass the same checks.
"""
import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import bruteforce as bf
import graphgen
import oracle

SRC = os.path.join(os.path.dirname(oracle.__file__), "lv_oracle.c")

MUTANTS = {
    "stay_drops_self_volume": ("(sigma[A] - k[i])", "(sigma[A])"),
    "tie_to_largest_id": ("(s == best_score && C < best)", "(s == best_score && C > best)"),
    "self_loop_counted_in_W": ("if (j == i) continue;", ""),
    "loops_not_doubled": ("if (idx[e] == i) x *= 2;", ""),
    "direction_swapped": ("if (dir == ORC_DOWN && best > A)", "if (dir == ORC_DOWN && best < A)"),
    "non_strict_gain": ("best_score <= stay", "best_score < stay"),
    "score_sign": ("M * acc[C] - k[i] * sigma[C]", "M * acc[C] + k[i] * sigma[C]"),
    "modularity_sq_term": ("sq += tot[c] * tot[c];", "sq += tot[c];"),
    "renumber_by_label": ("if (map[c[i]] < 0) map[c[i]] = next++;", "if (map[c[i]] < 0) map[c[i]] = c[i];"),
    "aggregate_drops_weights": ("a2[out - 1] = (int32_t)s;", "a2[out - 1] = t[e].w;"),
    "stop_after_one_zero_sweep": ("if (s >= 2 && moves[s - 1] <= theta && moves[s - 2] <= theta) break;",
                                  "if (moves[s - 1] <= theta) break;"),
    "lpa_stay_ignores_own_label": (": wA;", ": 0;"),
    "prune_one_sweep_back": ("act[i] = chg1[i] | chg2[i];", "act[i] = chg1[i];"),
    "prune_ignores_neighbours": ("for (int32_t e = off[i]; e < off[i + 1]; ++e) chg1[idx[e]] = 1;", ""),
    "prune_from_second_sweep": ("if (prune && s > 2) {", "if (prune && s > 1) {"),
}


def detect() -> list:
    """Compact pins; returns the names of the checks that failed."""
    failed = []
    # brute-force decisions and modularity on tiny graphs
    dec_bad = q_bad = False
    for s in range(40):
        rng = np.random.default_rng(500 + s)
        n = int(rng.integers(2, 8))
        edges = bf.random_graph(rng, n, 0.6, 4, True)
        if not edges:
            continue
        A = bf.dense_adjacency(n, edges)
        try:
            adj = oracle.adjacency(bf.to_csr(n, edges))
        except ValueError:
            dec_bad = True
            continue
        k, _ = oracle.degrees(adj)
        for trial in range(3):
            labels = rng.integers(0, n, size=n) if trial else np.arange(n)
            sigma = np.bincount(labels, weights=k, minlength=n).astype(np.int64)
            q, M = oracle.modularity_int(adj, labels)
            if M != sum(map(sum, A)) or Fraction(q, M * M) != bf.modularity(A, labels):
                q_bad = True
            for down in (True, False):
                for lpa in (False, True):
                    got, _ = oracle.sweep(adj, labels, sigma, oracle.DOWN if down else oracle.UP,
                                          oracle.LPA if lpa else oracle.LOUVAIN)
                    if list(got) != bf.sweep(A, list(labels), down, lpa):
                        dec_bad = True
    if dec_bad:
        failed.append("decisions")
    if q_bad:
        failed.append("modularity")
    # renumber vs numpy first occurrence
    c = np.array([5, 2, 5, 0, 2, 6, 0], dtype=np.int32)
    lab, _ = oracle.renumber(c)
    if list(lab) != [0, 1, 0, 2, 1, 3, 2]:
        failed.append("renumber")
    # aggregation vs scipy
    import scipy.sparse as sp

    g = graphgen.sbm(300, 30, 0.3, 0.02, seed=4)
    g.weights = graphgen.pair_weights(g, 1, 8, seed=4)
    adj = oracle.adjacency(g)
    labels = (np.arange(g.n) // 7).astype(np.int32)
    co = oracle.aggregate(adj, labels, int(labels.max()) + 1)
    Am = sp.csr_matrix((adj.a.astype(np.int64), adj.idx, adj.off), shape=(g.n, g.n))
    S = sp.csr_matrix((np.ones(g.n, np.int64), (np.arange(g.n), labels)))
    ref = (S.T @ Am @ S).tocsr()
    ref.sort_indices()
    if not (np.array_equal(co.idx, ref.indices) and np.array_equal(co.a, ref.data)):
        failed.append("aggregate")
    # closed form + worked trace (per-sweep counts)
    edges = [(0, 1, 1), (0, 2, 1), (1, 2, 1), (3, 4, 1), (3, 5, 1), (4, 5, 1), (2, 3, 1)]
    r = oracle.louvain(bf.to_csr(6, edges))
    if Fraction(r.q_int, r.M * r.M) != Fraction(5, 14) or list(r.levels[0].moves) != [3, 1, 0, 0]:
        failed.append("trace")
    # pruned levels vs the brute-force replay (LPA on small graphs, Louvain on tiny ones)
    prune_bad = False
    for t in range(60):
        lpa = t % 2 == 0
        rng = np.random.default_rng(9500 + t)
        n = int(rng.integers(2, 25 if lpa else 10))
        edges = bf.random_graph(rng, n, float(rng.uniform(0.1, 0.6)), 5, bool(t % 3 == 0))
        if not edges:
            continue
        A = bf.dense_adjacency(n, edges)
        try:
            adj = oracle.adjacency(bf.to_csr(n, edges))
            c, mv = oracle.local_move(adj, oracle.LPA if lpa else oracle.LOUVAIN, 20, 0, True)
        except (ValueError, RuntimeError):
            prune_bad = True
            break
        if (list(c), list(mv)) != bf.local_move(A, lpa, True):
            prune_bad = True
            break
    if prune_bad:
        failed.append("prune")
    return failed


def _swap(path):
    old = oracle._lib
    oracle._lib = oracle._configure(ctypes.CDLL(path))
    return old


def test_unmodified_oracle_passes_compact_pins():
    assert detect() == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    before, after = MUTANTS[name]
    src = open(SRC).read()
    assert before in src, f"mutation anchor missing for {name}"
    mutated = src.replace(before, after, 1)
    c_path = tmp_path / f"{name}.c"
    so_path = tmp_path / f"lib{name}.so"
    c_path.write_text(mutated)
    subprocess.run(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-w", "-o", str(so_path), str(c_path)],
                   check=True)
    old = _swap(str(so_path))
    try:
        caught = detect()
    finally:
        oracle._lib = old
    assert caught, f"no pin caught mutant {name}"
