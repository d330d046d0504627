"""Pins of the oracle's active-vertex pruning (Alg. 1's V_active, Alg. 2's
needCheck) under synchronous sweeps.

Rule: in sweep s a vertex is evaluated if s <= 2, or if it or a neighbour
changed community in sweep s-1 or s-2; otherwise it keeps its community.

Two independent checks:
  * a brute-force replay (tests/bruteforce.py) whose decisions come from
    recomputed Fraction modularity gains and whose active set is read off the
    label history, on tiny graphs;
  * a property of label propagation: there pruning changes nothing.  LPA's
    decision reads only the labels around a vertex and the sweep's direction.
    If neither the vertex nor a neighbour changed in sweeps s-1 and s-2, those
    labels are the ones sweep s-2 saw, in the same direction, and sweep s-2
    left the vertex where it was (by induction when it was itself skipped),
    so evaluating it in sweep s would not move it either.
"""
import numpy as np
import pytest

import bruteforce as bf
import graphgen
import oracle


def tiny_cases(count, nmax, p_lo, p_hi, seed0):
    for t in range(count):
        rng = np.random.default_rng(seed0 + t)
        n = int(rng.integers(2, nmax + 1))
        edges = bf.random_graph(rng, n, float(rng.uniform(p_lo, p_hi)), 5, bool(t % 2))
        if edges:
            yield n, edges


@pytest.mark.parametrize("lpa", [False, True], ids=["louvain", "lpa"])
def test_pruned_level_equals_bruteforce_replay(lpa):
    mode = oracle.LPA if lpa else oracle.LOUVAIN
    nmax, count = (30, 120) if lpa else (11, 160)
    cases = 0
    for n, edges in tiny_cases(count, nmax, 0.1, 0.6, 9100 if lpa else 9300):
        A = bf.dense_adjacency(n, edges)
        adj = oracle.adjacency(bf.to_csr(n, edges))
        for prune in (False, True):
            c, mv = oracle.local_move(adj, mode, 20, 0, prune)
            want_c, want_mv = bf.local_move(A, lpa, prune, 20, 0)
            assert list(c) == want_c and list(mv) == want_mv, (n, edges, prune)
        cases += 1
    assert cases > count // 2


def test_pruning_changes_louvain_somewhere():
    """The rule is a heuristic for Louvain (community volumes change without any
    label change nearby): on some tiny graph the pruned level must differ from
    the full one, otherwise the replay test above would not exercise it."""
    differ = 0
    for n, edges in tiny_cases(160, 11, 0.1, 0.6, 9300):
        A = bf.dense_adjacency(n, edges)
        full = bf.local_move(A, False, False)
        pruned = bf.local_move(A, False, True)
        differ += full != pruned
    assert differ > 0


@pytest.mark.parametrize("maker", ["sbm", "rmat", "rmat_w", "random"])
def test_pruned_lpa_equals_full_lpa(maker):
    for seed in range(3):
        if maker == "sbm":
            g = graphgen.sbm(1500, 40, 0.08, 0.002, seed=seed)
        elif maker == "rmat":
            g = graphgen.rmat(12, seed=seed)
        elif maker == "rmat_w":
            g = graphgen.rmat(11, seed=seed)
            g.weights = graphgen.pair_weights(g, 1, 9, seed=seed)
        else:
            rng = np.random.default_rng(40 + seed)
            g = bf.to_csr(300, bf.random_graph(rng, 300, 0.02, 6, True))
        full = oracle.lpa(g)
        pruned = oracle.lpa(g, prune=True)
        assert np.array_equal(full.labels, pruned.labels) and list(full.moves) == list(pruned.moves)


def test_pruned_worked_trace_golden():
    """Two triangles joined by a bridge: every vertex that matters stays active,
    so the pruned level repeats the full trace (moves 3, 1, 0, 0 on level 0;
    final Q = 5/14)."""
    edges = [(0, 1, 1), (0, 2, 1), (1, 2, 1), (3, 4, 1), (3, 5, 1), (4, 5, 1), (2, 3, 1)]
    r = oracle.louvain(bf.to_csr(6, edges), prune=True)
    assert list(r.levels[0].moves) == [3, 1, 0, 0]
    assert list(r.final_labels) == [0, 0, 0, 1, 1, 1]
    assert (r.q_int, r.M) == (70, 14)


@pytest.mark.parametrize("seed", [0, 1])
def test_pruned_louvain_invariants(seed):
    g = graphgen.sbm(2000, 50, 0.06, 0.001, seed=seed)
    r = oracle.louvain(g, prune=True)
    adj = oracle.adjacency(g)
    q, M = oracle.modularity_int(adj, r.final_labels)
    assert (q, M) == (r.q_int, r.M)
    qs = [lv.q_end for lv in r.accepted]
    assert qs == sorted(qs) and all(lv.q_end > lv.q_start for lv in r.accepted)
    for lv in r.accepted:
        lab = lv.labels
        first = np.unique(lab, return_index=True)[1]
        assert np.array_equal(np.sort(first), first) and lab.max() + 1 == lv.n_next
