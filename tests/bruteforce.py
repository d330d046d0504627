"""Brute-force definitions used to pin the oracle on tiny graphs.

Nothing here reuses the oracle's integer formulas.  Modularity is the textbook
Newman-Girvan sum over all vertex pairs (paper, Section II-C, citing Newman and
Girvan 2004), in exact ``fractions.Fraction`` arithmetic, and a move's gain is
measured as Q(after) - Q(before) by recomputing Q from scratch.  The weighted
degree counts a loop twice (Section II-A), so a loop of weight w contributes
2w to A_vv here, built straight from the edge list.
"""
from __future__ import annotations

from fractions import Fraction
from typing import Dict, List, Sequence, Tuple

import numpy as np


def dense_adjacency(n: int, edges: Sequence[Tuple[int, int, int]]) -> List[List[int]]:
    """Symmetric A from undirected weighted edges; a loop (v, v, w) gives A_vv = 2w."""
    A = [[0] * n for _ in range(n)]
    for u, v, w in edges:
        if u == v:
            A[u][u] += 2 * w
        else:
            A[u][v] += w
            A[v][u] += w
    return A


def modularity(A: List[List[int]], labels: Sequence[int]) -> Fraction:
    """Q = (1/2m) sum_ij [A_ij - k_i k_j / 2m] delta(c_i, c_j), exact."""
    n = len(A)
    k = [sum(row) for row in A]
    two_m = sum(k)
    if two_m == 0:
        return Fraction(0)
    q = Fraction(0)
    for i in range(n):
        for j in range(n):
            if labels[i] == labels[j]:
                q += Fraction(A[i][j]) - Fraction(k[i] * k[j], two_m)
    return q / two_m


def move_gain(A, labels, i: int, target: int) -> Fraction:
    """Q(after moving i alone to community `target`) - Q(before)."""
    after = list(labels)
    after[i] = target
    return modularity(A, after) - modularity(A, labels)


def neighbour_communities(A, labels, i: int) -> Dict[int, int]:
    """community -> summed weight of edges from i to its members other than i."""
    out: Dict[int, int] = {}
    for j in range(len(A)):
        if j != i and A[i][j] > 0:
            out[labels[j]] = out.get(labels[j], 0) + A[i][j]
    return out


def decide(A, labels, i: int, down: bool, lpa: bool) -> int:
    """Brute-force decision of vertex i against partition `labels`.

    Louvain: the gain of every neighbouring community is measured by
    recomputing Q; the best (ties to the smallest id) is taken if its gain is
    positive and it lies in the sweep's direction.  LPA: the label with the
    largest neighbour weight, taken if heavier than the own label's weight and
    in the sweep's direction.
    """
    cur = labels[i]
    nb = neighbour_communities(A, labels, i)
    cands = sorted(c for c in nb if c != cur)
    if not cands:
        return cur
    if lpa:
        vals = {c: Fraction(nb[c]) for c in cands}
        stay = Fraction(nb.get(cur, 0))
    else:
        vals = {c: move_gain(A, labels, i, c) for c in cands}
        stay = Fraction(0)
    best = max(cands, key=lambda c: (vals[c], -c))
    if vals[best] <= stay:
        return cur
    if down and best > cur:
        return cur
    if not down and best < cur:
        return cur
    return best


def sweep(A, labels, down: bool, lpa: bool = False) -> List[int]:
    return [decide(A, labels, i, down, lpa) for i in range(len(A))]


def local_move(A, lpa: bool = False, prune: bool = False, max_sweeps: int = 20, theta: int = 0):
    """One level of synchronous sweeps from singletons, every decision by
    `decide`; returns (labels, per-sweep mover counts).

    With `prune`, the set of vertices evaluated in sweep s is read off the
    label history: every vertex while s <= 2, afterwards vertex i only if some
    vertex of {i} and its neighbours carries a different label after sweep
    s-1 than after s-2, or after s-2 than after s-3.  Other vertices keep
    their label.  The level ends after two consecutive sweeps with at most
    `theta` movers, or after `max_sweeps`.
    """
    n = len(A)
    hist = [list(range(n))]  # hist[t] = labels after sweep t

    def changed_in(t: int, j: int) -> bool:
        return t >= 1 and hist[t][j] != hist[t - 1][j]

    moves: List[int] = []
    for s in range(1, max_sweeps + 1):
        cur = hist[-1]
        down = s % 2 == 1
        nxt = []
        for i in range(n):
            if prune and s > 2:
                closed = [i] + [j for j in range(n) if j != i and A[i][j] > 0]
                if not any(changed_in(s - 1, j) or changed_in(s - 2, j) for j in closed):
                    nxt.append(cur[i])
                    continue
            nxt.append(decide(A, cur, i, down, lpa))
        moves.append(sum(a != b for a, b in zip(cur, nxt)))
        hist.append(nxt)
        if s >= 2 and moves[-1] <= theta and moves[-2] <= theta:
            break
    return hist[-1], moves


def random_graph(rng: np.random.Generator, n: int, p: float, wmax: int, loops: bool):
    edges = []
    for u in range(n):
        for v in range(u, n):
            if u == v and not loops:
                continue
            if rng.random() < p:
                edges.append((u, v, int(rng.integers(1, wmax + 1))))
    return edges


def to_csr(n: int, edges):
    """Caller-convention CSR (a loop entry carries its own weight w)."""
    import graphgen

    if not edges:
        return graphgen.CSR(n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32))
    u, v, w = zip(*edges)
    return graphgen.from_edges(n, list(u), list(v), list(w))
