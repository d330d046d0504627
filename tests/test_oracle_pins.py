"""Pins for the CPU oracle: each check compares it with something other than itself.

- brute force on tiny graphs: textbook modularity in exact fractions, and
  per-vertex decisions whose gains are measured as Q(after) - Q(before);
- library routines: networkx modularity, scipy S^T A S, numpy first-occurrence;
- closed forms: two cliques joined by a bridge, disjoint cliques;
- a hand-derived worked trace (tests/golden);
- invariants of the method at any size.
"""
from fractions import Fraction
import os

import numpy as np
import pytest

import bruteforce as bf
import graphgen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny_cases(count, seed0=0, nmax=8, loops=True):
    for s in range(count):
        rng = np.random.default_rng(seed0 + s)
        n = int(rng.integers(1, nmax + 1))
        edges = bf.random_graph(rng, n, float(rng.uniform(0.2, 0.9)), 5, loops)
        yield rng, n, edges


def test_modularity_matches_textbook_fraction():
    """Q_int / M^2 equals the Newman-Girvan pair sum exactly (Section II-C)."""
    checked = 0
    for rng, n, edges in tiny_cases(300):
        if not edges:
            continue
        A = bf.dense_adjacency(n, edges)
        adj = oracle.adjacency(bf.to_csr(n, edges))
        for _ in range(3):
            labels = rng.integers(0, n, size=n)
            q_int, M = oracle.modularity_int(adj, labels)
            assert M == sum(map(sum, A))
            assert Fraction(q_int, M * M) == bf.modularity(A, labels)
            checked += 1
    assert checked > 500


@pytest.mark.parametrize("lpa", [False, True])
def test_sweep_decisions_match_bruteforce_gain(lpa):
    """Every vertex's decision equals the brute-force rule on random partitions.

    The brute force measures each candidate's gain by recomputing Q, so a
    wrong sign, a dropped -k_i term in stay, or a transposed operand in the
    integer score makes some decision differ.
    """
    mode = oracle.LPA if lpa else oracle.LOUVAIN
    mism = 0
    total = 0
    for rng, n, edges in tiny_cases(250, seed0=1000):
        if not edges:
            continue
        A = bf.dense_adjacency(n, edges)
        adj = oracle.adjacency(bf.to_csr(n, edges))
        k, M = oracle.degrees(adj)
        for trial in range(3):
            labels = rng.integers(0, n, size=n) if trial else np.arange(n)
            sigma = np.bincount(labels, weights=k, minlength=n).astype(np.int64)
            for down in (True, False):
                got, mv = oracle.sweep(adj, labels, sigma, oracle.DOWN if down else oracle.UP, mode)
                want = bf.sweep(A, list(labels), down, lpa)
                mism += int(np.sum(got != np.array(want)))
                assert mv == int(np.sum(got != labels))
                total += n
    assert mism == 0
    assert total > 1000


def test_decide_vertices_equals_full_sweep():
    g = graphgen.rmat(10, seed=7)
    adj = oracle.adjacency(g)
    k, M = oracle.degrees(adj)
    rng = np.random.default_rng(3)
    c = np.arange(g.n, dtype=np.int32)
    full, _ = oracle.sweep(adj, c, k, oracle.DOWN)
    verts = rng.choice(g.n, 200, replace=False)
    part = oracle.decide_vertices(adj, verts, c, k, oracle.DOWN)
    assert np.array_equal(part, full[verts])


def test_modularity_matches_networkx():
    nx = pytest.importorskip("networkx")
    for rng, n, edges in tiny_cases(60, seed0=77, nmax=12):
        if not edges:
            continue
        G = nx.Graph()
        G.add_nodes_from(range(n))
        for u, v, w in edges:
            G.add_edge(u, v, weight=w)
        labels = rng.integers(0, max(1, n // 2), size=n)
        comms = [set(np.flatnonzero(labels == c).tolist()) for c in np.unique(labels)]
        q_nx = nx.community.modularity(G, comms, weight="weight")
        _, _, q = oracle.modularity(bf.to_csr(n, edges), labels)
        assert abs(q - q_nx) <= 1e-12 * max(1.0, abs(q_nx))


def test_aggregation_matches_scipy_StAS():
    sp = pytest.importorskip("scipy.sparse")
    g = graphgen.sbm(600, 50, 0.2, 0.01, seed=11)
    g.weights = graphgen.pair_weights(g, 1, 8, seed=11)
    adj = oracle.adjacency(g)
    c, _ = oracle.local_move(adj)
    labels, n2 = oracle.renumber(c)
    coarse = oracle.aggregate(adj, labels, n2)
    A = sp.csr_matrix((adj.a.astype(np.int64), adj.idx, adj.off), shape=(adj.n, adj.n))
    S = sp.csr_matrix((np.ones(adj.n, np.int64), (np.arange(adj.n), labels)), shape=(adj.n, n2))
    ref = (S.T @ A @ S).tocsr()
    ref.sort_indices()
    assert np.array_equal(coarse.off, ref.indptr)
    assert np.array_equal(coarse.idx, ref.indices)
    assert np.array_equal(coarse.a, ref.data)


def test_renumber_is_first_occurrence_rank():
    rng = np.random.default_rng(5)
    for _ in range(50):
        n = int(rng.integers(1, 300))
        c = rng.integers(0, n, size=n).astype(np.int32)
        lab, n2 = oracle.renumber(c)
        uniq, first = np.unique(c, return_index=True)
        rank = np.empty(len(uniq), np.int64)
        rank[np.argsort(first)] = np.arange(len(uniq))
        expect = rank[np.searchsorted(uniq, c)]
        assert n2 == len(uniq)
        assert np.array_equal(lab, expect)


def clique_edges(p, base=0):
    return [(base + i, base + j, 1) for i in range(p) for j in range(i + 1, p)]


@pytest.mark.parametrize("p", [3, 4, 5, 6, 8])
def test_two_cliques_with_bridge_closed_form(p):
    """Two K_p joined by one edge: the two cliques, Q = 2C(p,2)/(2C(p,2)+1) - 1/2."""
    edges = clique_edges(p) + clique_edges(p, p) + [(p - 1, p, 1)]
    r = oracle.louvain(bf.to_csr(2 * p, edges))
    assert list(r.final_labels) == [0] * p + [1] * p
    c2 = p * (p - 1) // 2
    assert Fraction(r.q_int, r.M * r.M) == Fraction(2 * c2, 2 * c2 + 1) - Fraction(1, 2)


@pytest.mark.parametrize("kp", [(2, 3), (3, 4), (5, 5), (4, 7)])
def test_disjoint_cliques_closed_form(kp):
    """k disjoint K_p: one community per clique, Q = 1 - 1/k."""
    k, p = kp
    edges = sum((clique_edges(p, b * p) for b in range(k)), [])
    r = oracle.louvain(bf.to_csr(k * p, edges))
    assert list(r.final_labels) == [b for b in range(k) for _ in range(p)]
    assert Fraction(r.q_int, r.M * r.M) == 1 - Fraction(1, k)
    lp = oracle.lpa(bf.to_csr(k * p, edges))
    assert list(lp.labels) == [b for b in range(k) for _ in range(p)]


def test_lpa_path_of_two():
    lp = oracle.lpa(bf.to_csr(2, [(0, 1, 1)]))
    assert list(lp.labels) == [0, 0]
    assert list(lp.moves) == [1, 0, 0]


def parse_golden(path):
    out = {"sweeps": []}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        head, *rest = line.split()
        if head == "edges":
            out["edges"] = [tuple(map(int, e.split("-"))) for e in rest]
        elif head == "sweep":
            parts = line.split("|")
            s, d, mv = parts[0].split()[1:4]
            out["sweeps"].append((int(s), d, int(mv), list(map(int, parts[1].split())), int(parts[2])))
        elif head == "final_q":
            out["final_q"] = Fraction(rest[0])
        elif head == "level1":
            out["level1"] = dict(zip(rest[::2], map(int, rest[1::2])))
        elif head == "level0_labels":
            out["level0_labels"] = list(map(int, rest))
        else:
            out[head] = int(rest[0])
    return out


def test_worked_trace_golden():
    gd = parse_golden(os.path.join(GOLDEN, "two_triangles_bridge.txt"))
    n = gd["n"]
    g = bf.to_csr(n, [(u, v, 1) for u, v in gd["edges"]])
    adj = oracle.adjacency(g)
    k, M = oracle.degrees(adj)
    assert M == gd["M"]
    assert oracle.singleton_qint(adj) == gd["q_singleton"]
    c = np.arange(n, dtype=np.int32)
    sigma = k.copy()
    for s, d, mv, labels, qint in gd["sweeps"]:
        c, got_mv = oracle.sweep(adj, c, sigma, oracle.DOWN if d == "down" else oracle.UP)
        sigma = np.bincount(c, weights=k, minlength=n).astype(np.int64)
        assert got_mv == mv and list(c) == labels
        assert oracle.modularity_int(adj, c)[0] == qint
    r = oracle.louvain(g)
    assert list(r.levels[0].labels) == gd["level0_labels"]
    assert list(r.levels[0].moves) == [s[2] for s in gd["sweeps"]]
    l1 = r.levels[1]
    assert (l1.q_start, l1.q_end, int(l1.accepted)) == (gd["level1"]["q_start"], gd["level1"]["q_end"],
                                                        gd["level1"]["accepted"])
    assert Fraction(r.q_int, r.M * r.M) == gd["final_q"]


def check_invariants(g, r):
    adj = oracle.adjacency(g)
    graphs = r.graphs
    prev_q = None
    for lvl, rec in enumerate(r.accepted):
        a_l, a_n = graphs[lvl], graphs[lvl + 1]
        # total weight preserved and k' = Sigma_tot of the level's partition
        assert int(a_n.a.astype(np.int64).sum()) == r.M
        k_l, _ = oracle.degrees(a_l)
        k_n, _ = oracle.degrees(a_n)
        assert np.array_equal(k_n, np.bincount(rec.labels, weights=k_l, minlength=rec.n_next).astype(np.int64))
        # coarsening preserves Q_int exactly
        assert oracle.modularity_int(a_l, rec.labels)[0] == oracle.singleton_qint(a_n) == rec.q_end
        # labels contiguous, first-occurrence order
        _, first = np.unique(rec.labels, return_index=True)
        assert np.all(np.diff(rec.labels[np.sort(first)]) == 1) and rec.labels[0] == 0
        assert rec.q_end > rec.q_start
        if prev_q is not None:
            assert rec.q_start == prev_q
        prev_q = rec.q_end
    assert oracle.modularity_int(adj, r.final_labels)[0] == r.q_int


@pytest.mark.parametrize("maker", ["sbm", "rmat", "lfr"])
def test_invariants(maker):
    if maker == "sbm":
        g = graphgen.sbm(4096, 128, 0.05, 0.0005, seed=1)
    elif maker == "rmat":
        g = graphgen.rmat(12, seed=2)
    else:
        g, _ = graphgen.lfr(3000, kmax=200, smin=20, smax=300, seed=3)
    r = oracle.louvain(g, keep_graphs=True)
    assert len(r.accepted) >= 1
    check_invariants(g, r)


def test_thread_count_does_not_change_results():
    g = graphgen.rmat(12, seed=9)
    t0 = oracle.num_threads()
    try:
        oracle.set_threads(1)
        r1 = oracle.louvain(g)
        oracle.set_threads(max(2, t0))
        r2 = oracle.louvain(g)
    finally:
        oracle.set_threads(t0)
    assert np.array_equal(r1.final_labels, r2.final_labels)
    assert [list(l.moves) for l in r1.levels] == [list(l.moves) for l in r2.levels]


def test_sbm_quality_sanity():
    """Planted-partition SBM (4096 vertices, 32 blocks): a sanity bound, not parity."""
    g = graphgen.sbm(4096, 128, 0.05, 0.0005, seed=1)
    planted = np.arange(g.n) // 128
    _, _, q_planted = oracle.modularity(g, planted)
    r = oracle.louvain(g)
    assert q_planted > 0.7
    assert r.q > 0.65


def test_rejects_bad_weights_and_overflow():
    g = graphgen.from_edges(3, [0, 1], [1, 2], [1, 0])
    with pytest.raises(ValueError):
        oracle.adjacency(g)
    big = graphgen.from_edges(2, [0], [1], [2**30])
    with pytest.raises(ValueError):
        oracle.adjacency(big)  # M = 2^31 exceeds the exact-integer bound
