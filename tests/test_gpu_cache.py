"""The entry cache (per CSR entry, the neighbour's (community, volume) pair of
the previous sweep, rewritten after each commit only where a pair changed)
against the oracle.  cache_pct=100 makes every sweep after the first two read
the cache whatever the share of changed pairs, so each case below runs
mostly on cached sweeps; cached_sweeps checks that it did.  Results must be
bit-identical to the oracle's, as without the cache."""
import sys

import numpy as np
import pytest

import bruteforce as bf
import graphgen
import oracle
import paper_2507_06471_amd as lvp

pytestmark = pytest.mark.gpu

ALWAYS = {"cache_pct": 100}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check_louvain(g, tuning=ALWAYS, keep_order=False, device=False, hipgraph=True, timing=False, keep_graphs=False,
                  max_sweeps=20):
    say(f"louvain {g.name or 'graph'} n={g.n} nnz={g.nnz} tuning={tuning} keep_order={keep_order}")
    want = oracle.louvain(g, max_sweeps=max_sweeps, keep_graphs=keep_graphs)
    with lvp.Graph.from_csr(g, keep_order=keep_order, device=device) as dg:
        got = lvp.louvain(dg, max_sweeps=max_sweeps, tuning=tuning, hipgraph=hipgraph, timing=timing,
                          keep_graphs=keep_graphs)
    assert len(got.levels) == len(want.levels)
    for a, b in zip(got.levels, want.levels):
        assert a.moves == [int(x) for x in b.moves]
        assert (a.info["n_next"], a.info["q_start"], a.info["q_end"]) == (b.n_next, b.q_start, b.q_end)
        if b.accepted:
            assert np.array_equal(a.labels, b.labels)
    assert np.array_equal(got.final_labels, want.final_labels)
    assert got.q_int == want.q_int
    if keep_graphs:
        for lvl, a in enumerate(got.accepted):
            co = want.graphs[lvl + 1]
            off, idx, w = a.graph
            assert np.array_equal(off, co.off) and np.array_equal(idx, co.idx) and np.array_equal(w, co.a)
    return got


def check_lpa(g, tuning=ALWAYS, keep_order=False):
    want = oracle.lpa(g)
    with lvp.Graph.from_csr(g, keep_order=keep_order) as dg:
        got = lvp.lpa(dg, tuning=tuning)
    assert got.moves == [int(x) for x in want.moves]
    assert np.array_equal(got.labels, want.labels)
    assert got.info["q_end"] == want.q_int
    return got


def cached(level0_info):
    return level0_info["cached_sweeps"]


@pytest.mark.parametrize("seed", range(24))
def test_tiny_graphs_with_loops_and_weights(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 60))
    g = bf.to_csr(n, bf.random_graph(rng, n, float(rng.uniform(0.05, 0.4)), 9, True))
    g.name = f"tiny{seed}"
    got = check_louvain(g, keep_graphs=True)
    sw = got.levels[0].info["sweeps"]
    assert cached(got.levels[0].info) == max(0, sw - 2)
    lp = check_lpa(g)
    assert cached(lp.info) == max(0, lp.info["sweeps"] - 2)


def test_sbm_4096():
    got = check_louvain(graphgen.sbm(4096, 128, 0.05, 0.0005, seed=1), keep_graphs=True)
    assert cached(got.levels[0].info) > 0


@pytest.mark.parametrize("scale", [12, 16, 18])
def test_rmat(scale):
    g = graphgen.rmat(scale, seed=2)
    got = check_louvain(g)
    assert cached(got.levels[0].info) == got.levels[0].info["sweeps"] - 2
    assert got.levels[0].info["refreshed_entries"] > 0
    lp = check_lpa(g)
    assert cached(lp.info) > 0


def test_rmat18_default_threshold():
    # default threshold (10 % of the entries changed): R-MAT's pairs settle
    # after a few sweeps, so the later sweeps of level 0 read the cache
    g = graphgen.rmat(18, seed=2)
    got = check_louvain(g, tuning=None)
    assert cached(got.levels[0].info) >= 5, got.levels[0].info["cached_sweeps"]
    check_lpa(g, tuning=None)


def test_lfr_weighted():
    g, _ = graphgen.lfr(30000, kmax=1500, smin=30, smax=3000, seed=3)
    got = check_louvain(g, keep_graphs=True)
    assert cached(got.levels[0].info) > 0
    check_lpa(g)


@pytest.mark.parametrize("tuning", [
    {"block_max": 600, "hub_mode": 2, "part_keys": 500},                      # bucketed partitions
    {"block_max": 64, "hub_mode": 2, "part_keys": 32, "part_slots": 64},       # many buckets, overflows
    {"block_max": 600, "hub_mode": 1, "part_keys": 500},                      # compact partitions
    {"sub_max": 8, "wave_max": 8, "block_max": 8, "part_keys": 40, "part_slots": 64, "hub_mode": 1},
    {"sub_max": 1, "wave_max": 2, "block_max": 3, "part_keys": 256},
    {"sub_max": 4, "wave_max": 64, "block_max": 4096, "part_keys": 4096},
])
def test_every_class_and_partition_path(tuning):
    t = dict(tuning, cache_pct=100)
    g = graphgen.rmat(14, seed=5)
    got = check_louvain(g, tuning=t)
    assert cached(got.levels[0].info) > 0
    check_lpa(g, tuning=t)


def test_weighted_bucketed_partitions():
    g, _ = graphgen.lfr(20000, kmax=1500, smin=30, smax=3000, seed=7)
    t = {"block_max": 100, "hub_mode": 2, "part_keys": 40, "part_slots": 64, "cache_pct": 100}
    check_louvain(g, tuning=t)
    check_lpa(g, tuning=t)


def test_input_order_storage_and_device_input():
    g = graphgen.rmat(14, seed=6)
    got = check_louvain(g, keep_order=True)
    assert cached(got.levels[0].info) > 0
    check_lpa(g, keep_order=True)
    check_louvain(g, device=True)


def test_eager_and_timed_drivers():
    g = graphgen.rmat(14, seed=8)
    a = check_louvain(g, hipgraph=False)
    b = check_louvain(g, timing=True)
    assert cached(a.levels[0].info) > 0 and cached(b.levels[0].info) > 0
    info = b.levels[0].info
    names = lvp.KERNEL_NAMES
    assert info["kern_launches"][names.index("cache/refresh")] == info["sweeps"]
    assert info["kern_launches"][names.index("commit")] == info["sweeps"]


def test_without_cache_same_results():
    g = graphgen.rmat(16, seed=9)
    with lvp.Graph.from_csr(g) as dg:
        a = lvp.louvain(dg, tuning=ALWAYS)
        b = lvp.louvain(dg, tuning=ALWAYS, cache=False)
        la = lvp.lpa(dg, tuning=ALWAYS)
        lb = lvp.lpa(dg, tuning=ALWAYS, cache=False)
    assert cached(a.levels[0].info) > 0 and cached(b.levels[0].info) == 0
    assert np.array_equal(a.final_labels, b.final_labels) and a.q_int == b.q_int
    assert [lv.moves for lv in a.levels] == [lv.moves for lv in b.levels]
    assert np.array_equal(la.labels, lb.labels) and la.moves == lb.moves
    with lvp.Graph.from_csr(g, entry_cache=False) as dg:
        c = lvp.louvain(dg, tuning=ALWAYS)
    assert cached(c.levels[0].info) == 0
    assert np.array_equal(a.final_labels, c.final_labels)


def test_pruned_and_asynchronous_runs_do_not_use_it():
    g = graphgen.rmat(14, seed=10)
    with lvp.Graph.from_csr(g) as dg:
        p = lvp.louvain(dg, tuning=ALWAYS, prune=True)
        q = lvp.louvain(dg, tuning=ALWAYS, asynchronous=True)
    assert cached(p.levels[0].info) == 0 and cached(q.levels[0].info) == 0
    want = oracle.louvain(g, prune=True)
    assert np.array_equal(p.final_labels, want.final_labels)


def test_packed_batch():
    rng = np.random.default_rng(21)
    gs = []
    for t in range(9):
        if t % 3 == 0:
            gs.append(graphgen.rmat(int(rng.integers(8, 13)), seed=100 + t))
        elif t % 3 == 1:
            gs.append(graphgen.sbm(1024, 128, 0.08, 0.002, seed=200 + t))
        else:
            n = int(rng.integers(5, 50))
            gs.append(bf.to_csr(n, bf.random_graph(rng, n, 0.2, 5, True)))
    with lvp.Graph.batch(gs) as bg:
        got = lvp.louvain(bg, tuning=ALWAYS)
        lp = lvp.lpa(bg, tuning=ALWAYS)
    for i, g in enumerate(gs):
        want = oracle.louvain(g)
        assert np.array_equal(got[i].final_labels, want.final_labels), i
        assert got[i].q_int == want.q_int
        assert [lv.moves for lv in got[i].levels] == [[int(x) for x in lv.moves] for lv in want.levels], i
        wl = oracle.lpa(g)
        assert np.array_equal(lp[i].labels, wl.labels) and lp[i].moves == [int(x) for x in wl.moves], i


def test_edge_list_graph():
    u, v = graphgen.rmat_edges(12, 16, seed=3)
    with lvp.Graph.from_edges(1 << 12, u, v, drop_loops=True, simple=True) as eg:
        off, idx, _ = eg.csr()
        got = lvp.louvain(eg, tuning=ALWAYS)
    g = graphgen.CSR(1 << 12, off, idx, None)
    want = oracle.louvain(g)
    assert cached(got.levels[0].info) > 0
    assert np.array_equal(got.final_labels, want.final_labels) and got.q_int == want.q_int
