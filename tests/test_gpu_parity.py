"""GPU path vs the CPU oracle through the C ABI: bit-exact labels at every level,
identical per-sweep move counts, identical Q_int (so FP64 Q is identical too)."""
import sys

import numpy as np
import pytest

import bruteforce as bf
import graphgen
import oracle
import paper_2507_06471_amd as lvp

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def compare_louvain(g, tuning=None, max_sweeps=20, max_levels=32, keep_graphs=False, device=False, keep_order=False,
                    prune=False, hipgraph=True, timing=False):
    say(f"case {g.name or 'graph'} n={g.n} nnz={g.nnz} tuning={tuning} keep_order={keep_order} prune={prune}")
    want = oracle.louvain(g, max_sweeps=max_sweeps, max_levels=max_levels, keep_graphs=keep_graphs, prune=prune)
    with lvp.Graph.from_csr(g, device=device, keep_order=keep_order) as dg:
        got = lvp.louvain(dg, max_sweeps=max_sweeps, max_levels=max_levels, keep_graphs=keep_graphs,
                          tuning=tuning, prune=prune, hipgraph=hipgraph, timing=timing)
    assert got.M == want.M
    assert len(got.levels) == len(want.levels)
    for lvl, (a, b) in enumerate(zip(got.levels, want.levels)):
        assert a.moves == [int(x) for x in b.moves], f"level {lvl} moves"
        assert (a.info["n"], a.info["n_next"], a.info["q_start"], a.info["q_end"]) == (
            b.n, b.n_next, b.q_start, b.q_end), f"level {lvl} stats"
        assert bool(a.info["accepted"]) == b.accepted
        if b.accepted:
            assert np.array_equal(a.labels, b.labels), f"level {lvl} labels"
    assert np.array_equal(got.final_labels, want.final_labels)
    assert got.q_int == want.q_int
    assert got.q == want.q  # both divide the same integers the same way
    if keep_graphs:
        for lvl, a in enumerate(got.accepted):
            co = want.graphs[lvl + 1]
            off, idx, w = a.graph
            assert np.array_equal(off, co.off) and np.array_equal(idx, co.idx) and np.array_equal(w, co.a)
    return got, want


def compare_lpa(g, max_sweeps=20, threshold=0, tuning=None, keep_order=False, prune=False):
    say(f"lpa case {g.name or 'graph'} n={g.n} nnz={g.nnz} prune={prune}")
    want = oracle.lpa(g, max_sweeps=max_sweeps, theta=threshold, prune=prune)
    with lvp.Graph.from_csr(g, keep_order=keep_order) as dg:
        got = lvp.lpa(dg, max_sweeps=max_sweeps, threshold=threshold, tuning=tuning, prune=prune)
    assert got.moves == [int(x) for x in want.moves]
    assert np.array_equal(got.labels, want.labels)
    assert got.info["q_end"] == want.q_int


def test_worked_trace():
    edges = [(0, 1, 1), (0, 2, 1), (1, 2, 1), (3, 4, 1), (3, 5, 1), (4, 5, 1), (2, 3, 1)]
    got, _ = compare_louvain(bf.to_csr(6, edges), keep_graphs=True)
    assert got.levels[0].moves == [3, 1, 0, 0]
    assert list(got.final_labels) == [0, 0, 0, 1, 1, 1]


@pytest.mark.parametrize("seed", range(40))
def test_tiny_random_graphs_with_loops_and_weights(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 60))
    edges = bf.random_graph(rng, n, float(rng.uniform(0.02, 0.4)), 9, True)
    g = bf.to_csr(n, edges)
    g.name = f"tiny{seed}"
    compare_louvain(g, keep_graphs=True)
    compare_lpa(g)


def test_sbm_4096_planted_partition():
    g = graphgen.sbm(4096, 128, 0.05, 0.0005, seed=1)
    got, _ = compare_louvain(g, keep_graphs=True)
    assert got.q > 0.65


@pytest.mark.parametrize("scale", [12, 16, 18])
def test_rmat(scale):
    g = graphgen.rmat(scale, seed=2)
    compare_louvain(g)


def test_rmat_lpa():
    compare_lpa(graphgen.rmat(16, seed=2))


def test_lfr_weighted():
    g, _ = graphgen.lfr(30000, kmax=1500, smin=30, smax=3000, seed=3)
    compare_louvain(g, keep_graphs=True)
    compare_lpa(g)


@pytest.mark.parametrize("tuning", [
    {"sub_max": 1, "wave_max": 2, "block_max": 3, "part_keys": 256},    # nearly all partitioned
    {"sub_max": 8, "wave_max": 8, "block_max": 8, "part_keys": 40, "part_slots": 64},  # forces overflows
    {"sub_max": 8, "wave_max": 8, "block_max": 8, "part_keys": 40, "part_slots": 64, "hub_mode": 1},
    {"block_max": 600, "hub_mode": 1, "part_keys": 500},                   # compact re-reading partitions
    {"sub_max": 32, "wave_max": 128, "block_max": 512, "part_keys": 1000},
    {"sub_max": 4, "wave_max": 64, "block_max": 4096, "part_keys": 4096},
    {"block_max": 600, "hub_mode": 2, "part_keys": 500},                   # bucketed partitions
    {"block_max": 300, "hub_mode": 2, "part_keys": 100, "part_slots": 128},  # buckets + overflows
    {"block_max": 64, "hub_mode": 2, "part_keys": 32, "part_slots": 64},     # many small buckets
    {"block_max": 64, "hub_mode": 2, "part_keys": 48, "hub_chunk": 1024},
    {"block_max": 300, "hub_mode": 2, "part_keys": 200, "hub_chunk": 4096},
    {"agg_sort": 1},                                                       # aggregation by sorting only
    {"agg_sort": 1, "block_max": 64, "hub_mode": 2, "part_keys": 48},
])
def test_tuning_never_changes_results(tuning):
    # the class bounds also route coarse vertices between aggregation in LDS
    # and the sorted path for long segments; coarse graphs are compared too
    g = graphgen.rmat(14, seed=5)
    compare_louvain(g, tuning=tuning, keep_graphs=True)
    compare_lpa(g, tuning=tuning)


@pytest.mark.parametrize("tuning", [
    {"block_max": 200, "hub_mode": 2, "part_keys": 64},
    {"block_max": 100, "hub_mode": 2, "part_keys": 40, "part_slots": 64},
])
def test_weighted_bucketed_partitions(tuning):
    g, _ = graphgen.lfr(20000, kmax=1500, smin=30, smax=3000, seed=7)
    compare_louvain(g, tuning=tuning)
    compare_lpa(g, tuning=tuning)


def hub_star_graph(leaves=40000, seed=61):
    # vertex 0 joins every leaf; leaves form a ring with random chords, so
    # communities form along it while the hub row stays 40,000 entries long
    rng = np.random.default_rng(seed)
    ring = np.arange(1, leaves + 1)
    u = np.concatenate([np.zeros(leaves, dtype=np.int64), ring, rng.integers(1, leaves + 1, size=leaves // 2)])
    v = np.concatenate([ring, np.roll(ring, -1), rng.integers(1, leaves + 1, size=leaves // 2)])
    keep = u != v
    return graphgen.from_edges(leaves + 1, u[keep], v[keep], keep_loops=False)


@pytest.mark.parametrize("hub_chunk", [1024, 2048, 4096])
def test_hub_with_more_partitions_than_the_small_count_array(hub_chunk):
    # part_keys 32 splits the 40,000-entry hub row into 1,250 partitions, more
    # than the scatter pass's small per-partition count array takes
    g = hub_star_graph()
    g = graphgen.CSR(g.n, g.offsets, g.indices, None, "hub star")
    tuning = {"block_max": 64, "hub_mode": 2, "part_keys": 32, "part_slots": 2048, "hub_chunk": hub_chunk}
    compare_louvain(g, tuning=tuning)
    compare_lpa(g, tuning=tuning)


def test_device_resident_input():
    pytest.importorskip("torch")
    compare_louvain(graphgen.rmat(12, seed=8), device=True)


def test_labels_into_device_buffers():
    # final Louvain labels and LPA labels written straight into device tensors
    torch = pytest.importorskip("torch")
    g = graphgen.rmat(13, seed=9)
    say(f"case rmat13 out= device buffers n={g.n}")
    want = oracle.louvain(g)
    want_lpa = oracle.lpa(g)
    fin = torch.full((g.n,), -1, dtype=torch.int32, device="cuda")
    lab = torch.full((g.n,), -1, dtype=torch.int32, device="cuda")
    with lvp.Graph.from_csr(g) as dg:
        got = lvp.louvain(dg, level_labels=False, out=fin)
        got_lpa = lvp.lpa(dg, out=lab)
    assert got.final_labels is fin
    assert np.array_equal(fin.cpu().numpy(), want.final_labels) and got.q_int == want.q_int
    assert np.array_equal(lab.cpu().numpy(), want_lpa.labels)
    with lvp.Graph.batch([g, g]) as bg:
        with pytest.raises(ValueError):
            lvp.louvain(bg, out=fin)


@pytest.mark.parametrize("maker", ["rmat", "lfr", "tiny"])
def test_input_order_storage_gives_same_results(maker):
    # LV_KEEP_ORDER stores the input order; the default stores by degree
    if maker == "rmat":
        g = graphgen.rmat(13, seed=21)
    elif maker == "lfr":
        g, _ = graphgen.lfr(8000, kmax=400, smin=20, smax=800, seed=22)
    else:
        rng = np.random.default_rng(23)
        g = bf.to_csr(40, bf.random_graph(rng, 40, 0.2, 9, True))
        g.name = "tiny23"
    compare_louvain(g, keep_graphs=True, keep_order=True)
    compare_lpa(g, keep_order=True)
    rng = np.random.default_rng(24)
    lab = rng.integers(0, max(1, g.n // 3), size=g.n).astype(np.int32)
    with lvp.Graph.from_csr(g) as a, lvp.Graph.from_csr(g, keep_order=True) as b:
        assert lvp.modularity(a, lab) == lvp.modularity(b, lab) == oracle.modularity(g, lab)


def test_modularity_of_arbitrary_labels():
    g = graphgen.rmat(12, seed=4)
    g.weights = graphgen.pair_weights(g, 1, 5, seed=4)
    rng = np.random.default_rng(1)
    with lvp.Graph.from_csr(g) as dg:
        for t in range(5):
            lab = rng.integers(0, max(1, g.n // (t + 1)), size=g.n).astype(np.int32)
            qi, m, q = lvp.modularity(dg, lab)
            wq, wm, wqf = oracle.modularity(g, lab)
            assert (qi, m, q) == (wq, wm, wqf)


@pytest.mark.parametrize("case", ["empty", "single", "no_edges", "loops_only", "star", "clique", "path"])
def test_edge_cases(case):
    if case == "empty":
        g = graphgen.CSR(0, np.zeros(1, np.int32), np.zeros(0, np.int32), None)
    elif case == "single":
        g = graphgen.CSR(1, np.zeros(2, np.int32), np.zeros(0, np.int32), None)
    elif case == "no_edges":
        g = graphgen.CSR(50, np.zeros(51, np.int32), np.zeros(0, np.int32), None)
    elif case == "loops_only":
        g = bf.to_csr(5, [(v, v, v + 1) for v in range(5)])
    elif case == "star":
        g = bf.to_csr(200, [(0, v, 1) for v in range(1, 200)])
    elif case == "clique":
        g = bf.to_csr(40, [(u, v, 1) for u in range(40) for v in range(u + 1, 40)])
    else:
        g = bf.to_csr(100, [(v, v + 1, 1) for v in range(99)])
    g.name = case
    compare_louvain(g)
    if g.n > 0:
        compare_lpa(g)


def test_bad_inputs_rejected():
    off = np.array([0, 1, 2], np.int32)
    # asymmetric: 0->1 without 1->0
    with pytest.raises(lvp.LvError) as ei:
        lvp.Graph(2, off, np.array([1, 1], np.int32))
    assert ei.value.status == 3
    # unsorted row
    with pytest.raises(lvp.LvError) as ei:
        lvp.Graph(3, np.array([0, 2, 3, 4], np.int32), np.array([2, 1, 0, 0], np.int32), validate=False)
    assert ei.value.status == 2
    # index out of range
    with pytest.raises(lvp.LvError) as ei:
        lvp.Graph(2, off, np.array([1, 5], np.int32))
    assert ei.value.status == 2
    # zero weight
    with pytest.raises(lvp.LvError) as ei:
        lvp.Graph(2, off, np.array([1, 0], np.int32), np.array([0, 0], np.int32))
    assert ei.value.status == 4
    # volume overflow
    with pytest.raises(lvp.LvError) as ei:
        lvp.Graph(2, off, np.array([1, 0], np.int32), np.array([2**30, 2**30], np.int32))
    assert ei.value.status == 5
    # offsets not ending at nnz / decreasing
    with pytest.raises(lvp.LvError) as ei:
        lvp.Graph(2, np.array([0, 2, 1], np.int32), np.array([1, 0], np.int32))
    assert ei.value.status == 2
    with pytest.raises(lvp.LvError):
        lvp.Graph(2, np.array([1, 1, 2], np.int32), np.array([1, 0], np.int32))


def rejected_first_level_graph():
    """Heavy loops make every move lose (e.g. 80 * 1 - 11 * 62 < 0), so level 0
    is rejected and the singletons stay; vertex 1 has the longest row, so the
    degree-ordered storage puts it first (positions differ from ids)."""
    g = bf.to_csr(3, [(0, 1, 1), (1, 2, 1), (0, 0, 5), (1, 1, 30), (2, 2, 3)])
    g.name = "rejected-first-level"
    return g


def test_first_level_rejected_keeps_singletons():
    g = rejected_first_level_graph()
    got, want = compare_louvain(g)
    assert not want.levels[0].accepted and list(want.final_labels) == [0, 1, 2]
    assert list(got.final_labels) == [0, 1, 2]
    graphs = [graphgen.rmat(8, seed=1), g, graphgen.sbm(300, 30, 0.2, 0.01, seed=2)]
    with lvp.Graph.batch(graphs) as bg:
        rs = lvp.louvain(bg)
    for gg, r in zip(graphs, rs):
        assert np.array_equal(r.final_labels, oracle.louvain(gg).final_labels), gg.name
    with lvp.Server() as srv:
        tickets = [srv.submit(gg) for gg in graphs]
        for gg, t in zip(graphs, tickets):
            assert srv.wait(t, 60000)
            labels, info = srv.result(t, gg.n)
            assert np.array_equal(labels, oracle.louvain(gg).final_labels), gg.name


@pytest.mark.parametrize("maker", ["tiny", "sbm", "rmat14", "rmat16", "lfr", "rejected"])
def test_coarse_levels_stored_by_degree(maker):
    # order_min = 1 stores every coarse level by degree (the default does so
    # from 2^22 entries); results must not change
    if maker == "tiny":
        rng = np.random.default_rng(31)
        g = bf.to_csr(50, bf.random_graph(rng, 50, 0.15, 9, True))
    elif maker == "sbm":
        g = graphgen.sbm(4096, 128, 0.05, 0.0005, seed=1)
    elif maker == "lfr":
        g, _ = graphgen.lfr(20000, kmax=1500, smin=30, smax=3000, seed=7)
    elif maker == "rejected":
        g = rejected_first_level_graph()
    else:
        g = graphgen.rmat(int(maker[4:]), seed=2)
    tuning = {"order_min": 1}
    compare_louvain(g, tuning=tuning, keep_graphs=True)
    compare_louvain(g, tuning=dict(tuning, block_max=64, hub_mode=2, part_keys=48), prune=True)


def test_coarse_levels_stored_by_degree_in_batches():
    from test_gpu_batch import check_graph, mixed_batch

    graphs = mixed_batch(2, 33)
    with lvp.Graph.batch(graphs) as bg:
        got = lvp.louvain(bg, tuning={"order_min": 1})
    for g, r in zip(graphs, got):
        check_graph(r, oracle.louvain(g), g.name)
