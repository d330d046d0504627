"""Packed batches and sweep drivers through the C ABI.

A packed handle (lv_graph_create_batch) runs every graph under the same rules
as alone: each graph's levels, per-sweep move counts, labels and Q_int must
equal the oracle's for that graph by itself, bit for bit.  The captured
(hipGraph) and eager sweep drivers must agree with each other and with the
oracle."""
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


def check_graph(got, want, name):
    assert got.M == want.M, name
    assert len(got.levels) == len(want.levels), name
    for lvl, (a, b) in enumerate(zip(got.levels, want.levels)):
        assert a.moves == [int(x) for x in b.moves], f"{name} level {lvl} moves"
        assert (a.info["n"], a.info["n_next"], a.info["q_start"], a.info["q_end"]) == (
            b.n, b.n_next, b.q_start, b.q_end), f"{name} level {lvl} stats"
        assert bool(a.info["accepted"]) == b.accepted, name
        if b.accepted:
            assert np.array_equal(a.labels, b.labels), f"{name} level {lvl} labels"
    assert np.array_equal(got.final_labels, want.final_labels), name
    assert got.q_int == want.q_int and got.q == want.q, name


def mixed_batch(seed, count):
    rng = np.random.default_rng(seed)
    out = []
    for t in range(count):
        kind = t % 5
        if kind == 0:
            n = int(rng.integers(1, 50))
            g = bf.to_csr(n, bf.random_graph(rng, n, float(rng.uniform(0.02, 0.4)), 9, True))
        elif kind == 1:
            g = graphgen.sbm(int(rng.integers(200, 1200)), int(rng.integers(16, 64)), 0.1, 0.002,
                             seed=int(rng.integers(1 << 30)))
        elif kind == 2:
            g = graphgen.rmat(int(rng.integers(8, 12)), seed=int(rng.integers(1 << 30)))
        elif kind == 3:
            g = graphgen.rmat(10, seed=int(rng.integers(1 << 30)))
            g.weights = graphgen.pair_weights(g, 1, 7, seed=int(rng.integers(1 << 30)))
        else:
            n = int(rng.integers(1, 30))
            g = graphgen.CSR(n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), None)  # no edges
        g.name = f"b{seed}.{t}"
        out.append(g)
    return out


@pytest.mark.parametrize("seed,count", [(0, 5), (1, 12), (2, 33)])
def test_batch_equals_each_graph_alone(seed, count):
    graphs = mixed_batch(seed, count)
    say(f"batch seed={seed} count={count} n={[g.n for g in graphs]}")
    with lvp.Graph.batch(graphs) as bg:
        assert bg.count == count
        got = lvp.louvain(bg)
        lp = lvp.lpa(bg)
    assert len(got) == count and len(lp) == count
    for g, r, l in zip(graphs, got, lp):
        check_graph(r, oracle.louvain(g), g.name)
        want = oracle.lpa(g)
        assert l.moves == [int(x) for x in want.moves], g.name
        assert np.array_equal(l.labels, want.labels), g.name
        assert l.info["q_end"] == want.q_int, g.name


def test_batch_with_hubs_and_tuning():
    # one graph large enough for the partitioned path next to small ones
    graphs = [graphgen.rmat(14, seed=5), bf.to_csr(6, [(0, 1, 1), (0, 2, 1), (1, 2, 1), (3, 4, 1), (3, 5, 1),
                                                      (4, 5, 1), (2, 3, 1)]),
              graphgen.sbm(2048, 64, 0.08, 0.001, seed=9), graphgen.rmat(12, seed=6)]
    for t, g in enumerate(graphs):
        g.name = f"h{t}"
    tuning = {"sub_max": 8, "wave_max": 8, "block_max": 8, "part_keys": 40, "part_slots": 64, "hub_chunk": 1024}
    say("batch with forced partitions/overflows")
    with lvp.Graph.batch(graphs) as bg:
        got = lvp.louvain(bg, tuning=tuning)
    for g, r in zip(graphs, got):
        check_graph(r, oracle.louvain(g), g.name)


def test_batch_single_graph_matches_plain_handle():
    g = graphgen.rmat(12, seed=11)
    with lvp.Graph.batch([g]) as bg, lvp.Graph.from_csr(g) as dg:
        assert bg.count == 1
        a = lvp.louvain(bg)
        b = lvp.louvain(dg)
    assert a.q_int == b.q_int and np.array_equal(a.final_labels, b.final_labels)


@pytest.mark.parametrize("mode", ["hipgraph", "eager", "timing"])
def test_sweep_drivers_agree(mode):
    g = graphgen.rmat(15, seed=3)
    want = oracle.louvain(g)
    say(f"driver {mode}")
    with lvp.Graph.from_csr(g) as dg:
        for rep in range(2):  # replays of the captured sweeps are deterministic
            got = lvp.louvain(dg, timing=(mode == "timing"), hipgraph=(mode == "hipgraph"))
            check_graph(got, want, f"{mode} rep {rep}")
            l = lvp.lpa(dg, timing=(mode == "timing"), hipgraph=(mode == "hipgraph"))
            wl = oracle.lpa(g)
            assert np.array_equal(l.labels, wl.labels) and l.moves == [int(x) for x in wl.moves]


def test_batch_rejects_bad_member():
    good = graphgen.rmat(8, seed=1)
    bad = graphgen.CSR(2, np.array([0, 1, 2], np.int32), np.array([1, 1], np.int32), None)  # asymmetric
    with pytest.raises(lvp.LvError) as ei:
        lvp.Graph.batch([good, bad])
    assert ei.value.status == 3
    oob = graphgen.CSR(2, np.array([0, 1, 2], np.int32), np.array([1, 2], np.int32), None)
    with pytest.raises(lvp.LvError) as ei:
        lvp.Graph.batch([good, oob])
    assert ei.value.status == 2


def test_autotuned_results_equal_oracle():
    g = graphgen.rmat(14, seed=12)
    want = oracle.louvain(g)
    with lvp.Graph.from_csr(g) as dg:
        cfg, ms = lvp.autotune(dg)
        say(f"autotuned {cfg} est {ms:.3f} ms")
        assert ms > 0
        check_graph(lvp.louvain(dg, autotuned=True), want, "autotuned")
        l = lvp.lpa(dg, autotuned=True)
    wl = oracle.lpa(g)
    assert np.array_equal(l.labels, wl.labels)


def test_batch_final_partition_accessors():
    graphs = mixed_batch(5, 9)
    with lvp.Graph.batch(graphs) as bg:
        fp = lvp.louvain_final(bg, autotuned=True)
    base = 0
    for t, g in enumerate(graphs):
        want = oracle.louvain(g)
        assert np.array_equal(fp.labels[base:base + g.n], want.final_labels), g.name
        assert (fp.q_int[t], fp.M[t], fp.q[t]) == (want.q_int, want.M, want.q), g.name
        base += g.n


def test_gather_probe_reports_a_rate():
    g = graphgen.rmat(14, seed=3)
    with lvp.Graph.from_csr(g) as dg:
        rate = lvp.probe_gather(dg, reps=2)
    say(f"gather ceiling on R-MAT 14: {rate / 1e9:.1f} G entries/s")
    assert np.isfinite(rate) and rate > 0
    with pytest.raises(lvp.LvError):
        with lvp.Graph.from_csr(g) as dg:
            lvp.probe_gather(dg, reps=0)


def test_copy_probe_reports_a_bandwidth():
    g = graphgen.rmat(15, seed=4)
    with lvp.Graph.from_csr(g) as dg:
        rate = lvp.probe_copy(dg, reps=2)
        empty = lvp.Graph.from_csr(graphgen.CSR(3, np.zeros(4, np.int32), np.zeros(0, np.int32), None))
        try:
            zero = lvp.probe_copy(empty, reps=1)
        finally:
            empty.close()
    say(f"copy probe on R-MAT 15 ({g.nnz} entries): {rate / 1e9:.1f} GB/s")
    assert np.isfinite(rate) and 0 < rate < 20e12
    assert zero == 0.0
    with pytest.raises(lvp.LvError):
        with lvp.Graph.from_csr(g) as dg:
            lvp.probe_copy(dg, reps=0)
