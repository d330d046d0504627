"""The workloads at their full sizes, in the launch configuration the
benchmark times (captured sweeps, every degree class, the bucketed partition
path), against the oracle: every label and every per-sweep move count.

- R-MAT 24 (520.8 M entries) and LFR with 10 M vertices: level 0's local
  moving (all of its sweeps) and LPA against the oracle run here.
- R-MAT 24 and LFR 10 M, every level: the complete multi-level Louvain (and
  LPA) against per-level digests the oracle wrote beforehand (tests/golden/
  make_rmat24_digests.py, make_lfr10m_digests.py; minutes of CPU): sizes,
  Q_int, per-sweep move counts, SHA-256 of every level's labels and of every
  coarse graph.
- The 4,096-graph batch (about 1.15e9 entries in one handle): complete
  Louvain on the device, twelve evenly spaced graphs against the oracle run
  on each graph alone.
- The serving pool (32 R-MAT graphs of 10 k to 4 M vertices) through one
  server at once: every job against a one-graph-per-call run, and every job
  of up to 12 M entries against the oracle."""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import graphgen
import oracle
import paper_2507_06471_amd as lvp

pytestmark = pytest.mark.gpu

SWEEPS = 20  # the benchmark's sweep limit


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rmat24():
    say("generating R-MAT scale 24, edge factor 16, seed 2")
    g = graphgen.rmat(24, 16, seed=2)
    say(f"generated n={g.n} nnz={g.nnz}")
    adj = oracle.adjacency(g)
    return g, adj


@pytest.mark.timeout(600)
def test_rmat24_level0_louvain(rmat24):
    g, adj = rmat24
    say(f"oracle: {SWEEPS} Louvain sweeps over {g.nnz} entries")
    c, moves = oracle.local_move(adj, oracle.LOUVAIN, max_sweeps=SWEEPS)
    want, n2 = oracle.renumber(c)
    q_want, m_want = oracle.modularity_int(adj, want)
    say(f"oracle moves {list(moves)}; GPU: {SWEEPS} sweeps, one level")
    with lvp.Graph.from_csr(g, validate=False) as dg:
        got = lvp.louvain(dg, max_sweeps=SWEEPS, max_levels=1)
    lvl = got.levels[0]
    assert lvl.moves == [int(x) for x in moves]
    assert lvl.info["n_next"] == n2 and lvl.info["accepted"]
    assert np.array_equal(lvl.labels, want)
    assert np.array_equal(got.final_labels, want)
    assert (lvl.info["q_end"], got.M) == (q_want, m_want)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rmat24_seed2_digests.json")
GOLDEN_LFR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "lfr10m_seed3_digests.json")


def sha(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a, dtype="<i4").tobytes())
    return h.hexdigest()


def check_every_level(g, golden_path):
    with open(golden_path) as fh:
        gold = json.load(fh)
    assert (g.n, g.nnz) == (gold["n"], gold["nnz"])
    want = gold["louvain"]
    say(f"GPU: Louvain, every level, coarse graphs kept; {len(want['levels'])} levels in the digests")
    with lvp.Graph.from_csr(g, validate=False) as dg:
        got = lvp.louvain(dg, max_sweeps=gold["max_sweeps"], keep_graphs=True)
        lp = lvp.lpa(dg, max_sweeps=gold["max_sweeps"])
    assert (got.M, got.q_int) == (want["M"], want["q_int"])
    assert len(got.levels) == len(want["levels"])
    for lvl, (a, b) in enumerate(zip(got.levels, want["levels"])):
        say(f"level {lvl}: n={a.info['n']} nnz={a.info['nnz']} sweeps={a.info['sweeps']} "
            f"cached={a.info['cached_sweeps']}")
        i = a.info
        assert (i["n"], i["nnz"], i["n_next"], i["q_start"], i["q_end"], bool(i["accepted"])) == \
            (b["n"], b["nnz"], b["n_next"], b["q_start"], b["q_end"], b["accepted"]), f"level {lvl}"
        assert a.moves == b["moves"], f"level {lvl} moves"
        if b["accepted"]:
            assert sha(a.labels) == b["labels_sha256"], f"level {lvl} labels"
            off, idx, w = a.graph
            assert len(idx) == b["coarse_nnz"], f"level {lvl} coarse entries"
            assert sha(off, idx, w) == b["coarse_sha256"], f"level {lvl} coarse graph"
    assert sha(got.final_labels) == want["final_labels_sha256"]
    assert lp.moves == gold["lpa"]["moves"]
    assert sha(lp.labels) == gold["lpa"]["labels_sha256"]
    assert lp.info["q_end"] == gold["lpa"]["q_int"]


@pytest.mark.timeout(900)
def test_rmat24_every_level_against_golden_digests(rmat24):
    g, _ = rmat24
    check_every_level(g, GOLDEN)


@pytest.mark.timeout(600)
def test_rmat24_lpa(rmat24):
    g, adj = rmat24
    say(f"oracle: {SWEEPS} LPA sweeps over {g.nnz} entries")
    c, moves = oracle.local_move(adj, oracle.LPA, max_sweeps=SWEEPS)
    want, _ = oracle.renumber(c)
    say(f"oracle moves {list(moves)}; GPU LPA")
    with lvp.Graph.from_csr(g, validate=False) as dg:
        got = lvp.lpa(dg, max_sweeps=SWEEPS)
    assert got.moves == [int(x) for x in moves]
    assert np.array_equal(got.labels, want)


@pytest.fixture(scope="module")
def lfr10m():
    # the LFR configuration at full size: 10 M vertices, weights 1..8
    say("generating LFR n=10,000,000 seed 3")
    g, _ = graphgen.lfr(10_000_000, seed=3)
    say(f"generated n={g.n} nnz={g.nnz}")
    return g


@pytest.mark.timeout(600)
def test_lfr_10m_level0_louvain_and_lpa(lfr10m):
    g = lfr10m
    adj = oracle.adjacency(g)
    c, moves = oracle.local_move(adj, oracle.LOUVAIN, max_sweeps=SWEEPS)
    want, n2 = oracle.renumber(c)
    q_want, m_want = oracle.modularity_int(adj, want)
    c, lpa_moves = oracle.local_move(adj, oracle.LPA, max_sweeps=SWEEPS)
    want_lpa, _ = oracle.renumber(c)
    say(f"oracle moves {list(moves)}; LPA {list(lpa_moves)}; GPU")
    with lvp.Graph.from_csr(g, validate=False) as dg:
        got = lvp.louvain(dg, max_sweeps=SWEEPS, max_levels=1)
        got_lpa = lvp.lpa(dg, max_sweeps=SWEEPS)
    lvl = got.levels[0]
    assert lvl.moves == [int(x) for x in moves]
    assert lvl.info["n_next"] == n2 and np.array_equal(lvl.labels, want)
    assert (lvl.info["q_end"], got.M) == (q_want, m_want)
    assert got_lpa.moves == [int(x) for x in lpa_moves]
    assert np.array_equal(got_lpa.labels, want_lpa)


@pytest.mark.timeout(600)
def test_lfr_10m_every_level_against_golden_digests(lfr10m):
    check_every_level(lfr10m, GOLDEN_LFR)


@pytest.mark.timeout(600)
def test_batch_4096_graphs_sampled():
    # the batch configuration at full size (4,096 graphs packed in one
    # handle, about 1.15e9 entries), complete Louvain; sampled graphs against
    # the oracle run on each graph alone
    say("generating the 4,096-graph batch, seed 4")
    gs = graphgen.batch_mix(4096, seed=4)
    say(f"generated {sum(x.nnz for x in gs)} entries")
    with lvp.Graph.batch(gs, validate=False) as bg:
        got = lvp.louvain(bg, level_labels=False)
    assert len(got) == len(gs)
    for i in np.linspace(0, len(gs) - 1, 12).astype(int):
        say(f"graph {i}: n={gs[i].n} nnz={gs[i].nnz}")
        want = oracle.louvain(gs[i])
        assert np.array_equal(got[i].final_labels, want.final_labels), f"graph {i} labels"
        assert got[i].q_int == want.q_int and got[i].M == want.M
        assert [lv.moves for lv in got[i].levels] == [[int(x) for x in lv.moves] for lv in want.levels]


@pytest.mark.timeout(600)
def test_serving_pool_full_size():
    # the serving configuration's graphs (R-MAT, 10 k to 4 M vertices, edge
    # factor 8..16), all submitted at once to one server: every job against a
    # one-graph-per-call run, and those of up to 12 M entries against the oracle
    say("generating the serving pool, seed 5")
    pool = graphgen.serving_pool(32, seed=5)
    say(f"generated {len(pool)} graphs, {sum(g.nnz for g in pool)} entries")
    with lvp.Server() as srv:
        tickets = [srv.submit(g) for g in pool]
        served = []
        for g, t in zip(pool, tickets):
            assert srv.wait(t, 120000), g.name
            served.append(srv.result(t, g.n))
        st = srv.stats()
        say(f"stats {st}")
        assert st["completed"] == len(pool) and st["in_flight"] == 0 and st["mem_in_use"] == 0
    for g, (labels, info) in zip(pool, served):
        say(f"{g.name}: nnz={g.nnz}")
        assert info["status"] == 0, g.name
        with lvp.Graph.from_csr(g, validate=False) as dg:
            alone = lvp.louvain(dg, level_labels=False)
        assert np.array_equal(labels, alone.final_labels) and info["q_int"] == alone.q_int, g.name
        if g.nnz <= 12_000_000:
            want = oracle.louvain(g)
            assert np.array_equal(labels, want.final_labels), g.name
            assert (info["q_int"], info["m"]) == (want.q_int, want.M), g.name
