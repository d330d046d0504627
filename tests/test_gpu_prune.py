"""Active-vertex pruning (LV_PRUNE) through the C ABI against the oracle's
pruned levels: per-sweep move counts, every level's labels, Q_int, bit for
bit, across the degree classes, the partitioned hub paths, packed batches and
the sweep drivers."""
import numpy as np
import pytest

import bruteforce as bf
import graphgen
import oracle
import paper_2507_06471_amd as lvp
from test_gpu_batch import check_graph, mixed_batch
from test_gpu_parity import compare_louvain, compare_lpa, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("seed", range(20))
def test_tiny_random_graphs(seed):
    rng = np.random.default_rng(700 + seed)
    n = int(rng.integers(1, 60))
    g = bf.to_csr(n, bf.random_graph(rng, n, float(rng.uniform(0.02, 0.4)), 9, True))
    g.name = f"ptiny{seed}"
    compare_louvain(g, keep_graphs=True, prune=True)
    compare_lpa(g, prune=True)


@pytest.mark.parametrize("maker", ["sbm", "rmat12", "rmat16", "rmat18", "lfr"])
def test_generated_graphs(maker):
    if maker == "sbm":
        g = graphgen.sbm(4096, 128, 0.05, 0.0005, seed=1)
    elif maker == "lfr":
        g, _ = graphgen.lfr(30000, kmax=1500, smin=30, smax=3000, seed=3)
    else:
        g = graphgen.rmat(int(maker[4:]), seed=2)
    got, want = compare_louvain(g, prune=True)
    compare_lpa(g, prune=True)
    full = oracle.louvain(g)
    say(f"{maker}: pruned q={got.q:.6f} full q={full.q:.6f}")


@pytest.mark.parametrize("tuning", [
    {"sub_max": 1, "wave_max": 2, "block_max": 3, "part_keys": 256},
    {"sub_max": 8, "wave_max": 8, "block_max": 8, "part_keys": 40, "part_slots": 64},
    {"sub_max": 8, "wave_max": 8, "block_max": 8, "part_keys": 40, "part_slots": 64, "hub_mode": 1},
    {"block_max": 600, "hub_mode": 1, "part_keys": 500},
    {"block_max": 300, "hub_mode": 2, "part_keys": 100, "part_slots": 128},
    {"block_max": 64, "hub_mode": 2, "part_keys": 48, "hub_chunk": 1024},
])
def test_partitioned_paths(tuning):
    g = graphgen.rmat(14, seed=5)
    compare_louvain(g, tuning=tuning, prune=True)
    compare_lpa(g, tuning=tuning, prune=True)


def test_input_order_storage():
    g = graphgen.rmat(13, seed=21)
    compare_louvain(g, keep_graphs=True, keep_order=True, prune=True)
    compare_lpa(g, keep_order=True, prune=True)


@pytest.mark.parametrize("mode", ["eager", "timing"])
def test_sweep_drivers(mode):
    g = graphgen.rmat(15, seed=3)
    compare_louvain(g, prune=True, hipgraph=False, timing=(mode == "timing"))


@pytest.mark.parametrize("seed,count", [(0, 5), (2, 33)])
def test_packed_batch(seed, count):
    graphs = mixed_batch(seed, count)
    say(f"pruned batch seed={seed} count={count}")
    with lvp.Graph.batch(graphs) as bg:
        got = lvp.louvain(bg, prune=True)
        lp = lvp.lpa(bg, prune=True)
    for g, r, l in zip(graphs, got, lp):
        check_graph(r, oracle.louvain(g, prune=True), g.name)
        want = oracle.lpa(g, prune=True)
        assert l.moves == [int(x) for x in want.moves] and np.array_equal(l.labels, want.labels), g.name


def test_pruned_lpa_equals_full_lpa():
    g = graphgen.rmat(16, seed=9)
    with lvp.Graph.from_csr(g) as dg:
        a = lvp.lpa(dg)
        b = lvp.lpa(dg, prune=True)
    assert a.moves == b.moves and np.array_equal(a.labels, b.labels)
