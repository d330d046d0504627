"""Asynchronous sweeps (LV_ASYNC): labels and community volumes change in
place while a sweep runs, as the paper's Alg. 1 and Alg. 2 are written.
Results depend on scheduling, so there is no bit-exact oracle; every run is
checked for what must hold regardless of scheduling:

  * the reported Q_int and M equal the modularity of the returned labels,
    computed both by the library and by the oracle on the CPU;
  * every accepted level raised Q_int (Q_end > Q_start), its labels are
    contiguous in first-occurrence order, and the final labels are the
    composition of the accepted levels' labels;
  * a level that stopped before max_sweeps ended with a quiet sweep;
  * the partition's quality stays close to the synchronous sweeps' result.
"""
import numpy as np
import pytest

import bruteforce as bf
import graphgen
import oracle
import paper_2507_06471_amd as lvp
from test_gpu_batch import mixed_batch
from test_gpu_parity import say

pytestmark = pytest.mark.gpu


def check_run(g, r, max_sweeps=20):
    q, m, _ = oracle.modularity(g, r.final_labels)
    assert (q, m) == (r.q_int, r.M), "reported modularity differs from the labels' modularity"
    fin = np.arange(g.n, dtype=np.int64)
    for lv in r.levels:
        i = lv.info
        if i["sweeps"] < max_sweeps:
            assert lv.moves[-1] == 0, "a level ended without a quiet sweep"
        if not i["accepted"]:
            assert i["q_end"] <= i["q_start"]
            continue
        assert i["q_end"] > i["q_start"] and i["n_next"] <= i["n"]
        lab = lv.labels
        assert lab.min() >= 0 and lab.max() + 1 == i["n_next"]
        first = np.unique(lab, return_index=True)[1]
        assert np.array_equal(np.sort(first), first), "labels not in first-occurrence order"
        fin = lab[fin]
    assert np.array_equal(fin, r.final_labels)


@pytest.mark.parametrize("maker", ["sbm", "lfr", "rmat14", "rmat18"])
def test_async_louvain_invariants_and_quality(maker):
    if maker == "sbm":
        g = graphgen.sbm(4096, 128, 0.05, 0.0005, seed=1)
    elif maker == "lfr":
        g, _ = graphgen.lfr(30000, kmax=1500, smin=30, smax=3000, seed=3)
    else:
        g = graphgen.rmat(int(maker[4:]), seed=2)
    with lvp.Graph.from_csr(g) as dg:
        sync = lvp.louvain(dg)
        runs = [lvp.louvain(dg, asynchronous=True) for _ in range(2)]
        pruned = lvp.louvain(dg, asynchronous=True, prune=True)
    for r in runs + [pruned]:
        check_run(g, r)
    qa = [r.q for r in runs]
    say(f"{maker}: sync q={sync.q:.5f} levels={len(sync.accepted)}; async q={qa} "
        f"sweeps={[lv.info['sweeps'] for lv in runs[0].levels]}; async+prune q={pruned.q:.5f}")
    for q in qa + [pruned.q]:
        assert q >= sync.q - 0.03 - 0.03 * abs(sync.q), (maker, q, sync.q)
    if maker == "sbm":
        # scheduling decides which of two neighbours' moves lands first, so an
        # asynchronous run's Q varies from run to run (0.648 to 0.694 observed
        # against 0.690 synchronous); the planted blocks must still show
        assert min(qa) > 0.6


@pytest.mark.parametrize("seed", range(8))
def test_async_tiny_graphs(seed):
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(1, 60))
    g = bf.to_csr(n, bf.random_graph(rng, n, float(rng.uniform(0.02, 0.4)), 9, True))
    with lvp.Graph.from_csr(g) as dg:
        r = lvp.louvain(dg, asynchronous=True)
        lp = lvp.lpa(dg, asynchronous=True)
    check_run(g, r)
    q, m, _ = oracle.modularity(g, lp.labels)
    assert q == lp.info["q_end"]


def test_async_lpa():
    g = graphgen.sbm(4096, 128, 0.05, 0.0005, seed=1)
    with lvp.Graph.from_csr(g) as dg:
        sync = lvp.lpa(dg)
        a = lvp.lpa(dg, asynchronous=True)
    q, m, _ = oracle.modularity(g, a.labels)
    assert q == a.info["q_end"]
    first = np.unique(a.labels, return_index=True)[1]
    assert np.array_equal(np.sort(first), first) and a.labels.max() + 1 == len(first)
    say(f"lpa sync q={sync.info['q_end'] / float(m) ** 2:.5f} sweeps={sync.info['sweeps']}; "
        f"async q={q / float(m) ** 2:.5f} sweeps={a.info['sweeps']}")
    assert a.info["sweeps"] <= 20


def test_async_packed_batch():
    graphs = mixed_batch(3, 9)
    with lvp.Graph.batch(graphs) as bg:
        got = lvp.louvain(bg, asynchronous=True)
    for g, r in zip(graphs, got):
        check_run(g, r)
