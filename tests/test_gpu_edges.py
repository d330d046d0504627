"""Graph construction from an edge list (lv_graph_create_edges) and CSR
export (lv_graph_csr) through the C ABI, against the oracle's construction
from the same edges: offsets, indices and weights equal element by element."""
import numpy as np
import pytest

import bruteforce as bf
import graphgen
import oracle
import paper_2507_06471_amd as lvp
from test_gpu_batch import check_graph, mixed_batch
from test_gpu_parity import say
from test_oracle_edges import random_edge_list

pytestmark = pytest.mark.gpu


def built(n, src, dst, w=None, drop_loops=False, simple=False, keep_order=False, device=False):
    if device:
        import torch

        src, dst = torch.from_numpy(src).cuda(), torch.from_numpy(dst).cuda()
        w = None if w is None else torch.from_numpy(w).cuda()
        torch.cuda.synchronize()
    with lvp.Graph.from_edges(n, src, dst, w, drop_loops=drop_loops, simple=simple, keep_order=keep_order) as dg:
        return dg.csr(), dg.volume


def same(got, want):
    return all(np.array_equal(a, b) for a, b in zip(got, want))


@pytest.mark.parametrize("seed", range(12))
def test_random_multigraph_edge_lists(seed):
    rng = np.random.default_rng(4000 + seed)
    n = int(rng.integers(1, 3000 if seed % 3 else 40))
    m = int(rng.integers(0, 8 * n))
    src, dst, w = random_edge_list(rng, n, m, 9)
    say(f"edges seed={seed} n={n} m={len(src)}")
    for flags in ({}, {"drop_loops": True}, {"simple": True}, {"simple": True, "drop_loops": True}):
        wts = None if flags.get("simple") else w
        want = oracle.graph_from_edges(n, src, dst, wts, **flags)
        for keep_order in (False, True):
            got, _ = built(n, src, dst, wts, keep_order=keep_order, **flags)
            assert same(got, want), (flags, keep_order)


def test_device_resident_edges():
    rng = np.random.default_rng(4100)
    src, dst, w = random_edge_list(rng, 5000, 40000, 5)
    got, _ = built(5000, src, dst, w, device=True)
    assert same(got, oracle.graph_from_edges(5000, src, dst, w))


@pytest.mark.parametrize("scale", [12, 16])
def test_rmat_raw_samples(scale):
    u, v = graphgen.rmat_edges(scale, seed=2)
    g = graphgen.rmat(scale, seed=2)
    want = oracle.graph_from_edges(g.n, u, v, drop_loops=True, simple=True)
    with lvp.Graph.from_edges(g.n, u, v, drop_loops=True, simple=True) as dg:
        got = dg.csr()
        r = lvp.louvain(dg)
    assert same(got, want) and np.array_equal(got[0], g.offsets) and np.array_equal(got[1], g.indices)
    o = oracle.louvain(graphgen.CSR(g.n, want[0], want[1], None))
    assert r.q_int == o.q_int and np.array_equal(r.final_labels, o.final_labels)


@pytest.mark.parametrize("maker", ["weighted_loops", "rmat", "lfr"])
@pytest.mark.parametrize("keep_order", [False, True])
def test_csr_export_round_trip(maker, keep_order):
    if maker == "weighted_loops":
        rng = np.random.default_rng(4200)
        g = bf.to_csr(300, bf.random_graph(rng, 300, 0.05, 9, True))
    elif maker == "rmat":
        g = graphgen.rmat(14, seed=4)
    else:
        g, _ = graphgen.lfr(20000, kmax=1500, smin=30, smax=3000, seed=5)
    w = np.ones(g.nnz, np.int32) if g.weights is None else g.weights
    with lvp.Graph.from_csr(g, keep_order=keep_order) as dg:
        off, idx, wt = dg.csr()
    assert np.array_equal(off, g.offsets) and np.array_equal(idx, g.indices) and np.array_equal(wt, w)


def test_packed_export():
    graphs = mixed_batch(1, 12)
    with lvp.Graph.batch(graphs) as bg:
        off, idx, wt = bg.csr()
    vb = eb = 0
    for g in graphs:
        w = np.ones(g.nnz, np.int32) if g.weights is None else g.weights
        assert np.array_equal(off[vb:vb + g.n + 1] - eb, g.offsets), g.name
        assert np.array_equal(idx[eb:eb + g.nnz] - vb, g.indices) and np.array_equal(wt[eb:eb + g.nnz], w)
        vb += g.n
        eb += g.nnz


def test_edge_errors():
    with pytest.raises(lvp.LvError) as e:
        lvp.Graph.from_edges(3, np.array([0], np.int32), np.array([3], np.int32))
    assert e.value.status == 2
    with pytest.raises(lvp.LvError) as e:
        lvp.Graph.from_edges(3, np.array([0], np.int32), np.array([1], np.int32), np.array([0], np.int32))
    assert e.value.status == 4
    with pytest.raises(lvp.LvError) as e:
        lvp.Graph.from_edges(3, np.array([0], np.int32), np.array([1], np.int32), np.array([1], np.int32),
                             simple=True)
    assert e.value.status == 1
    with pytest.raises(lvp.LvError) as e:
        lvp.Graph.from_edges(2, np.array([0, 1], np.int32), np.array([1, 0], np.int32),
                             np.array([2**30, 2**30], np.int32))
    assert e.value.status == 5
    got, vol = built(4, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert got[0].tolist() == [0] * 5 and len(got[1]) == 0 and vol == 0
