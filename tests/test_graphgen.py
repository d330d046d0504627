"""Generator properties: canonical symmetric CSR, determinism, expected sizes."""
import numpy as np

import graphgen


def assert_canonical(g):
    off, idx = g.offsets, g.indices
    assert off[0] == 0 and off[-1] == len(idx) and np.all(np.diff(off) >= 0)
    rows = np.repeat(np.arange(g.n), np.diff(off))
    assert not np.any(rows == idx), "self-loop"
    for r in range(min(g.n, 2000)):
        seg = idx[off[r]:off[r + 1]]
        assert np.all(np.diff(seg) > 0), "unsorted or duplicate row"
    fwd = rows.astype(np.int64) * g.n + idx
    bwd = idx.astype(np.int64) * g.n + rows
    assert np.array_equal(np.sort(fwd), np.sort(bwd)), "not symmetric"


def test_rmat_canonical_and_deterministic():
    a = graphgen.rmat(12, seed=5)
    b = graphgen.rmat(12, seed=5)
    c = graphgen.rmat(12, seed=6)
    assert_canonical(a)
    assert np.array_equal(a.offsets, b.offsets) and np.array_equal(a.indices, b.indices)
    assert not np.array_equal(a.indices, c.indices)
    assert a.n == 4096 and 0.6 * 16 * 4096 * 2 < a.nnz < 16 * 4096 * 2


def test_rmat_truncated_vertex_count():
    g = graphgen.rmat(11, n=1500, samples=1500 * 8, seed=3)
    assert_canonical(g)
    assert g.n == 1500 and g.indices.max() < 1500


def test_sbm_density_matches_probabilities():
    g = graphgen.sbm(4096, 128, 0.05, 0.0005, seed=1)
    assert_canonical(g)
    rows = np.repeat(np.arange(g.n), np.diff(g.offsets))
    intra = np.sum(rows // 128 == g.indices // 128) // 2
    inter = g.nnz // 2 - intra
    exp_in = 32 * 128 * 127 / 2 * 0.05
    exp_out = (4096 * 4095 / 2 - 32 * 128 * 127 / 2) * 0.0005
    assert abs(intra - exp_in) < 5 * np.sqrt(exp_in)
    assert abs(inter - exp_out) < 5 * np.sqrt(exp_out)


def test_lfr_shape():
    g, memb = graphgen.lfr(20000, kmax=500, smin=20, smax=2000, seed=3)
    assert_canonical(g)
    deg = np.diff(g.offsets)
    assert 15 < deg.mean() < 22
    assert g.weights.min() >= 1 and g.weights.max() <= 8
    rows = np.repeat(np.arange(g.n), deg)
    mixing = np.mean(memb[rows] != memb[g.indices])
    assert 0.2 < mixing < 0.4
    # weights symmetric
    key_f = rows.astype(np.int64) * g.n + g.indices
    key_b = g.indices.astype(np.int64) * g.n + rows
    o_f, o_b = np.argsort(key_f), np.argsort(key_b)
    assert np.array_equal(g.weights[o_f], g.weights[o_b])


def test_from_edges_merges_and_keeps_loops():
    g = graphgen.from_edges(3, [0, 0, 1, 2], [1, 1, 1, 0], [2, 3, 4, 1])
    assert list(g.offsets) == [0, 2, 4, 5]
    assert list(g.indices) == [1, 2, 0, 1, 0]
    assert list(g.weights) == [5, 1, 5, 4, 1]
