"""Pins of the oracle's edge-list -> CSR construction (Section II-A graph
model; repeated pairs merged with summed weights, as in Section III-B).

  * brute force: the dense adjacency built straight from the edge list
    (tests/bruteforce.py, loops doubled the way the weighted degree counts
    them) equals the oracle's adjacency of the built CSR;
  * a library: scipy's COO -> CSR with duplicate summation;
  * a worked example by hand, the special flags, and R-MAT raw samples,
    whose loop-free simple graph is exactly the generator's own CSR.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import bruteforce as bf
import graphgen
import oracle


def random_edge_list(rng, n, m, wmax):
    src = rng.integers(0, n, size=m)
    dst = np.where(rng.random(m) < 0.1, src, rng.integers(0, n, size=m))  # some loops
    rep = rng.integers(0, m, size=m // 3)  # some pairs listed again, in either orientation
    flip = rng.random(len(rep)) < 0.5
    src2 = np.concatenate([src, np.where(flip, dst[rep], src[rep])])
    dst2 = np.concatenate([dst, np.where(flip, src[rep], dst[rep])])
    w = rng.integers(1, wmax + 1, size=len(src2))
    return src2.astype(np.int32), dst2.astype(np.int32), w.astype(np.int32)


def csr_ok(n, off, idx):
    assert off[0] == 0 and off[-1] == len(idx) and np.all(np.diff(off) >= 0)
    for r in range(n):
        row = idx[off[r]:off[r + 1]]
        assert np.all(np.diff(row) > 0)


@pytest.mark.parametrize("seed", range(25))
def test_matches_bruteforce_dense_adjacency(seed):
    rng = np.random.default_rng(3000 + seed)
    n = int(rng.integers(1, 14))
    src, dst, w = random_edge_list(rng, n, int(rng.integers(0, 30)), 6)
    off, idx, wt = oracle.graph_from_edges(n, src, dst, w)
    csr_ok(n, off, idx)
    A = np.array(bf.dense_adjacency(n, list(zip(src.tolist(), dst.tolist(), w.tolist()))), dtype=np.int64).reshape(n, n)
    adj = oracle.adjacency(graphgen.CSR(n, off, idx, wt))
    got = np.zeros((n, n), dtype=np.int64)
    for r in range(n):
        got[r, adj.idx[adj.off[r]:adj.off[r + 1]]] = adj.a[adj.off[r]:adj.off[r + 1]]
    assert np.array_equal(got, A)
    # simple: every adjacent pair once with weight 1 (a loop's entry 1, so A_vv = 2)
    off_s, idx_s, wt_s = oracle.graph_from_edges(n, src, dst, None, simple=True)
    assert np.array_equal(off_s, off) and np.array_equal(idx_s, idx) and np.all(wt_s == 1)
    # drop_loops: the same graph without its diagonal
    off_d, idx_d, wt_d = oracle.graph_from_edges(n, src, dst, w, drop_loops=True)
    Ad = A.copy()
    np.fill_diagonal(Ad, 0)
    gd = np.zeros((n, n), dtype=np.int64)
    for r in range(n):
        gd[r, idx_d[off_d[r]:off_d[r + 1]]] = wt_d[off_d[r]:off_d[r + 1]]
    assert np.array_equal(gd, Ad)


@pytest.mark.parametrize("seed", range(5))
def test_matches_scipy_coo_sum_duplicates(seed):
    rng = np.random.default_rng(3100 + seed)
    n = 500
    src, dst, w = random_edge_list(rng, n, 4000, 9)
    off, idx, wt = oracle.graph_from_edges(n, src, dst, w)
    loop = src == dst
    rows = np.concatenate([src, dst[~loop]])
    cols = np.concatenate([dst, src[~loop]])
    vals = np.concatenate([w, w[~loop]]).astype(np.int64)
    ref = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    ref.sum_duplicates()
    ref.sort_indices()
    assert np.array_equal(off, ref.indptr) and np.array_equal(idx, ref.indices) and np.array_equal(wt, ref.data)


def test_worked_example():
    # pairs {0,1}: 2 + 3 (both orientations); loop at 2: 4 + 1; {1,2}: 1; vertex 3 isolated
    off, idx, wt = oracle.graph_from_edges(4, [0, 1, 2, 1, 2], [1, 0, 2, 2, 2], [2, 3, 4, 1, 1])
    assert off.tolist() == [0, 1, 3, 5, 5]
    assert idx.tolist() == [1, 0, 2, 1, 2]
    assert wt.tolist() == [5, 5, 1, 1, 5]
    off, idx, wt = oracle.graph_from_edges(4, [0, 1, 2, 1, 2], [1, 0, 2, 2, 2], drop_loops=True, simple=True)
    assert off.tolist() == [0, 1, 3, 4, 4] and idx.tolist() == [1, 0, 2, 1] and wt.tolist() == [1, 1, 1, 1]


@pytest.mark.parametrize("scale", [8, 11, 14])
def test_rmat_raw_samples_give_the_generator_graph(scale):
    u, v = graphgen.rmat_edges(scale, seed=7)
    g = graphgen.rmat(scale, seed=7)
    off, idx, wt = oracle.graph_from_edges(g.n, u, v, drop_loops=True, simple=True)
    assert np.array_equal(off, g.offsets) and np.array_equal(idx, g.indices) and np.all(wt == 1)


def test_empty_and_errors():
    off, idx, wt = oracle.graph_from_edges(3, [], [])
    assert off.tolist() == [0, 0, 0, 0] and len(idx) == 0
    off, idx, wt = oracle.graph_from_edges(0, [], [])
    assert off.tolist() == [0]
    with pytest.raises(ValueError):
        oracle.graph_from_edges(3, [0], [3])
    with pytest.raises(ValueError):
        oracle.graph_from_edges(3, [0], [1], [0])
    with pytest.raises(OverflowError):
        oracle.graph_from_edges(2, [0, 1], [1, 0], [2**31 - 1, 5])
