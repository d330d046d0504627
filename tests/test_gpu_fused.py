"""The persistent fused sweep kernel (lv_tuning.fused: every class below the
hub class in one launch per sweep, workgroups taking blocks of rows of any
class from a device counter) and the LDS table capacity knob
(lv_tuning.table_pct) against the oracle: they only change which lanes do
the work and how full the tables get, never a result."""
import numpy as np
import pytest

import bruteforce as bf
import graphgen
import oracle
import paper_2507_06471_amd as lvp
from test_gpu_batch import mixed_batch
from test_gpu_parity import compare_louvain, compare_lpa, say

pytestmark = pytest.mark.gpu

TUNINGS = [
    {"fused": 1},
    {"fused": 1, "cache_pct": 100},
    {"fused": 1, "table_pct": 100},
    {"fused": 1, "table_pct": 400, "block_max": 600, "hub_mode": 2, "part_keys": 500},
    {"fused": 1, "sub_max": 8, "wave_max": 8, "block_max": 8, "part_keys": 40, "part_slots": 64},
    {"table_pct": 100},
    {"table_pct": 137, "cache_pct": 100},
    {"table_pct": 300, "part_slots": 1024},
]


@pytest.mark.parametrize("tuning", TUNINGS)
def test_rmat_and_lfr(tuning):
    compare_louvain(graphgen.rmat(14, seed=5), tuning=tuning, keep_graphs=True)
    compare_lpa(graphgen.rmat(14, seed=5), tuning=tuning)
    g, _ = graphgen.lfr(20000, kmax=1500, smin=30, smax=3000, seed=7)
    compare_louvain(g, tuning=tuning)


@pytest.mark.parametrize("seed", range(12))
def test_tiny_graphs(seed):
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(2, 60))
    g = bf.to_csr(n, bf.random_graph(rng, n, float(rng.uniform(0.05, 0.4)), 9, True))
    g.name = f"tiny{seed}"
    for t in ({"fused": 1}, {"fused": 1, "table_pct": 100, "cache_pct": 100}):
        compare_louvain(g, tuning=t, keep_graphs=True)
        compare_lpa(g, tuning=t)


def test_sbm_and_rmat18():
    compare_louvain(graphgen.sbm(4096, 128, 0.05, 0.0005, seed=1), tuning={"fused": 1})
    compare_louvain(graphgen.rmat(18, seed=2), tuning={"fused": 1})


@pytest.mark.parametrize("fused", [0, 1])
def test_packed_batch(fused):
    gs = mixed_batch(44, 12)
    tuning = {"fused": fused, "table_pct": 150}
    with lvp.Graph.batch(gs) as bg:
        got = lvp.louvain(bg, tuning=tuning)
    for i, g in enumerate(gs):
        want = oracle.louvain(g)
        assert np.array_equal(got[i].final_labels, want.final_labels), i
        assert got[i].q_int == want.q_int
        assert [lv.moves for lv in got[i].levels] == [[int(x) for x in lv.moves] for lv in want.levels], i


def test_timed_driver_reports_the_fused_launch():
    g = graphgen.rmat(14, seed=8)
    with lvp.Graph.from_csr(g) as dg:
        r = lvp.louvain(dg, tuning={"fused": 1}, timing=True)
    info = r.levels[0].info
    k = lvp.KERNEL_NAMES.index("fused")
    assert info["kern_launches"][k] == info["sweeps"] - 1 and info["kern_ms"][k] > 0
    assert np.array_equal(r.final_labels, oracle.louvain(g).final_labels)
