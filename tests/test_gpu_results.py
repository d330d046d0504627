"""Result buffers through the C ABI: a result handle keeps its labels after
the graph handle that produced it is destroyed (its buffers then belong to
the result alone), and repeated calls on one handle reuse the pooled result
buffers instead of allocating new ones.  Labels are checked against the
oracle (Alg. 3 around Alg. 2; Alg. 1 for LPA)."""
import ctypes
import sys

import numpy as np
import pytest

import graphgen
import oracle
import paper_2507_06471_amd as lvp

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def free_bytes(torch):
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def test_result_outlives_its_graph():
    g = graphgen.rmat(14, seed=41)
    want = oracle.louvain(g, max_sweeps=20)
    lib = lvp.load_library()
    h = lvp.Graph.from_csr(g)
    p, _keep = lvp.make_params()
    r = ctypes.c_void_p()
    say(f"lv_louvain on R-MAT 14 (n={g.n}), then lv_graph_destroy before reading the result")
    assert lib.lv_louvain(h.handle, ctypes.byref(p), ctypes.byref(r)) == lvp.LV_OK
    h.close()
    acc, att = ctypes.c_int32(), ctypes.c_int32()
    assert lib.lv_result_num_levels(r, ctypes.byref(acc), ctypes.byref(att)) == lvp.LV_OK
    assert acc.value == sum(1 for lv in want.levels if lv.accepted)
    fin = np.empty(g.n, dtype=np.int32)
    assert lib.lv_result_final_labels(r, fin.ctypes.data, lvp.LV_MEM_HOST) == lvp.LV_OK
    assert np.array_equal(fin, want.final_labels)
    lab0 = np.empty(g.n, dtype=np.int32)
    assert lib.lv_result_level_labels(r, 0, lab0.ctypes.data, lvp.LV_MEM_HOST) == lvp.LV_OK
    assert np.array_equal(lab0, want.levels[0].labels)
    assert lib.lv_result_destroy(r) == lvp.LV_OK


def test_repeated_calls_reuse_result_buffers():
    import torch

    g = graphgen.rmat(16, seed=42)
    want = oracle.louvain(g, max_sweeps=20)
    want_lpa = oracle.lpa(g)
    h = lvp.Graph.from_csr(g)
    out = torch.empty(g.n, dtype=torch.int32, device="cuda")
    first = lvp.louvain(h)  # fills the handle's pool with this graph's level and final label buffers
    lvp.lpa(h)              # and an LPA output buffer
    before = free_bytes(torch)
    for rep in range(3):
        got = lvp.louvain(h)
        assert np.array_equal(got.final_labels, want.final_labels)
        for a, b in zip(got.accepted, [lv for lv in want.levels if lv.accepted]):
            assert np.array_equal(a.labels, b.labels)
        lp = lvp.lpa(h)  # host output: through a pooled buffer
        assert np.array_equal(lp.labels, want_lpa.labels)
        lvp.lpa(h, out=out)  # device output: written in place
        assert np.array_equal(out.cpu().numpy(), want_lpa.labels)
        say(f"rep {rep}: free device bytes {free_bytes(torch)} (after the first calls {before})")
        assert free_bytes(torch) == before
    assert np.array_equal(first.final_labels, want.final_labels)
    h.close()
