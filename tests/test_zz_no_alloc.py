"""lv_modularity_noalloc, the allocation-free variant of lv_modularity,
through the C ABI: on two calls in a row (the second on a smaller graph) it
must give exactly what lv_modularity gives, without changing the device's
free memory; oversize graphs, labels outside [0, n) and host labels are
refused before any kernel runs."""
import sys

import numpy as np
import pytest

import graphgen
import paper_2507_06471_amd as lvp

pytestmark = pytest.mark.gpu

LV_E_ARG, LV_E_TOO_LARGE = 1, 9


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def free_bytes(torch):
    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


def test_noalloc_equals_lv_modularity_on_two_calls():
    import torch

    rng = np.random.default_rng(7)
    big = graphgen.rmat(16, seed=31)                       # 65,536 vertices, stored by degree
    small = graphgen.sbm(4096, 128, 0.05, 0.0005, seed=1)  # 4,096 vertices
    cases = []
    for g in (big, small):
        h = lvp.Graph.from_csr(g)
        part = lvp.louvain(h, level_labels=False).final_labels
        rand = rng.integers(0, g.n, size=g.n).astype(np.int32)
        for lab in (part, rand):
            want = lvp.modularity(h, lab)
            cases.append((h, torch.from_numpy(np.ascontiguousarray(lab)).cuda(), want))
    lvp.modularity_noalloc(cases[0][0], cases[0][1])  # the first call on this device looks up the array
    before = free_bytes(torch)
    for h, lab, want in cases:  # big graph first, then the smaller one
        got = lvp.modularity_noalloc(h, lab)
        say(f"n={h.n}: lv_modularity {want}, noalloc {got}")
        assert got == want
    assert free_bytes(torch) == before
    for h, _, _ in cases[::2]:
        h.close()


def test_noalloc_refuses_what_it_cannot_take():
    import torch

    n = (lvp.NOALLOC_SCRATCH_BYTES - 256) // 12 + 1  # one vertex too many for the scratch array
    off = np.full(n + 1, 2, dtype=np.int32)  # one edge, 0 - 1; every other vertex isolated
    off[0], off[1] = 0, 1
    idx = np.array([1, 0], dtype=np.int32)
    with lvp.Graph(n, off, idx, validate=True) as h:
        lab = torch.zeros(n, dtype=torch.int32, device="cuda")
        with pytest.raises(lvp.LvError) as ei:
            lvp.modularity_noalloc(h, lab)
        assert ei.value.status == LV_E_TOO_LARGE
    g = graphgen.sbm(4096, 128, 0.05, 0.0005, seed=1)
    with lvp.Graph.from_csr(g) as h:
        bad = torch.full((g.n,), g.n, dtype=torch.int32, device="cuda")
        with pytest.raises(lvp.LvError) as ei:
            lvp.modularity_noalloc(h, bad)
        assert ei.value.status == LV_E_ARG
        pinned = torch.zeros(g.n, dtype=torch.int32).pin_memory()
        lib = lvp.load_library()
        import ctypes
        qi, m, q = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
        st = lib.lv_modularity_noalloc(h.handle, pinned.data_ptr(), ctypes.byref(qi), ctypes.byref(m), ctypes.byref(q))
        assert st == LV_E_ARG
        # still usable afterwards
        lab = torch.zeros(g.n, dtype=torch.int32, device="cuda")
        assert lvp.modularity_noalloc(h, lab) == lvp.modularity(h, np.zeros(g.n, dtype=np.int32))
