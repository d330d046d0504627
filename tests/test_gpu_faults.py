"""Out-of-memory paths through the C ABI, forced from the host.

LV_FAULT_ALLOC_AT=k makes the k-th device (or pinned host) allocation of one
entry-point call fail with out-of-memory.  For every k up to the number of
allocations a call makes, on a fresh handle: the call must return
LV_E_NOMEM, the same handle must then give the oracle's result, and once
every handle is destroyed the device's free memory must be back where it
started (nothing leaked).  No kernel ever runs on a failed allocation: the
library stops at the failing call."""
import os
import sys

import numpy as np
import pytest

import graphgen
import oracle
import paper_2507_06471_amd as lvp

pytestmark = pytest.mark.gpu

LV_E_NOMEM = 6
# a forced hub class (rows above 64 entries take the partitioned path) so that
# the hub plan's allocations are exercised too
TUNING = {"block_max": 64, "wave_max": 32, "sub_max": 8}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def free_bytes():
    import torch

    torch.cuda.synchronize()
    return torch.cuda.mem_get_info()[0]


@pytest.fixture
def fault_env():
    yield
    os.environ.pop("LV_FAULT_ALLOC_AT", None)


def _sweep_faults(g, make, call, check, limit=400):
    """For k = 1, 2, ...: fresh handle, call with the k-th allocation failing,
    then the same call again without faults; stops at the first k the call
    survives.  Returns the number of failing k."""
    failed = 0
    for k in range(1, limit + 1):
        h = make()
        try:
            os.environ["LV_FAULT_ALLOC_AT"] = str(k)
            try:
                call(h)
                survived = True
            except lvp.LvError as e:
                assert e.status == LV_E_NOMEM, f"k={k}: {e}"
                survived = False
            os.environ.pop("LV_FAULT_ALLOC_AT", None)
            check(call(h))
        finally:
            h.close()
        if survived:
            return failed
        failed += 1
    raise AssertionError("calls kept failing past the limit")


def test_louvain_out_of_memory_leaves_handle_usable(fault_env):
    g = graphgen.rmat(14, 16, seed=11)
    want = oracle.louvain(g)
    say(f"R-MAT 14: n={g.n} nnz={g.nnz}, oracle Q_int {want.q_int}")
    base = free_bytes()

    def check(got):
        assert np.array_equal(got.final_labels, want.final_labels) and got.q_int == want.q_int

    failed = _sweep_faults(g, lambda: lvp.Graph.from_csr(g),
                           lambda h: lvp.louvain(h, tuning=TUNING, keep_graphs=True), check)
    say(f"louvain: {failed} allocation points forced to fail, each recovered")
    assert failed > 10
    assert abs(free_bytes() - base) < (32 << 20)


def test_lpa_and_modularity_out_of_memory(fault_env):
    g = graphgen.sbm(4096, 128, 0.05, 0.0005, seed=1)
    want = oracle.lpa(g)
    base = free_bytes()

    def check_lpa(got):
        assert np.array_equal(got.labels, want.labels) and got.moves == [int(x) for x in want.moves]

    failed = _sweep_faults(g, lambda: lvp.Graph.from_csr(g), lambda h: lvp.lpa(h, tuning=TUNING), check_lpa)
    say(f"lpa: {failed} allocation points forced to fail")
    assert failed > 3

    def check_q(got):
        assert got[:2] == (want.q_int, want.M)

    failed = _sweep_faults(g, lambda: lvp.Graph.from_csr(g), lambda h: lvp.modularity(h, want.labels), check_q)
    say(f"modularity: {failed} allocation points forced to fail")
    assert abs(free_bytes() - base) < (32 << 20)


def test_create_out_of_memory(fault_env):
    g = graphgen.rmat(12, 8, seed=12)
    want = oracle.louvain(g)
    base = free_bytes()
    failed = 0
    for k in range(1, 200):
        os.environ["LV_FAULT_ALLOC_AT"] = str(k)
        try:
            h = lvp.Graph.from_csr(g, validate=True)
        except lvp.LvError as e:
            assert e.status == LV_E_NOMEM, f"k={k}: {e}"
            failed += 1
            continue
        finally:
            os.environ.pop("LV_FAULT_ALLOC_AT", None)
        with h:
            got = lvp.louvain(h)
        assert np.array_equal(got.final_labels, want.final_labels)
        break
    say(f"create: {failed} allocation points forced to fail")
    assert failed > 3
    assert abs(free_bytes() - base) < (32 << 20)
