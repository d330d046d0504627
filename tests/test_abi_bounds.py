"""Size bounds the C ABI enforces on the host before any GPU work (no GPU needed).

The row loops of the move, aggregation and scatter kernels step 32-bit entry
counters by up to 2^13 past a row's end, so the library accepts at most
LV_MAX_NNZ = 2^31 - 1 - 2^16 CSR entries per handle (one graph, or a packed
set of graphs) and rejects more with LV_E_OVERFLOW, checked on host-resident
offsets before the device is touched."""
import ctypes
import os
import re

import numpy as np

import paper_2507_06471_amd as lvp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LV_E_OVERFLOW = 5
MAX_ROW_STEP = 1 << 13  # the largest per-iteration step of a row loop (1024 lanes x 8 entries)


def header_max_nnz() -> int:
    text = open(os.path.join(ROOT, "include", "lv.h")).read()
    m = re.search(r"#define\s+LV_MAX_NNZ\s+\((\d+)\s*-\s*(\d+)\)", text)
    return int(m.group(1)) - int(m.group(2))


def test_bound_leaves_room_for_every_row_step():
    bound = header_max_nnz()
    assert bound == (1 << 31) - 1 - (1 << 16)
    # the last row's counter, at most one step past the last entry, stays below 2^31
    assert bound + MAX_ROW_STEP < (1 << 31) - 1


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def test_create_csr_rejects_too_many_entries_without_gpu():
    lib = lvp.load_library()
    bound = header_max_nnz()
    off = np.array([0, bound + 1], dtype=np.int32)
    dummy = np.zeros(1, dtype=np.int32)  # never read: the bound is checked first
    out = ctypes.c_void_p(12345)
    st = lib.lv_graph_create_csr(1, _ptr(off), _ptr(dummy), None, 0, 0, None, ctypes.byref(out))
    assert st == LV_E_OVERFLOW
    assert out.value == 12345  # out-parameters are written only on success


def test_create_batch_rejects_too_many_packed_entries_without_gpu():
    lib = lvp.load_library()
    # two graphs of 2^30 entries each: together above the bound
    offs = [np.array([0, 1 << 30], dtype=np.int32) for _ in range(2)]
    dummy = np.zeros(1, dtype=np.int32)
    ns = np.array([1, 1], dtype=np.int32)
    P = ctypes.POINTER(ctypes.c_int32)
    off_arr = (P * 2)(*[_ptr(o) for o in offs])
    idx_arr = (P * 2)(_ptr(dummy), _ptr(dummy))
    out = ctypes.c_void_p(0)
    st = lib.lv_graph_create_batch(2, _ptr(ns), off_arr, idx_arr, None, 0, 0, None, ctypes.byref(out))
    assert st == LV_E_OVERFLOW
    assert out.value is None
