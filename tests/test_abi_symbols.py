"""The C-ABI library loads and exports every entry point include/lv.h declares (no GPU needed)."""
import ctypes
import os
import re

import paper_2507_06471_amd as lvp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(lv_[a-z0-9_]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    lib = lvp.load_library()
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert declared_functions() <= set(lvp.SIGNATURES)


def test_status_strings_without_gpu():
    lib = lvp.load_library()
    assert lib.lv_status_str(0) == b"ok"
    assert lib.lv_status_str(3) == b"asymmetric graph"


def test_params_default_without_gpu():
    p, _ = lvp.make_params()
    assert (p.max_sweeps, p.max_levels, p.lpa_threshold, p.flags) == (20, 32, 0, 0)


def test_null_arguments_rejected_without_gpu():
    lib = lvp.load_library()
    out = ctypes.c_void_p()
    assert lib.lv_graph_create_csr(-1, None, None, None, 0, 0, None, ctypes.byref(out)) == 1
    assert lib.lv_louvain(None, None, ctypes.byref(out)) == 1
    assert lib.lv_graph_destroy(None) == 1
