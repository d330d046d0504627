"""Host logic of bench.py: the digest that ties stored counter records to the
move kernels' code."""
import os
import shutil
import sys

sys.path.insert(0, os.path.join(os.path.dirname(__file__), ".."))

import bench  # noqa: E402


def _copy_sources(tmp_path):
    src = os.path.join(bench.ROOT, "paper_2507_06471_amd", "csrc")
    dst = tmp_path / "paper_2507_06471_amd" / "csrc"
    dst.mkdir(parents=True)
    for f in bench.KERNEL_SOURCES:
        shutil.copy(os.path.join(src, f), dst / f)
    return dst


def test_digest_ignores_comments_not_code(tmp_path, monkeypatch):
    d = _copy_sources(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    base = bench.kernel_source_digest()
    assert base == bench.kernel_source_digest()

    p = d / "lv_internal.h"
    text = p.read_text()
    # reworded comments and re-indented lines keep the record
    p.write_text("// a new first line\n/* a block\n   comment */\n" + text.replace("\n", "\n  "))
    assert bench.kernel_source_digest() == base

    # a changed constant does not
    assert "L4_SLOTS = 16" in text
    p.write_text(text.replace("L4_SLOTS = 16", "L4_SLOTS = 32"))
    assert bench.kernel_source_digest() != base
