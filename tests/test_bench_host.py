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


def test_measured_traffic_scales_by_the_copy_factors(tmp_path, monkeypatch):
    src = bench.kernel_source_digest()
    f = tmp_path / "pmc.txt"
    f.write_text("# header line\n"
                 f"slot=hub/scatter kernel=k fetch_kib=1000.0 write_kib=300.0 copy_fetch_factor=0.5000 "
                 f"copy_write_factor=1.0000 src={src}\n"
                 f"slot=l8k kernel=k2 fetch_kib=10.0 write_kib=0.0 copy_fetch_factor=0.5000 "
                 f"copy_write_factor=1.0000 src=0000000000000000\n")
    monkeypatch.setattr(bench, "PMC_FILE", str(f))
    # (1000 / 0.5 + 300 / 1.0) KiB
    assert bench.measured_traffic("hub/scatter") == (2000 + 300) * 1024
    # a record taken from other kernel code, or no record, gives no figure
    assert bench.measured_traffic("l8k") is None
    assert bench.measured_traffic("l1k") is None
    monkeypatch.setattr(bench, "PMC_FILE", str(tmp_path / "absent.txt"))
    assert bench.measured_traffic("hub/scatter") is None


def test_committed_counters_describe_the_current_kernels():
    # the stored record of the dominant kernel matches the sources it is read with
    assert bench.measured_traffic("hub/scatter") is not None
