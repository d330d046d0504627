"""The binding's ctypes structures against the C header: a program compiled
with gcc from include/lv.h prints every struct's size and field offsets."""
import ctypes
import os
import shutil
import subprocess

import pytest

import paper_2507_06471_amd as lvp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = ["lv_tuning", "lv_params", "lv_level_info", "lv_server_config", "lv_job_info", "lv_server_stats"]


def c_layout(tmp_path):
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "lv.h"', "int main(void) {"]
    for name in STRUCTS:
        cls = getattr(lvp, name)
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{name}.{field} %zu\\n", offsetof({name}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    exe = tmp_path / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return dict((k, int(v)) for k, v in (line.split() for line in out.splitlines()))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_ctypes_structs_match_the_header(tmp_path):
    want = c_layout(tmp_path)
    for name in STRUCTS:
        cls = getattr(lvp, name)
        assert ctypes.sizeof(cls) == want[name], name
        for field, _ in cls._fields_:
            assert getattr(cls, field).offset == want[f"{name}.{field}"], f"{name}.{field}"
