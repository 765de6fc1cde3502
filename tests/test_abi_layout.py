"""The ctypes structures of the Python binding against the C header: every
structure's size and every field's offset, read from a C program built with
gcc against include/mbp.h (CPU only; nothing is loaded or launched)."""
import ctypes as C
import os
import shutil
import subprocess

import pytest

import paper_2106_03583_amd as m

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# binding structure -> C typedef of the same layout
PAIRS = [
    (m.BlockDesc, "mbp_block_desc"),
    (m.SynthDesc, "mbp_synth_desc"),
    (m.Options, "mbp_options"),
    (m.SolveInfo, "mbp_solve_info"),
    (m.ProfileInfo, "mbp_profile_info"),
    (m.Tuning, "mbp_tuning"),
    (m.PlanSummary, "mbp_plan_summary"),
]


def _c_layout(tmp_path):
    lines = ['#include <stdio.h>', '#include "mbp.h"', "int main(void) {"]
    for py, cname in PAIRS:
        lines.append(f'    printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'    printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
                        "-o", str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60, check=True).stdout
    table = {}
    for line in out.splitlines():
        cname, what, value = line.split()
        table[(cname, what)] = int(value)
    return table


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_binding_structs_match_header(tmp_path):
    table = _c_layout(tmp_path)
    for py, cname in PAIRS:
        assert C.sizeof(py) == table[(cname, "size")], (cname, C.sizeof(py), table[(cname, "size")])
        for field, _ in py._fields_:
            off = getattr(py, field).offset
            assert off == table[(cname, field)], (cname, field, off, table[(cname, field)])
