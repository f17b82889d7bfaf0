"""CPU: the ctypes mirrors of the C-ABI structs have the layout of include/pimd.h.

A small C program built with the host compiler prints sizeof and the offset of
every field of each struct; the Python mirrors must agree field for field, so a
field added to the header but not to the binding (or the other way round) fails
here rather than as a silently shifted argument on the GPU.
"""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2503_23728_amd import abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = ["pimd_bpnn_model", "pimd_gfn_model", "pimd_metad", "pimd_config", "pimd_tuning", "pimd_estimates"]


def _c_layout(tmp_path):
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "pimd.h"', "int main(void) {"]
    for name in STRUCTS:
        lines.append(f'    printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in getattr(abi, name)._fields_:
            lines.append(f'    printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ["    return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    r = subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    return {tuple(l.split()[:2]): int(l.split()[2]) for l in out.splitlines()}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs a host C compiler")
def test_ctypes_mirrors_match_the_header(tmp_path):
    c = _c_layout(tmp_path)
    for name in STRUCTS:
        cls = getattr(abi, name)
        assert ctypes.sizeof(cls) == c[(name, "size")], name
        for field, _ in cls._fields_:
            assert getattr(cls, field).offset == c[(name, field)], (name, field)
