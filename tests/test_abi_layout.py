"""The ctypes mirrors of the C ABI's structs have the header's layout.

A small C program, compiled against include/leja_logdet.h with the host C
compiler, prints sizeof and offsetof of every field of ld_csr, ld_options and
ld_stats; they must equal the ctypes declarations the Python binding passes.
"""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2603_02207_amd import _native as nat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_struct_layout_matches_header(tmp_path):
    structs = {"ld_csr": nat.LdCsr, "ld_options": nat.LdOptions, "ld_stats": nat.LdStats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "leja_logdet.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            a, b, c = line.split()
            got[(a, b)] = int(c)
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for field, _ in cls._fields_:
            assert got[(cname, field)] == getattr(cls, field).offset, (cname, field)
