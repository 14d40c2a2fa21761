"""The Python binding mirrors include/spmv.h: every SPMV_* constant has the
header's value, and the ctypes structures have the C structures' size and
field offsets (a small C program built with gcc prints the C side).  No GPU."""
from __future__ import annotations

import ctypes
import os
import re
import subprocess
import tempfile

from paper_1106_5908_amd import spmv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spmv.h")


def header_defines():
    out = {}
    with open(HEADER) as f:
        for line in f:
            m = re.match(r"#define\s+(SPMV_\w+)\s+(-?\d+|0x[0-9a-fA-F]+)u?\b", line)
            if m:
                out[m.group(1)] = int(m.group(2), 0)
    return out


def test_constants_match_header():
    defs = header_defines()
    assert len(defs) > 20
    for name, value in defs.items():
        assert hasattr(spmv, name), name
        assert getattr(spmv, name) == value, name


def test_struct_layouts_match_header():
    structs = {"spmv_info_t": spmv.spmv_info_t, "spmv_plan_t": spmv.spmv_plan_t}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "spmv.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for field, _ in py._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "layout.c"), os.path.join(d, "layout")
        with open(src, "w") as f:
            f.write("\n".join(lines) + "\n")
        subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), src, "-o", exe])
        got = subprocess.check_output([exe], text=True).split("\n")
    c_side = {}
    for ln in got:
        if ln:
            name, field, val = ln.split()
            c_side[(name, field)] = int(val)
    for cname, py in structs.items():
        assert c_side[(cname, "size")] == ctypes.sizeof(py), cname
        for field, _ in py._fields_:
            assert c_side[(cname, field)] == getattr(py, field).offset, (cname, field)
