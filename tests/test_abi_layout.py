"""The ctypes mirrors of the C-ABI's structs match the header: size and every
member's offset, read from a small C program compiled against the header
with the host compiler."""
import ctypes as C
import os
import shutil
import subprocess
import tempfile

import pytest

from paper_2603_00413_amd import binding as B
from paper_2603_00413_amd import serve as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = [
    ("dt_env", B._Env), ("dt_absorption", B._Absorption), ("dt_field", B._Field),
    ("dt_scene", B._Scene), ("dt_timing", B._Timing), ("dt_trace_params", B._Params),
    ("dt_camera", B._Camera), ("dt_rays", B._Rays), ("dt_serve_scene", S._ServeScene),
    ("dt_serve_admit", S._Admit),
]


def _c_layout():
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "difftrans.h"', "int main(void) {"]
    for cname, py in STRUCTS:
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in py._fields_:
            lines.append(f'  printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ["  return 0;", "}"]
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    with tempfile.TemporaryDirectory() as t:
        src, exe = os.path.join(t, "layout.c"), os.path.join(t, "layout")
        with open(src, "w") as fh:
            fh.write("\n".join(lines) + "\n")
        subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    got = {}
    for ln in out.splitlines():
        parts = ln.split()
        got[(parts[0], parts[1])] = int(parts[2])
    return got


def test_ctypes_structs_match_the_header():
    got = _c_layout()
    for cname, py in STRUCTS:
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f in py._fields_:
            assert got[(cname, f[0])] == getattr(py, f[0]).offset, (cname, f[0])
