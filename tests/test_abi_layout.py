"""The ctypes structures of the binding have the layout of include/pp.h.

A small C program compiled with the host compiler prints sizeof and the
offset of every field of the public structs; the binding must agree field by
field (a mismatch would make the library write outside the caller's records).
"""
import ctypes
import os
import subprocess

import pytest

from paper_2502_10640_amd import pp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = {"pp_bunch": pp.Bunch, "pp_state": pp.State, "pp_diag": pp.Diag, "pp_tuning": pp.Tuning,
           "pp_profile": pp.Profile}


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    d = tmp_path_factory.mktemp("layout")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "pp.h"', "int main(void) {"]
    for cname, cls in STRUCTS.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    res = {}
    for line in out.splitlines():
        s, f, v = line.split()
        res[(s, f)] = int(v)
    return res


@pytest.mark.parametrize("cname", list(STRUCTS))
def test_struct_layout_matches_header(c_layout, cname):
    cls = STRUCTS[cname]
    assert ctypes.sizeof(cls) == c_layout[(cname, "sizeof")]
    for f, _ in cls._fields_:
        assert getattr(cls, f).offset == c_layout[(cname, f)], (cname, f)
