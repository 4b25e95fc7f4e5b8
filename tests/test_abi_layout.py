"""The ctypes mirrors of the C-ABI structs (paper_2605_15418_amd/rw.py) have the
layout include/rw.h gives them: a C program compiled by gcc against the header
prints every field's offset and size and each struct's size, and the ctypes
fields must agree, in the header's order (CPU only)."""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = ("rw_surface", "rw_doe_desc", "rw_param_ref", "rw_config", "rw_stats", "rw_profile")


def _header_fields():
    """Field names of each typedef'd struct of rw.h, in declaration order."""
    src = open(os.path.join(ROOT, "include", "rw.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    out = {}
    for m in re.finditer(r"typedef struct\s*\w*\s*\{(.*?)\}\s*(\w+)\s*;", src, re.S):
        names = []
        for decl in (d.strip() for d in m.group(1).split(";")):
            if not decl:
                continue
            # "double n_A, n_B" -> n_A, n_B; "double asph[4]" -> asph; pointers keep the name
            first, *rest = decl.split(",")
            names.append(re.findall(r"(\w+)\s*(?:\[[^\]]*\])?\s*$", first)[0])
            names += [re.findall(r"(\w+)", r)[0] for r in rest]
        out[m.group(2)] = names
    return out


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    fields = _header_fields()
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "rw.h"', "int main(void) {"]
    for s in STRUCTS:
        lines.append(f'  printf("{s} size %zu\\n", sizeof({s}));')
        for f in fields[s]:
            lines.append(f'  printf("{s} {f} %zu %zu\\n", offsetof({s}, {f}), '
                         f'sizeof((({s}*)0)->{f}));')
    lines += ["  return 0;", "}"]
    d = tmp_path_factory.mktemp("abi")
    c = d / "layout.c"
    c.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(c)],
                   check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    size, field = {}, {}
    for line in out.splitlines():
        p = line.split()
        if p[1] == "size":
            size[p[0]] = int(p[2])
        else:
            field[(p[0], p[1])] = (int(p[2]), int(p[3]))
    return fields, size, field


@pytest.mark.parametrize("name", STRUCTS)
def test_ctypes_struct_matches_the_header(c_layout, name):
    from paper_2605_15418_amd import rw as R
    fields, size, field = c_layout
    cls = getattr(R, name)
    assert [f[0] for f in cls._fields_] == fields[name]
    for fname, ftype in cls._fields_:
        off, sz = field[(name, fname)]
        assert getattr(cls, fname).offset == off, (name, fname)
        assert ctypes.sizeof(ftype) == sz, (name, fname)
    assert ctypes.sizeof(cls) == size[name]
