"""CPU check that the Python binding's ctypes structures match the C ABI.

A small C program, compiled with gcc against include/sph.h, prints sizeof and
offsetof of every field of every public structure; each must equal what
ctypes computes for the binding's structure of the same name, field by field.
A mismatch would pass silently garbled parameters or reports across the ABI.
"""
import ctypes
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = {            # C type -> binding class name
    "sph_params": "Params",
    "sph_body": "Body",
    "sph_report": "Report",
    "sph_body_report": "BodyReport",
    "sph_shape": "Shape",
    "sph_relax_report": "RelaxReport",
    "sph_allocator": "Allocator",
}


def c_layout(tmp_path):
    from paper_2512_09904_amd import sph
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "sph.h"', "int main(void) {"]
    for ctype, pyname in STRUCTS.items():
        cls = getattr(sph, pyname)
        lines.append(f'  printf("{ctype} #sizeof %zu\\n", sizeof({ctype}));')
        for name, _ in cls._fields_:
            lines.append(f'  printf("{ctype} {name} %zu\\n", offsetof({ctype}, {name}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-Wall", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)], text=True)
    table = {}
    for ln in out.splitlines():
        ctype, field, val = ln.split()
        table[(ctype, field)] = int(val)
    return table


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_ctypes_structures_match_the_header(tmp_path):
    from paper_2512_09904_amd import sph
    table = c_layout(tmp_path)
    for ctype, pyname in STRUCTS.items():
        cls = getattr(sph, pyname)
        assert ctypes.sizeof(cls) == table[(ctype, "#sizeof")], ctype
        for name, _ in cls._fields_:
            assert getattr(cls, name).offset == table[(ctype, name)], (ctype, name)
