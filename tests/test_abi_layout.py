"""The ctypes structures of the binding have the layout of the C structures
include/oi.h declares: the header is compiled by the host C compiler and
every field's offset, and each structure's size, must agree."""
import ctypes as C
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = ("oi_result", "oi_timing", "oi_autotune_result")


def _c_name(field):
    # Python keywords carry a trailing underscore in the binding
    return field[:-1] if field.endswith("_") else field


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs a host C compiler")
def test_struct_layouts_match_the_header(tmp_path):
    from paper_1704_04794_amd import _binding
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "oi.h"', "int main(void) {"]
    expect = {}
    for name in STRUCTS:
        cls = getattr(_binding, name)
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        expect[name] = C.sizeof(cls)
        for field, _ in cls._fields_:
            key = f"{name}.{field}"
            lines.append(f'  printf("{key} %zu\\n", offsetof({name}, {_c_name(field)}));')
            expect[key] = getattr(cls, field).offset
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {k: int(v) for k, v in (line.split() for line in out.splitlines())}
    assert got == expect
