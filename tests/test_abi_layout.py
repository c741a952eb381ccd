"""The binding's ctypes structures against the C declarations in include/:
size and every field's offset, from a small C program compiled with the host
compiler (no GPU; the library is not loaded)."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_1801_08655_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = ["helm_grid", "helm_options", "helm_solve_info", "helm_factor_info",
           "helm_kernel_stat", "helm_tile_choice", "helm_server_options", "helm_request_info",
           "helm_server_summary", "helm_problem", "helm_batch_options", "helm_problem_info",
           "helm_batch_summary"]


def _c_layout(tmp_path):
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "helm.h"',
             '#include "helm_serve.h"', '#include "helm_batch.h"', 'int main(void) {']
    for name in STRUCTS:
        cls = getattr(_lib, name)
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {tuple(l.split()[:2]): int(l.split()[2]) for l in out.splitlines()}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_ctypes_structures_match_the_headers(tmp_path):
    c = _c_layout(tmp_path)
    for name in STRUCTS:
        cls = getattr(_lib, name)
        assert ctypes.sizeof(cls) == c[(name, "size")], name
        for field, _ in cls._fields_:
            assert getattr(cls, field).offset == c[(name, field)], (name, field)
