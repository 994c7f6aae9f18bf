"""The ctypes mirrors of the C ABI's structs (paper_1804_04640_amd/_lib.py)
have the sizes and field offsets the header gives them, checked against a
C program compiled from include/fastcount.h with the host compiler."""
import ctypes
import os
import shutil
import subprocess
import tempfile

import pytest

from paper_1804_04640_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = {
    "fc_tuning": _lib.fc_tuning,
    "fc_pair_rec": _lib.fc_pair_rec,
    "fc_kernel_stat": _lib.fc_kernel_stat,
    "fc_reduce_params": _lib.fc_reduce_params,
}


def c_layout():
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "fastcount.h"', "int main(void) {"]
    for name, cls in STRUCTS.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (name, name))
        for field, _ in cls._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (name, field, name, field))
    lines.append("return 0; }")
    with tempfile.TemporaryDirectory() as d:
        src, exe = os.path.join(d, "layout.c"), os.path.join(d, "layout")
        with open(src, "w") as f:
            f.write("\n".join(lines) + "\n")
        subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), src, "-o", exe],
                       check=True, capture_output=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        a, b, v = line.split()
        got[(a, b)] = int(v)
    return got


def test_struct_sizes_and_offsets_match_the_header():
    got = c_layout()
    for name, cls in STRUCTS.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)
