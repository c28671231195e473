"""The Python binding's structures match the C header byte for byte: a small
C program built with the host compiler prints the size and every field offset
of each struct in include/ccfr.h, and ctypes must agree."""
import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2607_26901_amd import ccfr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = {
    "ccfr_params": ccfr.Params,
    "ccfr_candidates": ccfr.Candidates,
    "ccfr_regions": ccfr.Regions,
    "ccfr_step_params": ccfr.StepParams,
    "ccfr_tuning": ccfr.Tuning,
    "ccfr_status_info": ccfr.StatusInfo,
}


@pytest.fixture(scope="module")
def layout(tmp_path_factory):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    d = tmp_path_factory.mktemp("abi")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ccfr.h"', "int main(void) {"]
    for name, cls in STRUCTS.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for f in cls._fields_:
            lines.append(f'printf("{name} {f[0]} %zu\\n", offsetof({name}, {f[0]}));')
    lines.append('printf("ccfr_halfspace size %zu\\n", sizeof(ccfr_halfspace));')
    for f in ccfr.HALFSPACE_DTYPE.names:
        lines.append(f'printf("ccfr_halfspace {f} %zu\\n", offsetof(ccfr_halfspace, {f}));')
    lines += ["return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    table = {}
    for line in out.splitlines():
        s, f, v = line.split()
        table[(s, f)] = int(v)
    return table


@pytest.mark.parametrize("name", list(STRUCTS))
def test_struct_matches_header(layout, name):
    cls = STRUCTS[name]
    assert C.sizeof(cls) == layout[(name, "size")], name
    for f in cls._fields_:
        assert getattr(cls, f[0]).offset == layout[(name, f[0])], (name, f[0])


def test_halfspace_dtype_matches_header(layout):
    dt = ccfr.HALFSPACE_DTYPE
    assert dt.itemsize == layout[("ccfr_halfspace", "size")]
    for f in dt.names:
        assert dt.fields[f][1] == layout[("ccfr_halfspace", f)], f
