"""The ctypes structs of the binding have the C layout of include/ertvie.h: a small C
program built with the host compiler prints sizeof and offsetof of every field, and each
must equal the binding's (a mismatch would have the library read or write past a struct,
or read the wrong fields).  CPU only."""
import ctypes
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# C struct name -> binding class name
STRUCTS = {"ert_vie_opts": "VieOpts", "ert_solve_opts": "SolveOpts", "ert_solve_info": "SolveInfo",
           "ert_net_opts": "NetOpts", "ert_net_train_opts": "NetTrainOpts", "ert_fmm_info": "FmmInfo",
           "ert_fft_info": "FftInfo"}


def _c_layout(tmp_path, classes):
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ertvie.h"', 'int main(void) {']
    for cname, cls in classes.items():
        lines.append('printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in cls._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines += ['return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        a, b, c = line.split()
        got[(a, b)] = int(c)
    return got


def test_binding_structs_match_header(tmp_path):
    from paper_1610_00835_amd import ertvie
    classes = {c: getattr(ertvie, py) for c, py in STRUCTS.items()}
    got = _c_layout(tmp_path, classes)
    for cname, cls in classes.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
