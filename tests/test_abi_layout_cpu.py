"""The ctypes mirrors of the C-ABI structures (paper_1403_4747_amd/fda.py)
match include/fda.h field by field: a C program built with the host compiler
prints sizeof and offsetof of every field, compared with ctypes."""
import os
import shutil
import subprocess

import pytest

from paper_1403_4747_amd import fda as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PAIRS = [("fda_options", F.Options), ("fda_stats", F.Stats), ("fda_profile_result", F.ProfileResult),
         ("fda_m2l_config", F.M2LConfig), ("fda_tune_result", F.TuneResult), ("bm_stats", F.SolveStats)]


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    d = tmp_path_factory.mktemp("abi")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "fda.h"', "int main(void) {"]
    for cname, cls in PAIRS:
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    lay = {}
    for ln in out.splitlines():
        c, f, v = ln.split()
        lay[(c, f)] = int(v)
    return lay


@pytest.mark.parametrize("cname,cls", PAIRS, ids=[p[0] for p in PAIRS])
def test_ctypes_structure_matches_header(c_layout, cname, cls):
    assert c_layout[(cname, "sizeof")] == ctypes_sizeof(cls)
    for fname, _ in cls._fields_:
        assert c_layout[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


def ctypes_sizeof(cls):
    import ctypes

    return ctypes.sizeof(cls)
