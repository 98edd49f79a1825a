"""The binding's ctypes structures have the layout of the structs that
include/amr_lbm.h declares: sizes and field offsets as the host C compiler
lays them out (a mismatch would corrupt every call silently)."""
import ctypes as C
import os
import shutil
import subprocess

import pytest

from paper_2308_08085_amd import abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PAIRS = [(abi.Config, "amr_config"), (abi.TagParams, "amr_tag_params"), (abi.AdaptStats, "amr_adapt_stats"),
         (abi.BatchTuning, "amr_batch_tuning")]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_ctypes_structures_match_the_header(tmp_path):
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "amr_lbm.h"', "int main(void) {"]
    for cls, cname in PAIRS:
        lines.append('printf("%s sizeof %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in cls._fields_:
            lines.append('printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for line in out.splitlines():
        name, field, value = line.split()
        got[(name, field)] = int(value)
    for cls, cname in PAIRS:
        assert got[(cname, "sizeof")] == C.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
