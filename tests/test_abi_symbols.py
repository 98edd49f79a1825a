"""The C-ABI library loads on the host and exports every symbol include/amr_lbm.h
declares; configuration checks and the arena size query run without a GPU."""
import ctypes as C
import os
import re

import pytest

from paper_2308_08085_amd import abi, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "amr_lbm.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+char\s*\*\s*|amr_status\s+)(\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("amr_query_bytes", "amr_create", "amr_tag", "amr_adapt", "lbm_step", "amr_fields", "amr_destroy",
              "amr_last_error"):
        assert n in names
    assert set(names) == set(abi.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = abi.load()
    for n in _declared():
        assert hasattr(lib, n), n
    out = os.popen("nm -D --defined-only %s" % abi.LIB_PATH).read()
    for n in _declared():
        assert re.search(r"\bT %s$" % n, out, flags=re.M), n


def test_query_bytes_and_argument_errors_on_host():
    case = W.config2()
    nbytes = abi.query_bytes(case, "f32s")
    cap, capc = case.cap, case.cap * 64
    assert nbytes >= 2 * 19 * capc * 4 + 2 * 27 * cap * 4
    assert abi.query_bytes(case, "f16s") < nbytes < abi.query_bytes(case, "f64")
    bad = W.config2()
    bad.q = 15
    with pytest.raises(abi.AmrError) as e:
        abi.query_bytes(bad)
    assert e.value.code == abi.AMR_ERR_ARG
    assert "lattice" in str(e.value)
    bad = W.config2()
    bad.cap = 10
    with pytest.raises(abi.AmrError):
        abi.query_bytes(bad)
    lib = abi.load()
    out = C.c_uint64(0)
    assert lib.amr_query_bytes(None, C.byref(out)) == abi.AMR_ERR_ARG
    assert lib.amr_destroy(None) == abi.AMR_OK
    # a handle is never created without a device buffer
    cfg = abi.make_config(W.config1())
    h = C.c_void_p(0)
    assert lib.amr_create(C.byref(cfg), None, C.c_uint64(0), None, C.byref(h)) == abi.AMR_ERR_ARG
    assert not h.value
