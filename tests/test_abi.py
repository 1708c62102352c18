"""The C ABI library loads and exports what include/tcmis.h declares; host-side
argument checks return their documented codes before any device work (no GPU needed)."""
import ctypes
import os
import re

import pytest

from conftest import ROOT
from paper_2605_29604_amd import tcmis

HEADER = os.path.join(ROOT, "include", "tcmis.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mis_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(tcmis.LIB_PATH):
        pytest.fail("libtcmis.so is not built (run __graft_entry__.build())")
    return tcmis.lib()


def test_exports_match_header(L):
    decl = declared_functions()
    assert decl, "no functions parsed from the header"
    assert sorted(tcmis.EXPORTS) == decl
    for name in decl:
        assert hasattr(L, name), name


def test_strings(L):
    assert L.mis_version().decode().startswith("tcmis")
    assert L.mis_status_string(0).decode() == "ok"
    assert L.mis_status_string(-2).decode() == "adjacency not symmetric"
    assert L.mis_status_string(12345).decode() == "unknown status"


def test_default_opts(L):
    o = tcmis.MisBuildOpts()
    L.mis_default_opts(ctypes.byref(o))
    assert (o.path, o.tile, o.reorder, o.orient, o.validate, o.seed) == (0, 0, 0, -1, 0, 1)


def test_host_argument_errors(L):
    h = ctypes.c_void_p(None)
    csr = tcmis.MisCsr(10, 0, ctypes.c_void_p(8), None)
    assert L.mis_build_tiles(ctypes.byref(csr), None, None, None) == tcmis.MIS_EINVAL
    assert L.mis_build_tiles(None, None, None, ctypes.byref(h)) == tcmis.MIS_EINVAL
    bad = tcmis.MisCsr(-1, 0, ctypes.c_void_p(8), None)
    assert L.mis_build_tiles(ctypes.byref(bad), None, None, ctypes.byref(h)) == tcmis.MIS_EINVAL
    nul = tcmis.MisCsr(10, 5, None, None)
    assert L.mis_build_tiles(ctypes.byref(nul), None, None, ctypes.byref(h)) == tcmis.MIS_EINVAL
    nocol = tcmis.MisCsr(10, 5, ctypes.c_void_p(8), None)
    assert L.mis_build_tiles(ctypes.byref(nocol), None, None, ctypes.byref(h)) == tcmis.MIS_EINVAL
    for field, value in (("tile", 8), ("path", 7), ("reorder", 9), ("orient", 2), ("poll_rounds", -1)):
        o = tcmis.MisBuildOpts()
        L.mis_default_opts(ctypes.byref(o))
        setattr(o, field, value)
        assert L.mis_build_tiles(ctypes.byref(csr), ctypes.byref(o), None, ctypes.byref(h)) == tcmis.MIS_EINVAL
        assert field.split("_")[0] in L.mis_last_error().decode()
    big = tcmis.MisCsr((1 << 24) + 1, 0, ctypes.c_void_p(8), None)
    assert L.mis_build_tiles(ctypes.byref(big), None, None, ctypes.byref(h)) == tcmis.MIS_EINVAL
    assert "2^24" in L.mis_last_error().decode()
    assert not h.value
    assert L.mis_solve(None, None, 0, None, None) == tcmis.MIS_EINVAL
    assert L.mis_solve_batch(None, -1, None, None, None) == tcmis.MIS_EINVAL
    assert L.mis_solve_batch(None, 2, None, None, None) == tcmis.MIS_EINVAL
    assert L.mis_graph_bytes(None, None) == tcmis.MIS_EINVAL
    L.mis_free_tiles(None)
