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


def build(L, csr, opts, ws, ws_bytes, h):
    return L.mis_build_tiles(ctypes.byref(csr) if csr is not None else None,
                             ctypes.byref(opts) if opts is not None else None, ws, ws_bytes, None, h)


def test_host_argument_errors(L):
    h = ctypes.c_void_p(None)
    hp = ctypes.byref(h)
    ws = ctypes.c_void_p(1 << 20)   # never dereferenced: every call below fails on the host
    csr = tcmis.MisCsr(10, 0, ctypes.c_void_p(256), None)
    assert build(L, csr, None, ws, 1 << 40, None) == tcmis.MIS_EINVAL
    assert build(L, None, None, ws, 1 << 40, hp) == tcmis.MIS_EINVAL
    for bad in (tcmis.MisCsr(-1, 0, ctypes.c_void_p(256), None), tcmis.MisCsr(10, 5, None, None),
                tcmis.MisCsr(10, 5, ctypes.c_void_p(256), None), tcmis.MisCsr(10, 1 << 40, ctypes.c_void_p(256),
                                                                               ctypes.c_void_p(256))):
        assert build(L, bad, None, ws, 1 << 40, hp) == tcmis.MIS_EINVAL
    # 2^31 entries and more: the hybrid path only (64-bit entry offsets)
    wide = tcmis.MisCsr(10, 1 << 31, ctypes.c_void_p(256), ctypes.c_void_p(256))
    for path in ("tile", "csr"):
        assert build(L, wide, tcmis._opts(path=path), ws, 1 << 40, hp) == tcmis.MIS_EINVAL
        assert "2^31" in L.mis_last_error().decode()
    assert tcmis.mis_build_bytes(10, 1 << 31, path="hybrid") > (1 << 33)
    for field, value in (("tile", 8), ("path", 7), ("reorder", 9), ("orient", 2), ("poll_rounds", -1),
                         ("dense_min", -2), ("key_rule", 3), ("timing", 2), ("dyn_slack", -1)):
        o = tcmis.MisBuildOpts()
        L.mis_default_opts(ctypes.byref(o))
        setattr(o, field, value)
        assert build(L, csr, o, ws, 1 << 40, hp) == tcmis.MIS_EINVAL
        assert field.split("_")[0] in L.mis_last_error().decode()
    big = tcmis.MisCsr((1 << 24) + 1, 0, ctypes.c_void_p(256), None)
    assert build(L, big, None, ws, 1 << 40, hp) == tcmis.MIS_EINVAL
    assert "2^24" in L.mis_last_error().decode()
    # workspace checks: size from mis_build_bytes, alignment
    need = ctypes.c_size_t(0)
    assert L.mis_build_bytes(ctypes.byref(csr), None, ctypes.byref(need)) == 0 and need.value > 0
    assert build(L, csr, None, ws, need.value - 1, hp) == tcmis.MIS_EINVAL
    assert "workspace" in L.mis_last_error().decode()
    assert build(L, csr, None, ctypes.c_void_p((1 << 20) + 64), need.value, hp) == tcmis.MIS_EINVAL
    assert build(L, csr, None, None, need.value, hp) == tcmis.MIS_EINVAL
    assert not h.value
    assert L.mis_solve(None, None, 0, None, 0, None, None) == tcmis.MIS_EINVAL
    assert L.mis_solve_scratch_bytes(None, None) == tcmis.MIS_EINVAL
    assert L.mis_session_step(None, None) == tcmis.MIS_EINVAL
    assert L.mis_session_poll(None, 0, None, 0, None) == tcmis.MIS_EINVAL
    assert L.mis_graph_bytes(None, None) == tcmis.MIS_EINVAL
    L.mis_free_tiles(None)


def test_build_bytes_scaling(L):
    # footprint grows with the graph and is larger for tiles than for the CSR path
    small = tcmis.mis_build_bytes(1000, 8000, path="csr")
    big = tcmis.mis_build_bytes(100000, 800000, path="csr")
    big2 = tcmis.mis_build_bytes(200000, 1600000, path="csr")
    assert 1.8 < (big2 - small) / (big - small) < 2.2     # linear in the graph size
    assert tcmis.mis_build_bytes(100000, 800000, path="tile", tile=32, orient=0) > \
        tcmis.mis_build_bytes(100000, 800000, path="tile", tile=16, orient=1) > big


def test_batch_argument_errors(L):
    n = 10
    ok = [0, 4, 10]
    assert tcmis.mis_build_batch_bytes(n, 20, ok, path="tile") > tcmis.mis_build_bytes(n, 20, path="tile")
    for bad in ([0, 4, 9], [1, 4, 10], [0, 6, 4, 10]):
        with pytest.raises(tcmis.MisError) as ei:
            tcmis.mis_build_batch_bytes(n, 20, bad)
        assert ei.value.code == tcmis.MIS_EINVAL
    with pytest.raises(tcmis.MisError):
        tcmis.mis_build_batch_bytes((1 << 24) + 10, 0, [0, (1 << 24) + 10])   # one graph too large for the key rule
    assert tcmis.mis_build_batch_bytes((1 << 24) + 10, 0, [0, 1 << 23, (1 << 24) + 10]) > 0
    assert L.mis_solve_union(None, None, None, None, None, None) == tcmis.MIS_EINVAL
    assert L.mis_solve_batch(None, 1, None, None, 0, None, None, None, None) == tcmis.MIS_EINVAL
    assert L.mis_solve_batch_scratch_bytes(None, 1, None) == tcmis.MIS_EINVAL


def test_autotune_argument_errors(L):
    csr = tcmis.MisCsr(1000, 8000, ctypes.c_void_p(256), ctypes.c_void_p(256))
    need = ctypes.c_size_t(0)
    assert L.mis_autotune_bytes(ctypes.byref(csr), 0, None, None, ctypes.byref(need)) == 0
    # room for the largest trial build plus the trial output
    for path, tile in (("tile", 16), ("tile", 32), ("csr", 0)):
        one = tcmis.mis_build_bytes(1000, 8000, path=path, tile=tile)
        assert need.value >= one + 1000
    out = tcmis.MisBuildOpts()
    ws = ctypes.c_void_p(1 << 20)   # never dereferenced: every call below fails on the host
    assert L.mis_autotune(None, 0, None, None, ws, need.value, None, ctypes.byref(out), None) == tcmis.MIS_EINVAL
    assert L.mis_autotune(ctypes.byref(csr), 0, None, None, ws, need.value, None, None, None) == tcmis.MIS_EINVAL
    assert L.mis_autotune(ctypes.byref(csr), 0, None, None, ws, need.value - 1, None, ctypes.byref(out),
                          None) == tcmis.MIS_EINVAL
    assert "workspace" in L.mis_last_error().decode()
    assert L.mis_autotune(ctypes.byref(csr), 0, None, None, ctypes.c_void_p((1 << 20) + 8), need.value, None,
                          ctypes.byref(out), None) == tcmis.MIS_EINVAL
    o = tcmis.MisBuildOpts()
    L.mis_default_opts(ctypes.byref(o))
    o.blocks_per_cu = 33
    assert L.mis_autotune(ctypes.byref(csr), 0, None, ctypes.byref(o), ws, 1 << 40, None, ctypes.byref(out),
                          None) == tcmis.MIS_EINVAL
    assert "blocks_per_cu" in L.mis_last_error().decode()
    L.mis_autotune_clear()
