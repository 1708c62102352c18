"""Host logic of the serving session: the arena allocator (compiled with g++ from its
header, no GPU) and the session's argument checks."""
import ctypes
import os
import subprocess

import pytest

from conftest import ROOT
from paper_2605_29604_amd import tcmis


def test_arena_allocator(tmp_path):
    exe = str(tmp_path / "arena_check")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-Wall", "-Werror", "-o", exe,
                           os.path.join(ROOT, "tests", "host", "arena_check.cpp")])
    out = subprocess.check_output([exe], timeout=120).decode()
    assert out.startswith("ok"), out


@pytest.fixture(scope="module")
def L():
    return tcmis.lib()


def test_session_argument_errors(L):
    h = ctypes.c_void_p(None)
    cfg = tcmis.MisSessionConfig()
    L.mis_default_opts(ctypes.byref(cfg.opts))
    cfg.arena, cfg.arena_bytes, cfg.max_live, cfg.rounds_per_step = 1 << 20, 1 << 30, 4, 0
    assert L.mis_session_create(None, ctypes.byref(h)) == tcmis.MIS_EINVAL
    assert L.mis_session_create(ctypes.byref(cfg), None) == tcmis.MIS_EINVAL
    for field, value in (("arena", (1 << 20) + 16), ("arena", None), ("arena_bytes", 100), ("max_live", 0),
                         ("max_live", 257), ("rounds_per_step", -1), ("rounds_per_step", 1025)):
        bad = tcmis.MisSessionConfig()
        ctypes.pointer(bad)[0] = cfg
        setattr(bad, field, value)
        assert L.mis_session_create(ctypes.byref(bad), ctypes.byref(h)) == tcmis.MIS_EINVAL, field
        assert not h.value
    # persistent (cooperative) launches cannot run as concurrent requests: refused on the host
    bad = tcmis.MisSessionConfig()
    ctypes.pointer(bad)[0] = cfg
    bad.opts.launch = tcmis.LAUNCHES["persistent"]
    assert L.mis_session_create(ctypes.byref(bad), ctypes.byref(h)) == tcmis.MIS_EINVAL
    assert not h.value
    csr = tcmis.MisCsr(10, 0, ctypes.c_void_p(256), None)
    assert L.mis_session_admit(None, ctypes.byref(csr), 0, None, ctypes.c_void_p(256), None, 1) == tcmis.MIS_EINVAL
    n = ctypes.c_int32(0)
    assert L.mis_session_progress(None, 0, None, 0, ctypes.byref(n)) == tcmis.MIS_EINVAL
    assert L.mis_session_query(None, None, None, None) == tcmis.MIS_EINVAL
    L.mis_session_destroy(None)
    assert L.mis_status_string(tcmis.MIS_EBUSY).decode().startswith("busy")
