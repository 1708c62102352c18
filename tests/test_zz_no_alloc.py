"""The entry point that allocates nothing (mis_solve_noalloc, through the C ABI)
against the existing build + solve entry points on the same input and options, on
two calls in a row (the second graph smaller than the first, so the per-GPU array
holds the first call's contents), and against the oracle."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2605_29604_amd import gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CONFIGS = [dict(path="hybrid", dense_min=9), dict(path="hybrid", dense_min=1), dict(path="csr"),
           dict(path="tile", tile=16, reorder="key"), dict(path="tile", tile=32, reorder="none", orient=0)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def T():
    from paper_2605_29604_amd import tcmis
    return tcmis


def solve_with_handle(rp, ci, **opts):
    t = T()
    h = t.mis_build_tiles(rp, ci, **opts)
    out, st = t.mis_solve(h)
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    t.mis_free_tiles(h)
    return res, st["rounds"], st["n_in"]


@pytest.mark.parametrize("cfg", CONFIGS, ids=lambda c: "-".join(f"{k}={v}" for k, v in c.items()))
def test_noalloc_equals_build_and_solve(cfg):
    t = T()
    graphs = [gen.rmat(1 << 14, 8 << 14, seed=3), gen.er(3001, 12000, seed=5)]   # second call smaller
    for i, g in enumerate(graphs):
        print(f"case noalloc {cfg} graph {i} n={g.n}", flush=True)
        rp = torch.from_numpy(g.row_ptr).cuda()
        ci = torch.from_numpy(g.col_idx).cuda()
        assert t.mis_build_bytes(g.n, g.nnz, **cfg) <= t.lib().mis_noalloc_max_bytes()
        out = torch.full((g.n,), 9, dtype=torch.uint8, device="cuda")
        rounds, n_in = t.mis_solve_noalloc(rp, ci, out, seed=7, **cfg)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        ref, ref_rounds, ref_in = solve_with_handle(rp, ci, seed=7, **cfg)
        assert np.array_equal(got, ref) and rounds == ref_rounds and n_in == ref_in
        st, r, _ = oracle.roundsync(g.row_ptr, g.col_idx, oracle.keys(g.row_ptr, 7))
        assert np.array_equal(got, (st == oracle.IN).astype(np.uint8)) and rounds == r


def test_noalloc_refuses_what_it_cannot_hold():
    t = T()
    L = t.lib()
    cap = L.mis_noalloc_max_bytes()
    assert cap == 64 << 20
    # a structure beyond the array: refused on the host before any device work
    # (the pointers are never dereferenced)
    n, nnz = 1 << 22, 1 << 25
    csr = t.MisCsr(n, nnz, ctypes.c_void_p(256), ctypes.c_void_p(256))
    o = t._opts(path="hybrid")
    assert t.mis_build_bytes(n, nnz, path="hybrid") > cap
    rc = L.mis_solve_noalloc(ctypes.byref(csr), ctypes.byref(o), ctypes.c_void_p(256), None, None, None)
    assert rc == t.MIS_EINVAL and b"no-allocation" in L.mis_last_error()
    for bad in (dict(path="tile", reorder="rcm"), dict(path="csr", launch="graph"), dict(timing=True)):
        g = gen.er(100, 300, 1)
        rp = torch.from_numpy(g.row_ptr).cuda()
        ci = torch.from_numpy(g.col_idx).cuda()
        out = torch.empty(g.n, dtype=torch.uint8, device="cuda")
        with pytest.raises(t.MisError) as ei:
            t.mis_solve_noalloc(rp, ci, out, **bad)
        assert ei.value.code == t.MIS_EINVAL
