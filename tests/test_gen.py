"""Input generators: determinism, simple-graph properties, closed forms."""
import os
import subprocess
import sys

import numpy as np
import pytest

from conftest import ROOT, golden
from paper_2605_29604_amd import gen


def check_simple(g):
    n, rp, ci = g.n, g.row_ptr, g.col_idx
    assert rp[0] == 0 and rp[-1] == ci.size
    assert np.all(np.diff(rp) >= 0)
    assert ci.min(initial=0) >= 0 and ci.max(initial=-1) < n
    rows = np.repeat(np.arange(n), np.diff(rp))
    assert not np.any(rows == ci), "self-loop"
    # sorted rows, strictly increasing -> no duplicates
    same_row = rows[1:] == rows[:-1]
    assert np.all(ci[1:][same_row] > ci[:-1][same_row])
    # symmetric: the multiset of (row, col) equals that of (col, row)
    a = rows.astype(np.int64) * n + ci
    b = ci.astype(np.int64) * n + rows
    assert np.array_equal(np.sort(a), np.sort(b))


def test_splitmix_vector():
    want = [int(x) for x in golden("splitmix64_seed1234567.txt")]
    assert [int(x) for x in gen.splitmix64(1234567, 5)] == want


@pytest.mark.parametrize("maker", [
    lambda s: gen.er(2000, 9000, s),
    lambda s: gen.rmat(1 << 12, 8 << 12, s),
    lambda s: gen.rmat(3000, 20000, s),            # non power of two
    lambda s: gen.grid(9, 7, 5, 0.01, s),
])
def test_simple_and_deterministic(maker):
    g1, g2, g3 = maker(7), maker(7), maker(8)
    check_simple(g1)
    assert np.array_equal(g1.row_ptr, g2.row_ptr) and np.array_equal(g1.col_idx, g2.col_idx)
    assert not np.array_equal(g1.col_idx, g3.col_idx)


def test_exact_edge_counts():
    assert gen.er(10_000, 40_000).m == 40_000
    g = gen.rmat(1 << 14, 8 << 14)
    assert g.m == 8 << 14 and g.nnz == 16 << 14
    assert gen.grid_edges(256, 256, 256) == 50_135_040
    g = gen.grid(20, 20, 20, 0.01)
    assert g.m == gen.grid_edges(20, 20, 20) + int(0.01 * gen.grid_edges(20, 20, 20))


def test_grid_closed_form():
    s = 10
    g = gen.grid(s, s, s, 0.0)
    assert g.m == 3 * s * s * (s - 1)
    d = g.degrees()
    # corners 3, edges 4, faces 5, interior 6
    assert (d == 3).sum() == 8
    assert (d == 4).sum() == 12 * (s - 2)
    assert (d == 5).sum() == 6 * (s - 2) ** 2
    assert (d == 6).sum() == (s - 2) ** 3
    # v = x + s*y + s*s*z: x-neighbour of vertex 0 is 1, y-neighbour is s, z-neighbour s*s
    assert list(g.col_idx[g.row_ptr[0]:g.row_ptr[1]]) == [1, s, s * s]


def test_long_range_not_grid_edges():
    s = 12
    base = gen.grid(s, s, s, 0.0)
    g = gen.grid(s, s, s, 0.05)
    check_simple(g)
    extra = g.m - base.m
    assert extra == int(0.05 * base.m)
    # every grid edge is still present exactly once
    for v in range(0, s ** 3, 37):
        a = set(base.col_idx[base.row_ptr[v]:base.row_ptr[v + 1]])
        b = set(g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]])
        assert a <= b


def test_rmat_skew():
    g = gen.rmat(1 << 14, 8 << 14)
    d = np.sort(g.degrees())[::-1]
    # power-law-like: the top 1% of vertices carry a large share of the endpoints
    assert d[: len(d) // 100].sum() > 0.2 * d.sum()


def test_thread_count_independent():
    code = ("import hashlib;from paper_2605_29604_amd import gen;"
            "g=gen.rmat(1<<13, 8<<13, 3);print(hashlib.md5(g.col_idx.tobytes()).hexdigest())")
    outs = set()
    for t in ("1", "3"):
        env = dict(os.environ, GG_THREADS=t)
        outs.add(subprocess.check_output([sys.executable, "-c", code], cwd=ROOT, env=env).strip())
    assert len(outs) == 1


def test_batch_spec():
    sp = gen.batch_spec(4096, 1)
    assert sp == gen.batch_spec(4096, 1) and sp != gen.batch_spec(4096, 2)
    ns = np.array([s[1] for s in sp])
    assert ns.min() >= 500 and ns.max() <= 200_000
    # log-uniform: the median is near the geometric mean of the range
    assert 6_000 < np.median(ns) < 14_000
    kinds = [s[0] for s in sp]
    assert kinds[::2] == ["er"] * 2048 and kinds[1::2] == ["rmat"] * 2048
    for kind, n, m, _ in sp[:200]:
        d = 2 * m / n
        assert (3.9 <= d <= 32.1) if kind == "er" else (7.9 <= d <= 24.1)


def test_union():
    gs = [gen.er(30, 60, 1), gen.er(0, 0, 1), gen.rmat(50, 120, 2), gen.er(1, 0, 3)]
    rp, ci, off = gen.union(gs)
    assert list(off) == [0, 30, 30, 80, 81]
    u = gen.Graph(int(off[-1]), rp, ci)
    check_simple(u)
    for i, g in enumerate(gs):
        o = int(off[i])
        for v in range(g.n):
            a = ci[rp[o + v]:rp[o + v + 1]] - o
            assert np.array_equal(a, g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]])


def test_serve_spec_and_grid_requests():
    sp = gen.serve_spec(600, 1)
    assert sp == gen.serve_spec(600, 1)
    kinds = [s[0] for s in sp]
    assert all(150 < kinds.count(k) < 250 for k in ("er", "rmat", "grid"))
    for kind, n, m, sd in sp:
        assert 900 <= n <= 4_100_000
        if kind == "grid":
            side = round(n ** (1 / 3))
            assert side ** 3 == n and m == gen.grid_edges(side, side, side) * 101 // 100
    g = gen.make("grid", 8 ** 3, gen.grid_edges(8, 8, 8) + 3, 5)
    check_simple(g)
    assert g.m == gen.grid_edges(8, 8, 8) + 3


def test_batch_union_equals_union_of_makes():
    spec = gen.batch_spec(40, seed=3, n_min=50, n_max=20000) + gen.serve_spec(12, seed=4, n_min=100, n_max=40000)
    spec.insert(5, ("er", 0, 0, 9))
    spec.insert(9, ("er", 1, 0, 9))
    # small threshold: the large graphs go through the one-at-a-time multithreaded pass
    rp, ci, off = gen.batch_union(spec, big_edges=20000)
    rp2, ci2, off2 = gen.union([gen.make(*s) for s in spec])
    assert np.array_equal(off, off2) and np.array_equal(rp, rp2) and np.array_equal(ci, ci2)
