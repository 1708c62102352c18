"""Seeded synthetic graph inputs (CSR) for the MIS solver and its oracle.

This module is the only code that the CPU oracle and the GPU library share: it
makes inputs and holds none of the solver's arithmetic.  All generation runs in
``graphgen.c`` (host C, compiled to ``libgraphgen.so`` next to this file).

The workloads stand in for the paper's SuiteSparse evaluation graphs (Table 1:
mesh/road graphs, power-law web and social graphs, a Graph500 Kronecker graph),
which are not available here; no item of that collection is reproduced.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build_lib() -> str:
    """Compile graphgen.c with gcc into libgraphgen.so (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
                           "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build_lib()
    lib = ctypes.CDLL(_LIB)
    i64, u64, i32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int
    p = ctypes.c_void_p
    lib.gg_er.argtypes = [i64, i64, u64, p, p]
    lib.gg_er.restype = i64
    lib.gg_rmat.argtypes = [i64, i64, u64, u64, u64, i32, u64, p, p]
    lib.gg_rmat.restype = i64
    lib.gg_grid.argtypes = [i64, i64, i64, i64, u64, p, p]
    lib.gg_grid.restype = i64
    lib.gg_grid_edges.argtypes = [i64, i64, i64]
    lib.gg_grid_edges.restype = i64
    lib.gg_union.argtypes = [i64, p, p, p, p, u64, u64, u64, p, p, i64, p, p]
    lib.gg_union.restype = i64
    lib.gg_splitmix64.argtypes = [u64, i64, p]
    lib.gg_splitmix64.restype = None
    _lib = lib
    return lib


@dataclass
class Graph:
    """Undirected simple graph in CSR form; every edge appears in both rows."""
    n: int
    row_ptr: np.ndarray  # int64[n+1]
    col_idx: np.ndarray  # int32[nnz], each row sorted ascending
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def m(self) -> int:
        """Undirected edges, each counted once."""
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)


def _alloc(n: int, m: int):
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    col_idx = np.zeros(max(2 * m, 1), dtype=np.int32)
    return row_ptr, col_idx


def _check(rc: int, what: str) -> int:
    if rc < 0:
        raise RuntimeError(f"{what}: generator error {rc}")
    return rc


def splitmix64(seed: int, count: int) -> np.ndarray:
    out = np.zeros(count, dtype=np.uint64)
    _load().gg_splitmix64(seed & (2**64 - 1), count, out.ctypes.data)
    return out


def er(n: int, m: int, seed: int = 1) -> Graph:
    """Erdos-Renyi G(n, m): m distinct uniform pairs u != v (redraw duplicates)."""
    row_ptr, col_idx = _alloc(n, m)
    _check(_load().gg_er(n, m, seed, row_ptr.ctypes.data, col_idx.ctypes.data), "er")
    return Graph(n, row_ptr, col_idx[: 2 * m], f"er_n{n}_m{m}_s{seed}")


RMAT_ABC = (0.57, 0.19, 0.19)


def rmat(n: int, m: int, seed: int = 1, abc=RMAT_ABC, permute: bool = True) -> Graph:
    """R-MAT with quadrant probabilities abc (d = rest), m distinct non-loop edges."""
    a32, b32, c32 = (int(math.floor(x * 2**32)) for x in abc)
    row_ptr, col_idx = _alloc(n, m)
    _check(_load().gg_rmat(n, m, a32, b32, c32, int(permute), seed,
                           row_ptr.ctypes.data, col_idx.ctypes.data), "rmat")
    return Graph(n, row_ptr, col_idx[: 2 * m], f"rmat_n{n}_m{m}_s{seed}")


def grid_edges(sx: int, sy: int, sz: int) -> int:
    return int(_load().gg_grid_edges(sx, sy, sz))


def grid(sx: int, sy: int, sz: int, long_frac: float = 0.01, seed: int = 1) -> Graph:
    """3D 7-point mesh plus round-down(long_frac * grid edges) random long-range pairs."""
    mg = grid_edges(sx, sy, sz)
    n_long = int(math.floor(long_frac * mg))
    n = sx * sy * sz
    row_ptr, col_idx = _alloc(n, mg + n_long)
    m = _check(_load().gg_grid(sx, sy, sz, n_long, seed, row_ptr.ctypes.data,
                               col_idx.ctypes.data), "grid")
    return Graph(n, row_ptr, col_idx[: 2 * m], f"grid_{sx}x{sy}x{sz}_l{n_long}_s{seed}")


# ---- named workloads (the five synthetic configurations) ----

def workload(name: str, seed: int = 1) -> Graph:
    """Named synthetic workloads.

    er10k   : G(n=10,000, m=40,000), average degree exactly 8.
    rmat22  : R-MAT scale 22 (n=4,194,304), m=8n distinct edges (avg degree 16),
              a,b,c,d = .57,.19,.19,.05, random vertex relabelling.
    grid256 : 256^3 7-point mesh (50,135,040 edges) + 1% = 501,350 long-range pairs.
    Smaller variants for tests: rmat<k> (scale k, avg degree 16), grid<s> (s^3 mesh).
    """
    if name == "er10k":
        return er(10_000, 40_000, seed)
    if name.startswith("rmat"):
        scale = int(name[4:])
        n = 1 << scale
        return rmat(n, 8 * n, seed)
    if name.startswith("grid"):
        s = int(name[4:])
        return grid(s, s, s, 0.01, seed)
    raise KeyError(name)


# ---- batches of independent graphs ----

def batch_spec(count: int, seed: int = 1, n_min: int = 500, n_max: int = 200_000):
    """Per-graph recipe of a batch: graph g draws from the SplitMix64 stream seeded with
    seed_g = first output of the stream seeded with (seed XOR g).  Even g: Erdos-Renyi
    with an integer average degree uniform in [4, 32]; odd g: R-MAT with an integer
    average degree uniform in [8, 24]; n_g = round(exp(U[ln n_min, ln n_max]));
    m_g = round(n_g * d_g / 2) (capped to what the graph can hold)."""
    out = []
    for g in range(count):
        sg = int(splitmix64(seed ^ g, 1)[0])
        d = splitmix64(sg, 3)
        u1 = (int(d[0]) >> 11) / float(1 << 53)
        n = int(round(math.exp(math.log(n_min) + u1 * (math.log(n_max) - math.log(n_min)))))
        if g % 2 == 0:
            kind, deg = "er", 4 + int(((int(d[1]) >> 32) * 29) >> 32)
        else:
            kind, deg = "rmat", 8 + int(((int(d[1]) >> 32) * 17) >> 32)
        m = min(int(round(n * deg / 2)), n * (n - 1) // 4)
        out.append((kind, n, m, sg))
    return out


def serve_spec(count: int, seed: int = 1, n_min: int = 1000, n_max: int = 4_000_000):
    """Request mix of the serving workload: like batch_spec, but the kind is uniform
    over Erdos-Renyi, R-MAT and 3D grid (draw 2 of the graph's stream, multiply-shift
    to [0, 3)); a grid request has side round(n^(1/3)), n = side^3 and 1% long-range
    pairs, so its tuple is ("grid", side^3, grid edges + long-range pairs, seed)."""
    out = []
    for g in range(count):
        sg = int(splitmix64(seed ^ (g + 0x5E4E), 1)[0])
        d = splitmix64(sg, 3)
        u1 = (int(d[0]) >> 11) / float(1 << 53)
        n = int(round(math.exp(math.log(n_min) + u1 * (math.log(n_max) - math.log(n_min)))))
        kind = ("er", "rmat", "grid")[((int(d[2]) >> 32) * 3) >> 32]
        if kind == "grid":
            side = max(2, int(round(n ** (1.0 / 3.0))))
            mg = grid_edges(side, side, side)
            out.append(("grid", side ** 3, mg + int(math.floor(0.01 * mg)), sg))
            continue
        if kind == "er":
            deg = 4 + int(((int(d[1]) >> 32) * 29) >> 32)
        else:
            deg = 8 + int(((int(d[1]) >> 32) * 17) >> 32)
        out.append((kind, n, min(int(round(n * deg / 2)), n * (n - 1) // 4), sg))
    return out


def _cube_side(n: int) -> int:
    side = int(round(n ** (1.0 / 3.0)))
    while side ** 3 < n:
        side += 1
    while side ** 3 > n:
        side -= 1
    if side ** 3 != n:
        raise ValueError(f"grid request size {n} is not a cube")
    return side


def make(kind: str, n: int, m: int, seed: int) -> Graph:
    """One graph of a batch or serving spec tuple (kind, n, m, seed)."""
    if kind == "er":
        return er(n, m, seed)
    if kind == "rmat":
        return rmat(n, m, seed)
    side = _cube_side(n)
    row_ptr, col_idx = _alloc(n, m)
    _check(_load().gg_grid(side, side, side, m - grid_edges(side, side, side), seed, row_ptr.ctypes.data,
                           col_idx.ctypes.data), "grid")
    return Graph(n, row_ptr, col_idx[: 2 * m], f"grid_{side}^3_m{m}_s{seed}")


def batch_union(spec, big_edges: int = 1 << 22):
    """Disjoint union of the graphs of a spec, generated in parallel across graphs;
    identical to union([make(*s) for s in spec]).  Returns (row_ptr, col_idx, offsets)."""
    count = len(spec)
    kinds = np.array([{"er": 1, "rmat": 2, "grid": 3}[s[0]] for s in spec], dtype=np.int32)
    a = np.array([s[1] if s[0] != "grid" else _cube_side(s[1]) for s in spec], dtype=np.int64)
    b = np.array([s[2] if s[0] != "grid" else s[2] - grid_edges(*(3 * [_cube_side(s[1])])) for s in spec],
                 dtype=np.int64)
    seeds = np.array([s[3] for s in spec], dtype=np.uint64)
    voff = np.zeros(count + 1, dtype=np.int64)
    eoff = np.zeros(count + 1, dtype=np.int64)
    voff[1:] = np.cumsum([s[1] for s in spec])
    eoff[1:] = np.cumsum([2 * s[2] for s in spec])
    row_ptr = np.zeros(int(voff[-1]) + 1, dtype=np.int64)
    col_idx = np.zeros(max(int(eoff[-1]), 1), dtype=np.int32)
    a32, b32, c32 = (int(math.floor(x * 2**32)) for x in RMAT_ABC)
    _check(_load().gg_union(count, kinds.ctypes.data, a.ctypes.data, b.ctypes.data, seeds.ctypes.data,
                            a32, b32, c32, voff.ctypes.data, eoff.ctypes.data, big_edges,
                            row_ptr.ctypes.data, col_idx.ctypes.data), "batch")
    return row_ptr, col_idx[: int(eoff[-1])], voff


def union(graphs):
    """Disjoint union of graphs: (row_ptr int64, col_idx int32, offsets int64[count+1])."""
    offsets = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        offsets[i + 1] = offsets[i] + g.n
    nnz = sum(g.nnz for g in graphs)
    row_ptr = np.zeros(int(offsets[-1]) + 1, dtype=np.int64)
    col_idx = np.zeros(nnz, dtype=np.int32)
    e = 0
    for i, g in enumerate(graphs):
        o = int(offsets[i])
        row_ptr[o + 1: o + g.n + 1] = g.row_ptr[1:] + e
        col_idx[e: e + g.nnz] = g.col_idx + o
        e += g.nnz
    return row_ptr, col_idx, offsets
