"""Brute-force enumeration of all maximal independent sets (n <= 20) -- test only.

Every subset S of V (a bitmask) is tested against the definition of an MIS
(Introduction: no two members adjacent, and no vertex can be added): for every
vertex v, v in S implies S ∩ N(v) = ∅, and v not in S implies S ∩ N(v) ≠ ∅.
The enumerator is itself pinned by textbook counts (Padovan numbers for paths,
Perrin numbers for cycles, Moon-Moser 3^(n/3) for disjoint triangles).
"""
from __future__ import annotations

import numpy as np

MAX_N = 20


def neighbour_masks(n: int, edges) -> np.ndarray:
    nb = np.zeros(n, dtype=np.int64)
    for u, v in edges:
        nb[u] |= 1 << v
        nb[v] |= 1 << u
    return nb


def all_mis(n: int, edges) -> np.ndarray:
    """All maximal independent sets of the graph, as sorted int64 bitmasks."""
    if n > MAX_N:
        raise ValueError("brute force is limited to 20 vertices")
    nb = neighbour_masks(n, edges)
    subsets = np.arange(1 << n, dtype=np.int64)
    ok = np.ones(subsets.size, dtype=bool)
    for v in range(n):
        member = (subsets >> v) & 1 == 1
        touches = (subsets & nb[v]) != 0
        ok &= np.where(member, ~touches, touches)
    return subsets[ok]


def edges_from_csr(row_ptr, col_idx):
    out = []
    for v in range(len(row_ptr) - 1):
        for e in range(row_ptr[v], row_ptr[v + 1]):
            u = int(col_idx[e])
            if v < u:
                out.append((v, u))
    return out


def to_indicator(mask: int, n: int) -> np.ndarray:
    return np.array([(mask >> v) & 1 for v in range(n)], dtype=np.uint8)


def lex_greatest_in_key_order(masks, key_arr) -> int:
    """The mask whose indicator, read in decreasing key order, is lexicographically greatest."""
    # keys are distinct 64-bit integers: sort exactly with Python ints
    order = sorted(range(len(key_arr)), key=lambda v: -int(key_arr[v]))
    best, best_tuple = None, None
    for m in masks:
        t = tuple(((int(m) >> v) & 1) for v in order)
        if best_tuple is None or t > best_tuple:
            best, best_tuple = int(m), t
    return best
