import json
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: full-size workloads (seconds of CPU each)")


def golden(name):
    path = os.path.join(GOLDEN, name)
    if name.endswith(".json"):
        with open(path) as f:
            return json.load(f)
    with open(path) as f:
        return [line.strip() for line in f if line.strip() and not line.startswith("#")]


def csr_from_edges(n, edges):
    """Symmetric CSR (rows sorted) from an undirected edge list."""
    adj = [[] for _ in range(n)]
    for u, v in edges:
        adj[u].append(v)
        adj[v].append(u)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    for v in range(n):
        row_ptr[v + 1] = row_ptr[v] + len(adj[v])
    col_idx = np.array([u for v in range(n) for u in sorted(adj[v])], dtype=np.int32)
    return row_ptr, col_idx


def random_graph(n, p, rng):
    edges = [(u, v) for u in range(n) for v in range(u + 1, n) if rng.random() < p]
    return edges


def distinct_keys(n, rng):
    """Distinct random 64-bit keys (as uint64)."""
    ks = set()
    while len(ks) < n:
        ks.add(int(rng.integers(0, 2**63 - 1)) * 2 + int(rng.integers(0, 2)))
    arr = np.array(sorted(ks), dtype=np.uint64)
    rng.shuffle(arr)
    return arr
