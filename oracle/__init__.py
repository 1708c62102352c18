"""CPU oracle for round-synchronous priority MIS -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline``
leg may import this package.  The GPU library never calls it, and the two share
no code; they share only the seeded input generators
(``paper_2605_29604_amd.gen``), which hold none of the method's arithmetic.

All arithmetic lives in ``mis_oracle.c`` (plain C, compiled with gcc into
``libmis_oracle.so`` next to this file); ``brute.py`` holds the brute-force
enumerator used to pin it on tiny graphs.  See the header of ``mis_oracle.c`` for
the passages of the paper each function follows and for the readings taken
where the paper is silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mis_oracle.c")
_LIB = os.path.join(_HERE, "libmis_oracle.so")
_lib = None

UNDECIDED, IN, OUT = 0, 1, 2


def build_lib() -> str:
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
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
    i64, u64, p, i32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int
    lib.orc_splitmix_stream.argtypes = [u64, i64, p]
    lib.orc_splitmix_stream.restype = None
    lib.orc_q.argtypes = [i64]
    lib.orc_q.restype = u64
    lib.orc_key.argtypes = [u64, i64, i64]
    lib.orc_key.restype = u64
    lib.orc_keys.argtypes = [i64, p, u64, p]
    lib.orc_keys.restype = i32
    lib.orc_keys_rule.argtypes = [i64, p, u64, i32, p]
    lib.orc_keys_rule.restype = i32
    lib.orc_validate.argtypes = [i64, p, p]
    lib.orc_validate.restype = i32
    lib.orc_roundsync.argtypes = [i64, p, p, p, i64, p, p, i64]
    lib.orc_roundsync.restype = i64
    lib.orc_greedy.argtypes = [i64, p, p, p, p]
    lib.orc_greedy.restype = i64
    lib.orc_verify.argtypes = [i64, p, p, p]
    lib.orc_verify.restype = i32
    lib.orc_lfmis_cert.argtypes = [i64, p, p, p, p]
    lib.orc_lfmis_cert.restype = i64
    lib.orc_mindeg_greedy.argtypes = [i64, p, p, p]
    lib.orc_mindeg_greedy.restype = i64
    _lib = lib
    return lib


def _csr(row_ptr, col_idx):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    if ci.size == 0:
        ci = np.zeros(1, dtype=np.int32)
    return rp, ci


def splitmix64(seed: int, count: int) -> np.ndarray:
    out = np.zeros(count, dtype=np.uint64)
    _load().orc_splitmix_stream(seed & (2**64 - 1), count, out.ctypes.data)
    return out


def q(deg: int) -> int:
    return int(_load().orc_q(deg))


def key(seed: int, v: int, deg: int) -> int:
    return int(_load().orc_key(seed & (2**64 - 1), v, deg))


def keys(row_ptr, seed: int) -> np.ndarray:
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    n = rp.size - 1
    out = np.zeros(max(n, 1), dtype=np.uint64)
    if _load().orc_keys(n, rp.ctypes.data, seed & (2**64 - 1), out.ctypes.data) != 0:
        raise ValueError("default key rule needs n <= 2^24")
    return out[:n]


KEY_RULES = {"degree": 0, "hash": 1, "eq1": 2}


def keys_rule(row_ptr, seed: int, rule: str) -> np.ndarray:
    """Keys of one graph under a priority heuristic of Section 3.3 (see orc_keys_rule)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    n = rp.size - 1
    out = np.zeros(max(n, 1), dtype=np.uint64)
    rc = _load().orc_keys_rule(n, rp.ctypes.data, seed & (2**64 - 1), KEY_RULES[rule], out.ctypes.data)
    if rc != 0:
        raise ValueError("key rule needs n <= 2^24 and a known rule")
    return out[:n]


def validate(row_ptr, col_idx) -> int:
    rp, ci = _csr(row_ptr, col_idx)
    return int(_load().orc_validate(rp.size - 1, rp.ctypes.data, ci.ctypes.data))


def roundsync(row_ptr, col_idx, key_arr, max_rounds: int = 0):
    """Round-synchronous MIS (Algorithm 2, fixed priorities).

    Returns (status uint8[n], rounds, trace int64[rounds, 3]) where trace rows are
    (|C_r|, vertices removed as neighbours of candidates, |A| after round r).
    """
    rp, ci = _csr(row_ptr, col_idx)
    n = rp.size - 1
    k = np.ascontiguousarray(key_arr, dtype=np.uint64)
    if k.size == 0:
        k = np.zeros(1, dtype=np.uint64)
    status = np.zeros(max(n, 1), dtype=np.uint8)
    cap = max(n, 1) + 1
    trace = np.zeros(3 * cap, dtype=np.int64)
    r = int(_load().orc_roundsync(n, rp.ctypes.data, ci.ctypes.data, k.ctypes.data, max_rounds,
                                  status.ctypes.data, trace.ctypes.data, cap))
    if r < 0:
        raise MemoryError("oracle allocation failed")
    return status[:n], r, trace[: 3 * r].reshape(r, 3)


def mis(row_ptr, col_idx, key_arr) -> np.ndarray:
    """in/out vector (uint8, 1 = in the set) of the round-synchronous solve."""
    status, _, _ = roundsync(row_ptr, col_idx, key_arr)
    return (status == IN).astype(np.uint8)


def greedy(row_ptr, col_idx, key_arr) -> np.ndarray:
    rp, ci = _csr(row_ptr, col_idx)
    n = rp.size - 1
    k = np.ascontiguousarray(key_arr, dtype=np.uint64)
    if k.size == 0:
        k = np.zeros(1, dtype=np.uint64)
    out = np.zeros(max(n, 1), dtype=np.uint8)
    if _load().orc_greedy(n, rp.ctypes.data, ci.ctypes.data, k.ctypes.data, out.ctypes.data) < 0:
        raise MemoryError
    return out[:n]


def verify(row_ptr, col_idx, in_set) -> int:
    """0 = maximal independent set, 1 = not independent, 2 = not maximal."""
    rp, ci = _csr(row_ptr, col_idx)
    s = np.ascontiguousarray(in_set, dtype=np.uint8)
    if s.size == 0:
        s = np.zeros(1, dtype=np.uint8)
    return int(_load().orc_verify(rp.size - 1, rp.ctypes.data, ci.ctypes.data, s.ctypes.data))


def lfmis_cert(row_ptr, col_idx, key_arr, in_set) -> int:
    """0 if in(v) <=> (no higher-key neighbour is in) for all v, else 1 + first bad v."""
    rp, ci = _csr(row_ptr, col_idx)
    k = np.ascontiguousarray(key_arr, dtype=np.uint64)
    s = np.ascontiguousarray(in_set, dtype=np.uint8)
    if k.size == 0:
        k, s = np.zeros(1, np.uint64), np.zeros(1, np.uint8)
    return int(_load().orc_lfmis_cert(rp.size - 1, rp.ctypes.data, ci.ctypes.data,
                                      k.ctypes.data, s.ctypes.data))


def mindeg_greedy(row_ptr, col_idx) -> np.ndarray:
    rp, ci = _csr(row_ptr, col_idx)
    n = rp.size - 1
    out = np.zeros(max(n, 1), dtype=np.uint8)
    if _load().orc_mindeg_greedy(n, rp.ctypes.data, ci.ctypes.data, out.ctypes.data) < 0:
        raise MemoryError
    return out[:n]
