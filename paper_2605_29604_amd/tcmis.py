"""Thin ctypes binding of libtcmis.so (the C ABI in include/tcmis.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  PyTorch supplies device memory and the stream.  If the library is not
built, every entry point raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtcmis.so")

MIS_OK, MIS_EINVAL, MIS_ENOTSYM, MIS_ESELFLOOP, MIS_EDUP, MIS_ERANGE = 0, -1, -2, -3, -4, -5
MIS_ENOMEM, MIS_EBUSY, MIS_EHIP, MIS_EINTERNAL = -6, -7, -8, -9
PATH_AUTO, PATH_TILE, PATH_CSR, PATH_HYBRID = 0, 1, 2, 3
REORDER_AUTO, REORDER_NONE, REORDER_DEGREE, REORDER_KEY, REORDER_RCM = 0, 1, 2, 3, 4

PATHS = {"auto": PATH_AUTO, "tile": PATH_TILE, "csr": PATH_CSR, "hybrid": PATH_HYBRID}
LAUNCHES = {"auto": 0, "direct": 1, "graph": 2, "persistent": 3}
KEY_RULES = {"degree": 0, "hash": 1, "eq1": 2}
REORDERS = {"auto": REORDER_AUTO, "none": REORDER_NONE, "degree": REORDER_DEGREE,
            "key": REORDER_KEY, "rcm": REORDER_RCM}

# symbols declared in include/tcmis.h
EXPORTS = ["mis_default_opts", "mis_build_bytes", "mis_build_tiles", "mis_build_batch_bytes", "mis_build_batch",
           "mis_graph_bytes", "mis_solve", "mis_solve_scratch_bytes", "mis_solve_union", "mis_solve_batch",
           "mis_solve_batch_scratch_bytes", "mis_free_tiles", "mis_status_string", "mis_last_error",
           "mis_version", "mis_autotune_bytes", "mis_autotune", "mis_autotune_clear", "mis_session_create",
           "mis_session_admit", "mis_session_progress", "mis_session_step", "mis_session_poll", "mis_session_query",
           "mis_session_destroy",
           "mis_release_host_buffers", "mis_build_times", "mis_solve_noalloc", "mis_noalloc_max_bytes",
           "mis_update_edges"]


class MisCsr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p)]


class MisBuildOpts(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("tile", ctypes.c_int32), ("reorder", ctypes.c_int32),
                ("orient", ctypes.c_int32), ("validate", ctypes.c_int32), ("poll_rounds", ctypes.c_int32),
                ("launch", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("dense_min", ctypes.c_int32), ("key_rule", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("dyn_slack", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("keys", ctypes.c_void_p)]


class MisStats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("path", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("reorder", ctypes.c_int32), ("orient", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("n_in", ctypes.c_int64), ("tiles", ctypes.c_int64), ("tile_bytes", ctypes.c_int64),
                ("alg_bytes", ctypes.c_int64), ("units", ctypes.c_int64 * 8),
                ("kernel_ms", ctypes.c_float * 3), ("launches", ctypes.c_int32),
                ("trace_cap", ctypes.c_int32), ("graph", ctypes.c_int32), ("pad3_", ctypes.c_int32),
                ("trace", ctypes.POINTER(ctypes.c_int64))]


class MisSessionConfig(ctypes.Structure):
    _fields_ = [("arena", ctypes.c_void_p), ("arena_bytes", ctypes.c_size_t), ("max_live", ctypes.c_int32),
                ("rounds_per_step", ctypes.c_int32), ("opts", MisBuildOpts)]


class MisDone(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("rounds", ctypes.c_int32),
                ("n", ctypes.c_int64), ("n_in", ctypes.c_int64), ("admit_s", ctypes.c_double),
                ("done_s", ctypes.c_double)]


class MisError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_lib = None


def lib():
    """Loads libtcmis.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                           "or python paper_2605_29604_amd/build_lib.py")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    L.mis_default_opts.argtypes = [ctypes.POINTER(MisBuildOpts)]
    L.mis_default_opts.restype = None
    L.mis_build_bytes.argtypes = [ctypes.POINTER(MisCsr), ctypes.POINTER(MisBuildOpts),
                                  ctypes.POINTER(ctypes.c_size_t)]
    L.mis_build_bytes.restype = ctypes.c_int
    L.mis_build_tiles.argtypes = [ctypes.POINTER(MisCsr), ctypes.POINTER(MisBuildOpts), vp, ctypes.c_size_t,
                                  vp, ctypes.POINTER(vp)]
    L.mis_build_tiles.restype = ctypes.c_int
    L.mis_graph_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.mis_graph_bytes.restype = ctypes.c_int
    L.mis_solve.argtypes = [vp, vp, i32, vp, ctypes.c_size_t, ctypes.POINTER(MisStats), vp]
    L.mis_solve.restype = ctypes.c_int
    L.mis_solve_scratch_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_size_t)]
    L.mis_solve_scratch_bytes.restype = ctypes.c_int
    L.mis_build_batch_bytes.argtypes = [ctypes.POINTER(MisCsr), i32, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(MisBuildOpts), ctypes.POINTER(ctypes.c_size_t)]
    L.mis_build_batch_bytes.restype = ctypes.c_int
    L.mis_build_batch.argtypes = [ctypes.POINTER(MisCsr), i32, ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(MisBuildOpts), vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.mis_build_batch.restype = ctypes.c_int
    L.mis_solve_union.argtypes = [vp, vp, ctypes.POINTER(MisStats), ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_int64), vp]
    L.mis_solve_union.restype = ctypes.c_int
    L.mis_solve_batch_scratch_bytes.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(ctypes.c_size_t)]
    L.mis_solve_batch_scratch_bytes.restype = ctypes.c_int
    L.mis_solve_batch.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(vp), vp, ctypes.c_size_t,
                                  ctypes.POINTER(MisStats), ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_int64), vp]
    L.mis_solve_batch.restype = ctypes.c_int
    L.mis_autotune_bytes.argtypes = [ctypes.POINTER(MisCsr), i32, ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(MisBuildOpts), ctypes.POINTER(ctypes.c_size_t)]
    L.mis_autotune_bytes.restype = ctypes.c_int
    L.mis_autotune.argtypes = [ctypes.POINTER(MisCsr), i32, ctypes.POINTER(ctypes.c_int64),
                               ctypes.POINTER(MisBuildOpts), vp, ctypes.c_size_t, vp, ctypes.POINTER(MisBuildOpts),
                               ctypes.POINTER(ctypes.c_int32)]
    L.mis_autotune.restype = ctypes.c_int
    L.mis_autotune_clear.argtypes = []
    L.mis_autotune_clear.restype = None
    L.mis_session_create.argtypes = [ctypes.POINTER(MisSessionConfig), ctypes.POINTER(vp)]
    L.mis_session_create.restype = ctypes.c_int
    L.mis_session_admit.argtypes = [vp, ctypes.POINTER(MisCsr), i32, ctypes.POINTER(MisBuildOpts), vp, vp,
                                    ctypes.c_uint64]
    L.mis_session_admit.restype = ctypes.c_int
    L.mis_session_progress.argtypes = [vp, i32, ctypes.POINTER(MisDone), i32, ctypes.POINTER(ctypes.c_int32)]
    L.mis_session_progress.restype = ctypes.c_int
    L.mis_session_step.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.mis_session_step.restype = ctypes.c_int
    L.mis_session_poll.argtypes = [vp, i32, ctypes.POINTER(MisDone), i32, ctypes.POINTER(ctypes.c_int32)]
    L.mis_session_poll.restype = ctypes.c_int
    L.mis_session_query.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_size_t),
                                    ctypes.POINTER(ctypes.c_size_t)]
    L.mis_session_query.restype = ctypes.c_int
    L.mis_session_destroy.argtypes = [vp]
    L.mis_session_destroy.restype = None
    L.mis_free_tiles.argtypes = [vp]
    L.mis_free_tiles.restype = None
    L.mis_build_times.argtypes = [vp, ctypes.POINTER(ctypes.c_float), i32, ctypes.POINTER(ctypes.c_int32)]
    L.mis_build_times.restype = ctypes.c_int
    L.mis_solve_noalloc.argtypes = [ctypes.POINTER(MisCsr), ctypes.POINTER(MisBuildOpts), vp,
                                    ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64), vp]
    L.mis_solve_noalloc.restype = ctypes.c_int
    L.mis_noalloc_max_bytes.argtypes = []
    L.mis_noalloc_max_bytes.restype = ctypes.c_size_t
    L.mis_update_edges.argtypes = [vp, vp, vp, ctypes.c_int64, vp, ctypes.POINTER(MisStats), vp]
    L.mis_update_edges.restype = ctypes.c_int
    L.mis_release_host_buffers.argtypes = []
    L.mis_release_host_buffers.restype = None
    L.mis_status_string.argtypes = [ctypes.c_int]
    L.mis_status_string.restype = ctypes.c_char_p
    L.mis_last_error.argtypes = []
    L.mis_last_error.restype = ctypes.c_char_p
    L.mis_version.argtypes = []
    L.mis_version.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(rc: int):
    if rc != MIS_OK:
        L = lib()
        raise MisError(rc, f"{L.mis_status_string(rc).decode()}: {L.mis_last_error().decode()}")


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


@dataclass
class MisGraph:
    """A built handle; keeps the device CSR tensors alive (the CSR path reads them)."""
    handle: ctypes.c_void_p
    n: int
    nnz: int
    keepalive: tuple = field(default_factory=tuple)
    count: int = 0

    def bytes(self) -> int:
        b = ctypes.c_size_t(0)
        _check(lib().mis_graph_bytes(self.handle, ctypes.byref(b)))
        return int(b.value)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            _lib.mis_free_tiles(h)
            self.handle = None


def _opts(path="auto", tile=0, reorder="auto", orient=-1, validate=False, seed=1, keys=None, poll_rounds=0,
          launch="auto", blocks_per_cu=0, dense_min=0, key_rule="degree", timing=False, dyn_slack=0):
    o = MisBuildOpts()
    lib().mis_default_opts(ctypes.byref(o))
    o.path = PATHS[path] if isinstance(path, str) else int(path)
    o.tile = int(tile)
    o.reorder = REORDERS[reorder] if isinstance(reorder, str) else int(reorder)
    o.orient = int(orient)
    o.validate = int(bool(validate))
    o.poll_rounds = int(poll_rounds)
    o.launch = LAUNCHES[launch] if isinstance(launch, str) else int(launch)
    o.blocks_per_cu = int(blocks_per_cu)
    o.dense_min = int(dense_min)
    o.key_rule = KEY_RULES[key_rule] if isinstance(key_rule, str) else int(key_rule)
    o.timing = int(bool(timing))
    o.dyn_slack = int(dyn_slack)
    o.seed = int(seed) & (2**64 - 1)
    o.keys = _ptr(keys)
    return o


def mis_build_bytes(n: int, nnz: int, **opts) -> int:
    """Workspace bytes mis_build_tiles needs (host-only arithmetic)."""
    csr = MisCsr(n, nnz, ctypes.c_void_p(256), ctypes.c_void_p(256) if nnz else None)
    o = _opts(**opts)
    b = ctypes.c_size_t(0)
    _check(lib().mis_build_bytes(ctypes.byref(csr), ctypes.byref(o), ctypes.byref(b)))
    return int(b.value)


def mis_build_tiles(row_ptr, col_idx, path="auto", tile=0, reorder="auto", orient=-1, validate=False,
                    seed=1, keys=None, poll_rounds=0, launch="auto", blocks_per_cu=0, workspace=None,
                    stream=None, dense_min=0, key_rule="degree", timing=False, dyn_slack=0) -> MisGraph:
    """row_ptr: cuda int64[n+1]; col_idx: cuda int32[nnz]; keys: optional cuda uint64[n] (as int64).

    The device workspace comes from torch's allocator unless one is passed (a cuda
    uint8 tensor of at least mis_build_bytes bytes); the handle keeps it alive.
    """
    import torch
    L = lib()
    n = row_ptr.numel() - 1
    nnz = col_idx.numel()
    csr = MisCsr(n, nnz, _ptr(row_ptr), _ptr(col_idx) if nnz else None)
    o = _opts(path, tile, reorder, orient, validate, seed, keys, poll_rounds, launch, blocks_per_cu, dense_min,
              key_rule, timing, dyn_slack)
    need = ctypes.c_size_t(0)
    _check(L.mis_build_bytes(ctypes.byref(csr), ctypes.byref(o), ctypes.byref(need)))
    if workspace is None:
        workspace = torch.empty(int(need.value), dtype=torch.uint8, device=row_ptr.device)
    h = ctypes.c_void_p(None)
    _check(L.mis_build_tiles(ctypes.byref(csr), ctypes.byref(o), _ptr(workspace), workspace.numel(),
                             ctypes.c_void_p(_stream(stream)), ctypes.byref(h)))
    return MisGraph(h, n, nnz, (row_ptr, col_idx, keys, workspace))


def _stats_dict(st: MisStats, trace_buf) -> dict:
    rounds = st.rounds
    d = {
        "rounds": rounds, "path": st.path, "tile": st.tile, "reorder": st.reorder, "orient": st.orient,
        "n_in": st.n_in, "tiles": st.tiles, "tile_bytes": st.tile_bytes, "alg_bytes": st.alg_bytes,
        "units": list(st.units), "kernel_ms": list(st.kernel_ms), "launches": st.launches, "graph": st.graph,
    }
    if trace_buf is not None:
        k = min(rounds, st.trace_cap)
        d["trace"] = trace_buf[: 3 * k].reshape(k, 3).copy()
    return d


def _new_stats(trace_cap: int, timing: bool):
    st = MisStats()
    st.timing = int(bool(timing))
    buf = None
    if trace_cap > 0:
        buf = np.zeros(3 * trace_cap, dtype=np.int64)
        st.trace_cap = trace_cap
        st.trace = buf.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    return st, buf


def mis_solve_scratch_bytes(g: MisGraph) -> int:
    b = ctypes.c_size_t(0)
    _check(lib().mis_solve_scratch_bytes(g.handle, ctypes.byref(b)))
    return int(b.value)


def mis_solve(g: MisGraph, out=None, max_rounds=0, trace_cap=4096, timing=False, stream=None, scratch=None):
    """Returns (in_set cuda uint8[n], stats dict).  scratch: a cuda uint8 tensor of at
    least mis_solve_scratch_bytes(g) bytes for this solve's round state (None: the
    handle's own)."""
    import torch
    if out is None:
        out = torch.empty(max(g.n, 0), dtype=torch.uint8, device="cuda")
    st, buf = _new_stats(trace_cap, timing)
    sp, sb = (None, 0) if scratch is None else (_ptr(scratch), scratch.numel() * scratch.element_size())
    _check(lib().mis_solve(g.handle, _ptr(out) if g.n else None, int(max_rounds), sp, sb, ctypes.byref(st),
                           ctypes.c_void_p(_stream(stream))))
    return out, _stats_dict(st, buf)


def _offsets(offsets):
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    return off, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def mis_build_batch_bytes(n: int, nnz: int, offsets, **opts) -> int:
    csr = MisCsr(n, nnz, ctypes.c_void_p(256), ctypes.c_void_p(256) if nnz else None)
    off, offp = _offsets(offsets)
    o = _opts(**opts)
    b = ctypes.c_size_t(0)
    _check(lib().mis_build_batch_bytes(ctypes.byref(csr), len(off) - 1, offp, ctypes.byref(o), ctypes.byref(b)))
    return int(b.value)


def mis_build_batch(row_ptr, col_idx, offsets, path="auto", tile=0, reorder="auto", orient=-1, validate=False,
                    seed=1, keys=None, poll_rounds=0, launch="auto", blocks_per_cu=0, workspace=None,
                    stream=None, dense_min=0, key_rule="degree", timing=False, dyn_slack=0) -> MisGraph:
    """A batch of independent graphs given as their disjoint union (cuda CSR) and host
    vertex offsets (count+1).  Priorities use graph-local ids."""
    import torch
    L = lib()
    n = row_ptr.numel() - 1
    nnz = col_idx.numel()
    csr = MisCsr(n, nnz, _ptr(row_ptr), _ptr(col_idx) if nnz else None)
    off, offp = _offsets(offsets)
    o = _opts(path, tile, reorder, orient, validate, seed, keys, poll_rounds, launch, blocks_per_cu, dense_min,
              key_rule, timing, dyn_slack)
    need = ctypes.c_size_t(0)
    _check(L.mis_build_batch_bytes(ctypes.byref(csr), len(off) - 1, offp, ctypes.byref(o), ctypes.byref(need)))
    if workspace is None:
        workspace = torch.empty(int(need.value), dtype=torch.uint8, device=row_ptr.device)
    h = ctypes.c_void_p(None)
    _check(L.mis_build_batch(ctypes.byref(csr), len(off) - 1, offp, ctypes.byref(o), _ptr(workspace),
                             workspace.numel(), ctypes.c_void_p(_stream(stream)), ctypes.byref(h)))
    g = MisGraph(h, n, nnz, (row_ptr, col_idx, keys, workspace))
    g.count = len(off) - 1
    return g


def mis_solve_union(g: MisGraph, out=None, trace_cap=4096, stream=None):
    """Solves a handle built by mis_build_batch.  Returns (in_set cuda uint8[n] of the
    union, batch stats, per-graph rounds int32[count], per-graph set sizes int64[count])."""
    import torch
    if out is None:
        out = torch.empty(max(g.n, 0), dtype=torch.uint8, device="cuda")
    st, buf = _new_stats(trace_cap, False)
    rounds = np.zeros(max(g.count, 1), dtype=np.int32)
    sizes = np.zeros(max(g.count, 1), dtype=np.int64)
    _check(lib().mis_solve_union(g.handle, _ptr(out) if g.n else None, ctypes.byref(st),
                                 rounds.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                 sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                 ctypes.c_void_p(_stream(stream))))
    return out, _stats_dict(st, buf), rounds[: g.count], sizes[: g.count]


def _handle_array(graphs):
    arr = (ctypes.c_void_p * max(1, len(graphs)))()
    for i, g in enumerate(graphs):
        arr[i] = g.handle.value if isinstance(g.handle, ctypes.c_void_p) else g.handle
    return arr


def mis_solve_batch_scratch_bytes(graphs) -> int:
    b = ctypes.c_size_t(0)
    _check(lib().mis_solve_batch_scratch_bytes(_handle_array(graphs), len(graphs), ctypes.byref(b)))
    return int(b.value)


def mis_solve_batch(graphs, outs=None, scratch=None, stream=None):
    """Solves independently built single-graph hybrid handles together (one launch per
    round kernel over all of them).  Returns (list of cuda uint8 outputs, batch stats,
    per-graph rounds int32[count], per-graph set sizes int64[count])."""
    import torch
    graphs = list(graphs)
    if outs is None:
        outs = [torch.empty(max(g.n, 1), dtype=torch.uint8, device="cuda") for g in graphs]
    if scratch is None:
        scratch = torch.empty(max(1, mis_solve_batch_scratch_bytes(graphs)), dtype=torch.uint8, device="cuda")
    ptrs = (ctypes.c_void_p * max(1, len(graphs)))()
    for i, o in enumerate(outs):
        ptrs[i] = o.data_ptr()
    st, buf = _new_stats(0, False)
    rounds = np.zeros(max(len(graphs), 1), dtype=np.int32)
    sizes = np.zeros(max(len(graphs), 1), dtype=np.int64)
    _check(lib().mis_solve_batch(_handle_array(graphs), len(graphs), ptrs, _ptr(scratch), scratch.numel(),
                                 ctypes.byref(st), rounds.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                 sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                 ctypes.c_void_p(_stream(stream))))
    return outs, _stats_dict(st, buf), rounds[: len(graphs)], sizes[: len(graphs)]


_PATH_NAMES = {v: k for k, v in PATHS.items()}
_REORDER_NAMES = {v: k for k, v in REORDERS.items()}


def mis_autotune(row_ptr, col_idx, offsets=None, path="auto", tile=0, blocks_per_cu=0, seed=1, keys=None,
                 poll_rounds=0, launch="auto", workspace=None, stream=None, dense_min=0, key_rule="degree"):
    """Tuned build options for this graph (or batch, with host offsets) as a dict of
    mis_build_tiles / mis_build_batch keyword arguments, plus whether the profile
    bucket was already cached: (opts, from_cache)."""
    import torch
    L = lib()
    n = row_ptr.numel() - 1
    nnz = col_idx.numel()
    csr = MisCsr(n, nnz, _ptr(row_ptr), _ptr(col_idx) if nnz else None)
    count, offp = 0, None
    if offsets is not None:
        off, offp = _offsets(offsets)
        count = len(off) - 1
    o = _opts(path, tile, "auto", -1, False, seed, keys, poll_rounds, launch, blocks_per_cu, dense_min, key_rule)
    need = ctypes.c_size_t(0)
    _check(L.mis_autotune_bytes(ctypes.byref(csr), count, offp, ctypes.byref(o), ctypes.byref(need)))
    if workspace is None:
        workspace = torch.empty(int(need.value), dtype=torch.uint8, device=row_ptr.device)
    res = MisBuildOpts()
    cached = ctypes.c_int32(0)
    _check(L.mis_autotune(ctypes.byref(csr), count, offp, ctypes.byref(o), _ptr(workspace), workspace.numel(),
                          ctypes.c_void_p(_stream(stream)), ctypes.byref(res), ctypes.byref(cached)))
    opts = dict(path=_PATH_NAMES[res.path], tile=res.tile, reorder=_REORDER_NAMES[res.reorder],
                orient=res.orient, blocks_per_cu=res.blocks_per_cu, dense_min=res.dense_min, seed=seed,
                keys=keys, poll_rounds=poll_rounds, launch=launch, key_rule=key_rule)
    return opts, bool(cached.value)


def mis_autotune_clear():
    lib().mis_autotune_clear()


def mis_build_times(g: MisGraph) -> list:
    """Build-stage durations in ms of a handle built with timing=True (see the header)."""
    buf = (ctypes.c_float * 16)()
    cnt = ctypes.c_int32(0)
    _check(lib().mis_build_times(g.handle, buf, 16, ctypes.byref(cnt)))
    return [float(buf[i]) for i in range(min(cnt.value, 16))]


def mis_solve_noalloc(row_ptr, col_idx, out, stream=None, **opts):
    """Build + solve with no allocation (the library's per-GPU array); out: cuda uint8[n].
    Returns (rounds, set size)."""
    n = row_ptr.numel() - 1
    nnz = col_idx.numel()
    csr = MisCsr(n, nnz, _ptr(row_ptr), _ptr(col_idx) if nnz else None)
    o = _opts(**opts)
    r = ctypes.c_int32(0)
    k = ctypes.c_int64(0)
    _check(lib().mis_solve_noalloc(ctypes.byref(csr), ctypes.byref(o), _ptr(out) if n else None, ctypes.byref(r),
                                   ctypes.byref(k), ctypes.c_void_p(_stream(stream))))
    return int(r.value), int(k.value)


def mis_update_edges(g: MisGraph, edges, ops, in_set, stream=None) -> dict:
    """Edge edits on a dynamic handle and the repair of in_set (cuda uint8[n], updated in
    place).  edges: cuda int32[count, 2]; ops: cuda int8[count] (1 insert, 0 delete)."""
    st = MisStats()
    k = int(ops.numel())
    _check(lib().mis_update_edges(g.handle, _ptr(edges) if k else None, _ptr(ops) if k else None, k,
                                  _ptr(in_set) if g.n else None, ctypes.byref(st), ctypes.c_void_p(_stream(stream))))
    return {"rounds": st.rounds, "n_in": st.n_in, "entries_read": st.units[0]}


def mis_release_host_buffers() -> None:
    """Frees the idle pinned staging buffers of the round-loop polls."""
    lib().mis_release_host_buffers()


def mis_free_tiles(g: MisGraph):
    if g.handle:
        lib().mis_free_tiles(g.handle)
        g.handle = None


class Session:
    """Serving session over a device arena (a torch uint8 tensor it allocates or is given).

    admit() takes a request's CSR as HOST numpy / pinned torch arrays (copied to the
    arena by the library) or cuda tensors, and returns False when the session is busy
    (no slot or arena region free).  progress() returns the retired requests as dicts.
    The session keeps every request's host/device arrays alive until it retires.
    """

    def __init__(self, arena_bytes=None, max_live=8, rounds_per_step=4, arena=None, path="auto", tile=0,
                 reorder="auto", orient=-1, seed=1, launch="direct", blocks_per_cu=0):
        import torch
        if arena is None:
            arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device="cuda")
        self.arena = arena
        cfg = MisSessionConfig()
        cfg.arena = _ptr(arena)
        cfg.arena_bytes = arena.numel()
        cfg.max_live = int(max_live)
        cfg.rounds_per_step = int(rounds_per_step)
        cfg.opts = _opts(path, tile, reorder, orient, False, seed, None, 0, launch, blocks_per_cu)
        h = ctypes.c_void_p(None)
        _check(lib().mis_session_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h
        self.cap = int(max_live)
        self._keep = {}
        self._buf = (MisDone * self.cap)()

    def admit(self, row_ptr, col_idx, tag, out=None, host_out=None, opts=None) -> bool:
        """row_ptr/col_idx: both host (numpy or torch cpu, pinned preferred) or both cuda.
        out: cuda uint8[n] or None; host_out: host uint8[n] (numpy / torch cpu) or None."""
        import torch
        on_host = not (isinstance(row_ptr, torch.Tensor) and row_ptr.is_cuda)
        n = (row_ptr.numel() if isinstance(row_ptr, torch.Tensor) else row_ptr.size) - 1
        nnz = col_idx.numel() if isinstance(col_idx, torch.Tensor) else col_idx.size
        csr = MisCsr(n, nnz, _host_or_dev_ptr(row_ptr), _host_or_dev_ptr(col_idx) if nnz else None)
        o = None if opts is None else ctypes.byref(_opts(**opts))
        rc = lib().mis_session_admit(self.handle, ctypes.byref(csr), int(on_host), o,
                                     _host_or_dev_ptr(out) if out is not None else None,
                                     _host_or_dev_ptr(host_out) if host_out is not None else None,
                                     ctypes.c_uint64(int(tag)))
        if rc == MIS_EBUSY:
            return False
        _check(rc)
        self._keep[int(tag)] = (row_ptr, col_idx, out, host_out, opts)
        return True

    def step(self) -> int:
        """Enqueues the next rounds (or the output) of every request whose last batch
        drained; returns how many advanced."""
        adv = ctypes.c_int32(0)
        _check(lib().mis_session_step(self.handle, ctypes.byref(adv)))
        return adv.value

    def poll(self, wait=False):
        """Retires requests whose output landed (enqueues nothing)."""
        nd = ctypes.c_int32(0)
        _check(lib().mis_session_poll(self.handle, int(bool(wait)), self._buf, self.cap, ctypes.byref(nd)))
        return self._retired(nd.value)

    def progress(self, wait=False):
        nd = ctypes.c_int32(0)
        _check(lib().mis_session_progress(self.handle, int(bool(wait)), self._buf, self.cap, ctypes.byref(nd)))
        return self._retired(nd.value)

    def _retired(self, count):
        nd = ctypes.c_int32(count)
        res = []
        for i in range(nd.value):
            d = self._buf[i]
            res.append(dict(tag=int(d.tag), status=d.status, rounds=d.rounds, n=d.n, n_in=d.n_in,
                            admit_s=d.admit_s, done_s=d.done_s))
            self._keep.pop(int(d.tag), None)
        return res

    def query(self):
        live = ctypes.c_int32(0)
        used = ctypes.c_size_t(0)
        big = ctypes.c_size_t(0)
        _check(lib().mis_session_query(self.handle, ctypes.byref(live), ctypes.byref(used), ctypes.byref(big)))
        return live.value, used.value, big.value

    def close(self):
        if self.handle:
            lib().mis_session_destroy(self.handle)
            self.handle = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _host_or_dev_ptr(a):
    import torch
    if isinstance(a, torch.Tensor):
        return ctypes.c_void_p(a.data_ptr())
    return ctypes.c_void_p(a.ctypes.data)


def version() -> str:
    return lib().mis_version().decode()
