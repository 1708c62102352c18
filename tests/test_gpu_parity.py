"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit-exact.

Every case compares the whole in/out vector and the per-round trace (|C_r|,
vertices removed as neighbours of candidates, alive after r) with the oracle's
round-synchronous solve on the same seeded input.  Integer work: the bar is
bit-exact equality.
"""
import numpy as np
import pytest

import oracle
from conftest import csr_from_edges
from paper_2605_29604_amd import gen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# (path, tile, reorder, orient[, dense_min]); the hybrid path's dense_min: -1 = entry
# lists only, 1 = every block that fits 64 tiles is dense (bit tiles on the matrix
# cores wherever possible), 9 = the byte break-even of a bit tile against entry indices
HYBRID_CONFIGS = [("hybrid", 16, "none", 1, d) for d in (-1, 1, 9)]
ALL_CONFIGS = [("csr", 0, "none", 0)] + [
    ("tile", t, r, o) for t in (16, 32) for r in ("none", "degree", "key", "rcm") for o in (0, 1)
] + HYBRID_CONFIGS
FAST_CONFIGS = [("csr", 0, "none", 0), ("tile", 16, "key", 1), ("tile", 16, "none", 0),
                ("tile", 32, "degree", 1), ("tile", 32, "rcm", 0)] + HYBRID_CONFIGS


def kw(cfg):
    """Build keyword arguments of a config tuple."""
    d = dict(path=cfg[0], tile=cfg[1], reorder=cfg[2], orient=cfg[3])
    if len(cfg) > 4:
        d["dense_min"] = cfg[4]
    return d


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_29604_amd import tcmis
    tcmis.lib()


def tcmis_mod():
    from paper_2605_29604_amd import tcmis
    return tcmis


def to_dev(rp, ci):
    return (torch.from_numpy(np.ascontiguousarray(rp, dtype=np.int64)).cuda(),
            torch.from_numpy(np.ascontiguousarray(ci, dtype=np.int32)).cuda())


def expected(rp, ci, keys, max_rounds=0):
    st, r, tr = oracle.roundsync(rp, ci, keys, max_rounds=max_rounds)
    return (st == oracle.IN).astype(np.uint8), r, tr


def run(rp, ci, cfg, seed=1, keys=None, max_rounds=0, validate=True, poll_rounds=0, key_rule="degree"):
    T = tcmis_mod()
    drp, dci = to_dev(rp, ci)
    dkeys = None if keys is None else torch.from_numpy(keys.view(np.int64)).cuda()
    h = T.mis_build_tiles(drp, dci, seed=seed, keys=dkeys, validate=validate, poll_rounds=poll_rounds,
                          key_rule=key_rule, **kw(cfg))
    out, st = T.mis_solve(h, max_rounds=max_rounds)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    T.mis_free_tiles(h)
    return got, st


def check(rp, ci, cfg, seed=1, keys=None, label="", key_rule="degree"):
    k = oracle.keys_rule(rp, seed, key_rule) if keys is None else keys
    want, rounds, trace = expected(rp, ci, k)
    got, st = run(rp, ci, cfg, seed=seed, keys=keys, key_rule=key_rule)
    print(f"case {label} cfg={cfg} n={len(rp) - 1} rounds={rounds}", flush=True)
    assert np.array_equal(got, want), f"{label} {cfg}: {int((got != want).sum())} vertices differ"
    assert st["rounds"] == rounds, f"{label} {cfg}: rounds {st['rounds']} != {rounds}"
    assert np.array_equal(st["trace"], trace), f"{label} {cfg}: trace differs"
    assert st["n_in"] == int(want.sum())


@pytest.mark.parametrize("cfg", ALL_CONFIGS, ids=lambda c: "-".join(map(str, c)))
def test_er10k_all_configs(cfg):
    g = gen.workload("er10k", seed=1)
    check(g.row_ptr, g.col_idx, cfg, seed=1, label="er10k")


@pytest.mark.parametrize("cfg", ALL_CONFIGS, ids=lambda c: "-".join(map(str, c)))
def test_rmat14_all_configs(cfg):
    g = gen.rmat(1 << 14, 8 << 14, seed=3)
    check(g.row_ptr, g.col_idx, cfg, seed=5, label="rmat14")


@pytest.mark.parametrize("cfg", FAST_CONFIGS, ids=lambda c: "-".join(map(str, c)))
@pytest.mark.parametrize("name", ["rmat16", "grid24", "grid40"])
def test_workloads(name, cfg):
    g = gen.workload(name, seed=2)
    check(g.row_ptr, g.col_idx, cfg, seed=7, label=name)


@pytest.mark.parametrize("cfg", FAST_CONFIGS, ids=lambda c: "-".join(map(str, c)))
@pytest.mark.parametrize("n", [1, 2, 15, 17, 31, 33, 1000 + 7])
def test_ragged_sizes(n, cfg):
    m = min(n * (n - 1) // 2, 4 * n)
    g = gen.er(n, m, seed=n)
    check(g.row_ptr, g.col_idx, cfg, seed=3, label=f"er{n}")


@pytest.mark.parametrize("cfg", FAST_CONFIGS, ids=lambda c: "-".join(map(str, c)))
def test_edge_cases(cfg):
    # edgeless graph: everyone joins in round 1
    rp = np.zeros(41, dtype=np.int64)
    check(rp, np.zeros(0, np.int32), cfg, label="edgeless")
    # complete graph: only the top key
    n = 33
    rp, ci = csr_from_edges(n, [(u, v) for u in range(n) for v in range(u + 1, n)])
    check(rp, ci, cfg, label="K33")
    # star with a hub whose row-block spans several work segments
    s = 20000
    rp, ci = csr_from_edges(s + 1, [(0, i) for i in range(1, s + 1)])
    check(rp, ci, cfg, label="star20000")
    # perfect matching
    rp, ci = csr_from_edges(64, [(2 * i, 2 * i + 1) for i in range(32)])
    check(rp, ci, cfg, label="matching")


def heavy_tail_graph(seed):
    """Hubs of degree 33 .. 300 (rows longer than a lane's 32 entries), ordinary
    vertices of degree 1 .. 40, isolated vertices, and last vertices whose rows end the
    adjacency array (fewer than 32 entries after their starts)."""
    rng = np.random.default_rng(seed)
    n = 3000
    edges = set()
    for h in range(12):                      # hubs 0 .. 11
        for v in rng.choice(np.arange(12, n - 200), size=33 + 24 * h, replace=False):
            edges.add((h, int(v)))
    for v in range(12, n - 200):             # ordinary rows; every 7th vertex stays isolated
        if v % 7 == 0:
            continue
        for w in rng.choice(np.arange(12, n - 200), size=int(rng.integers(1, 6)), replace=False):
            if int(w) != v and int(w) % 7:
                edges.add((min(v, int(w)), max(v, int(w))))
    for t in range(1, 6):                    # the last rows of the array
        for w in rng.choice(np.arange(0, n - 6), size=3 * t, replace=False):
            if int(w) % 7 or int(w) < 12:
                edges.add((int(w), n - t))
    return csr_from_edges(n, sorted(edges))


@pytest.mark.parametrize("cfg", HYBRID_CONFIGS + [("csr", 0, "none", 0)], ids=lambda c: "-".join(map(str, c)))
@pytest.mark.parametrize("keys", ["degree", "random", "hubs_first"])
def test_round1_heavy_and_last_rows(cfg, keys):
    # round 1 takes a row's first 32 entries on its lane and longer rows with the whole
    # wave; rows among the array's last 32 entries take the wave path from their start;
    # caller keys go through the key-gather variant of the round-1 kernels
    rp, ci = heavy_tail_graph(11)
    n = len(rp) - 1
    rng = np.random.default_rng(5)
    k = None
    if keys == "random":
        k = np.array(rng.permutation(n) + 1, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15 >> 16)
    elif keys == "hubs_first":   # hubs out-rank everything: candidates after scanning whole long rows
        k = np.array(rng.permutation(n) + 1, dtype=np.uint64)
        k[:12] = np.uint64(1 << 40) + np.arange(12, dtype=np.uint64)
    check(rp, ci, cfg, keys=k, label=f"heavy_tail_{keys}")


@pytest.mark.parametrize("cfg", FAST_CONFIGS, ids=lambda c: "-".join(map(str, c)))
def test_deep_path_custom_keys(cfg):
    # keys increase along a path: ceil(n/2) rounds, two decisions per round
    n = 301
    rp, ci = csr_from_edges(n, [(i, i + 1) for i in range(n - 1)])
    keys = np.arange(1, n + 1, dtype=np.uint64) * np.uint64(0x9E3779B97F4A7C15 >> 8)
    check(rp, ci, cfg, keys=keys, label="path301")


@pytest.mark.parametrize("cfg", FAST_CONFIGS, ids=lambda c: "-".join(map(str, c)))
def test_entry_windows(cfg):
    # the entry pass stages a workgroup's rows in LDS when they fit (2048 rows per
    # 4096 entries) and looks them up in global memory otherwise: degree-2 rows put
    # the row span on either side of that bound, degree-1 and isolated rows far above
    for n in (6001, 6145, 8193):
        rp, ci = csr_from_edges(n, [(i, i + 1) for i in range(n - 1)])
        check(rp, ci, cfg, label=f"path{n}")
    m = 3000   # caterpillar: a path with one leaf on every vertex
    rp, ci = csr_from_edges(2 * m, [(i, i + 1) for i in range(m - 1)] + [(i, m + i) for i in range(m)])
    check(rp, ci, cfg, label="caterpillar3000")
    c = 5000   # a cycle on the even vertices, every odd vertex isolated
    rp, ci = csr_from_edges(2 * c, [(2 * i, 2 * ((i + 1) % c)) for i in range(c)])
    check(rp, ci, cfg, label="cycle5000-isolated")
    # the hybrid orientation stages 512 rows per 2048 entries: a 2D mesh (degree 4
    # inside, 2-3 on the rim) puts its windows on both sides of that bound
    s = 70
    rp, ci = csr_from_edges(s * s, [(y * s + x, y * s + x + 1) for y in range(s) for x in range(s - 1)] +
                            [(y * s + x, (y + 1) * s + x) for y in range(s - 1) for x in range(s)])
    check(rp, ci, cfg, label="mesh70x70")


@pytest.mark.parametrize("tile", [16, 32])
def test_default_keys_given_by_caller(tile):
    # the default keys passed in explicitly: the order sort then carries vertex ids
    # as a payload over all 64 key bits instead of reading them from the keys
    g = gen.rmat(1 << 14, 8 << 14, seed=4)
    keys = oracle.keys(g.row_ptr, 9)
    check(g.row_ptr, g.col_idx, ("tile", tile, "key", 1), seed=9, keys=keys, label="rmat14-keys")
    check(g.row_ptr, g.col_idx, ("tile", tile, "key", 1), seed=9, label="rmat14-default")
    # the hybrid path then compares gathered keys instead of degree classes and hashes
    for d in (-1, 1):
        check(g.row_ptr, g.col_idx, ("hybrid", 16, "none", 1, d), seed=9, keys=keys, label="rmat14-keys-hybrid")


@pytest.mark.parametrize("rule", ["hash", "eq1"])
@pytest.mark.parametrize("cfg", FAST_CONFIGS, ids=lambda c: "-".join(map(str, c)))
def test_key_rules(rule, cfg):
    # the priority heuristics of Section 3.3 computed on the device (H1: hash only;
    # Eq. 1 discretised) give the oracle's set and trace under the same rule
    for name in ("rmat14", "grid24"):
        g = gen.workload(name, seed=2)
        check(g.row_ptr, g.col_idx, cfg, seed=13, label=f"{name}-{rule}", key_rule=rule)


def test_one_degree_class_key_order():
    # every vertex of a cycle has degree 2, so all keys share their degree class: the
    # order sort's ties on the class and 22 hash bits come in runs averaging two,
    # thousands of them eight or longer (the path that sorts a run in memory)
    n = 1 << 23
    rp = np.arange(0, 2 * n + 1, 2, dtype=np.int64)
    nb = np.stack([(np.arange(n) - 1) % n, (np.arange(n) + 1) % n], axis=1)
    ci = np.sort(nb, axis=1).astype(np.int32).ravel()
    check(rp, ci, ("tile", 16, "key", 1), seed=5, label="cycle2^23")


def test_empty_graph():
    T = tcmis_mod()
    drp = torch.zeros(1, dtype=torch.int64, device="cuda")
    dci = torch.zeros(0, dtype=torch.int32, device="cuda")
    for path in ("csr", "tile", "hybrid"):
        h = T.mis_build_tiles(drp, dci, path=path, validate=True)
        out, st = T.mis_solve(h)
        assert out.numel() == 0 and st["rounds"] == 0
        T.mis_free_tiles(h)


@pytest.mark.parametrize("cfg", FAST_CONFIGS, ids=lambda c: "-".join(map(str, c)))
def test_round_limit(cfg):
    g = gen.workload("grid24", seed=1)
    k = oracle.keys(g.row_ptr, 1)
    _, full_rounds, _ = expected(g.row_ptr, g.col_idx, k)
    for j in range(1, full_rounds + 1):
        want, r, tr = expected(g.row_ptr, g.col_idx, k, max_rounds=j)
        got, st = run(g.row_ptr, g.col_idx, cfg, seed=1, max_rounds=j, poll_rounds=3)
        assert st["rounds"] == j and np.array_equal(st["trace"], tr)
        assert np.array_equal(got, want)


def test_repeat_and_poll_interval_deterministic():
    T = tcmis_mod()
    g = gen.workload("rmat16", seed=4)
    k = oracle.keys(g.row_ptr, 9)
    want, rounds, trace = expected(g.row_ptr, g.col_idx, k)
    drp, dci = to_dev(g.row_ptr, g.col_idx)
    for cfg in FAST_CONFIGS:
        for poll in (1, 2, 5):
            h = T.mis_build_tiles(drp, dci, **kw(cfg), seed=9,
                                  poll_rounds=poll)
            for _ in range(3):
                out, st = T.mis_solve(h)
                assert np.array_equal(out.cpu().numpy(), want)
                assert np.array_equal(st["trace"], trace)
            T.mis_free_tiles(h)


@pytest.mark.parametrize("cfg", FAST_CONFIGS + [("hybrid", 16, "none", 1, 1)], ids=lambda c: "-".join(map(str, c)))
def test_concurrent_solves_of_one_handle_with_caller_scratch(cfg):
    # one built handle, two solves in flight at once on two streams, each with its
    # own scratch for the round state (the handle is only read); then a third on the
    # handle's own state: all equal the oracle, set and round trace
    import threading
    T = tcmis_mod()
    g = gen.workload("rmat16", seed=6)
    k = oracle.keys(g.row_ptr, 3)
    want, rounds, trace = expected(g.row_ptr, g.col_idx, k)
    drp, dci = to_dev(g.row_ptr, g.col_idx)
    h = T.mis_build_tiles(drp, dci, seed=3, **kw(cfg))
    torch.cuda.synchronize()
    nb = T.mis_solve_scratch_bytes(h)
    assert 0 < nb < h.bytes()
    streams = [torch.cuda.Stream() for _ in range(2)]
    scratch = [torch.empty(nb, dtype=torch.uint8, device="cuda") for _ in range(2)]
    outs = [torch.full((g.n,), 7, dtype=torch.uint8, device="cuda") for _ in range(2)]
    res = [None, None]

    def solve(i):
        with torch.cuda.stream(streams[i]):
            res[i] = T.mis_solve(h, out=outs[i], scratch=scratch[i], stream=streams[i])[1]

    th = [threading.Thread(target=solve, args=(i,)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    torch.cuda.synchronize()
    print(f"case concurrent scratch cfg={cfg} n={g.n} scratch={nb}", flush=True)
    for i in range(2):
        assert np.array_equal(outs[i].cpu().numpy(), want), f"solve {i}"
        assert res[i]["rounds"] == rounds and np.array_equal(res[i]["trace"], trace)
    out, st = T.mis_solve(h)
    assert np.array_equal(out.cpu().numpy(), want) and np.array_equal(st["trace"], trace)
    with pytest.raises(T.MisError) as ei:   # too small
        T.mis_solve(h, scratch=scratch[0][: nb - 256])
    assert ei.value.code == T.MIS_EINVAL
    T.mis_free_tiles(h)


@pytest.mark.parametrize("bad", ["loop", "asym", "dup", "range", "tie"])
def test_validation_errors(bad):
    T = tcmis_mod()
    rp, ci = csr_from_edges(6, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5)])
    keys = None
    want = {"loop": T.MIS_ESELFLOOP, "asym": T.MIS_ENOTSYM, "dup": T.MIS_EDUP, "range": T.MIS_ERANGE,
            "tie": T.MIS_EINVAL}[bad]
    if bad == "loop":
        rp, ci = np.array([0, 1, 2]), np.array([0, 0])      # 0-0 loop; row 1 -> 0
    elif bad == "asym":
        rp, ci = np.array([0, 1, 1]), np.array([1])
    elif bad == "dup":
        rp, ci = np.array([0, 2, 4]), np.array([1, 1, 0, 0])
    elif bad == "range":
        rp, ci = np.array([0, 1, 2]), np.array([1, 7])
    else:
        keys = np.array([5, 5, 1, 2, 3, 4], dtype=np.uint64)
    drp, dci = to_dev(rp, ci)
    dkeys = None if keys is None else torch.from_numpy(keys.view(np.int64)).cuda()
    for path in ("csr", "tile", "hybrid"):
        with pytest.raises(T.MisError) as ei:
            T.mis_build_tiles(drp, dci, path=path, keys=dkeys, validate=True)
        assert ei.value.code == want


@pytest.mark.slow
@pytest.mark.parametrize("cfg", [("csr", 0, "none", 0), ("tile", 16, "key", 1), ("tile", 16, "key", 0),
                                 ("tile", 32, "key", 1), ("hybrid", 16, "none", 1, 9),
                                 ("hybrid", 16, "none", 1, 1)], ids=lambda c: "-".join(map(str, c)))
def test_rmat22_full(cfg):
    g = gen.workload("rmat22", seed=1)
    check(g.row_ptr, g.col_idx, cfg, seed=1, label="rmat22")


@pytest.mark.slow
@pytest.mark.parametrize("cfg", [("csr", 0, "none", 0), ("tile", 16, "none", 1), ("tile", 32, "rcm", 1),
                                 ("tile", 16, "rcm", 0), ("hybrid", 16, "none", 1, 9),
                                 ("hybrid", 16, "none", 1, -1)], ids=lambda c: "-".join(map(str, c)))
def test_grid256_full(cfg):
    g = gen.workload("grid256", seed=1)
    check(g.row_ptr, g.col_idx, cfg, seed=1, label="grid256")


@pytest.mark.parametrize("cfg", FAST_CONFIGS, ids=lambda c: "-".join(map(str, c)))
def test_launch_modes_and_graph_replays(cfg):
    # the captured round loop is replayed many times (several batches per solve and
    # several solves per handle, with host work and synchronisation in between);
    # every replay must give the direct-launch result, which must equal the oracle
    T = tcmis_mod()
    g = gen.workload("grid24", seed=3)
    k = oracle.keys(g.row_ptr, 6)
    want, rounds, trace = expected(g.row_ptr, g.col_idx, k)
    drp, dci = to_dev(g.row_ptr, g.col_idx)
    for launch in ("direct", "graph", "auto"):
        h = T.mis_build_tiles(drp, dci, **kw(cfg), seed=6,
                              poll_rounds=2, launch=launch)
        for rep in range(4):
            out, st = T.mis_solve(h)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), want), f"{launch} replay {rep}"
            assert np.array_equal(st["trace"], trace) and st["rounds"] == rounds
            # auto: a handle's first solve is launched directly, later ones replay a capture
            graph = 1 if launch == "graph" or (launch == "auto" and rep > 0) else 0
            assert st["graph"] == graph, f"{launch} replay {rep}: graph flag {st['graph']}"
            _ = torch.ones(1000, device="cuda").sum().item()   # unrelated eager work between replays
        T.mis_free_tiles(h)


@pytest.mark.parametrize("cfg", FAST_CONFIGS, ids=lambda c: "-".join(map(str, c)))
def test_output_at_any_alignment(cfg):
    # the result vector may start at any byte: the tile path writes four results per
    # store when it is 4-byte aligned and one per store otherwise; n is not a
    # multiple of 4, so the aligned case also has a tail
    T = tcmis_mod()
    g = gen.workload("er10k", seed=7)
    n = g.n - 3
    rp = g.row_ptr[: n + 1]
    keep = g.col_idx[: rp[-1]] < n
    src = np.repeat(np.arange(n), np.diff(rp))[keep]
    ci_ = g.col_idx[: rp[-1]][keep]
    rp2 = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp2, src + 1, 1)
    rp2 = np.cumsum(rp2)
    assert n % 4 != 0
    k = oracle.keys(rp2, 2)
    want, _, _ = expected(rp2, ci_, k)
    drp, dci = to_dev(rp2, ci_)
    h = T.mis_build_tiles(drp, dci, **kw(cfg), seed=2, validate=True)
    base = torch.full((n + 8,), 7, dtype=torch.uint8, device="cuda")
    for off in range(4):
        base.fill_(7)
        out, _ = T.mis_solve(h, out=base[off:off + n])
        torch.cuda.synchronize()
        b = base.cpu().numpy()
        assert np.array_equal(b[off:off + n], want), f"offset {off}"
        assert (b[:off] == 7).all() and (b[off + n:] == 7).all(), f"offset {off}: wrote outside the result"
    T.mis_free_tiles(h)


@pytest.mark.parametrize("cfg", FAST_CONFIGS, ids=lambda c: "-".join(map(str, c)))
def test_persistent_cooperative_rounds(cfg):
    # poll_rounds rounds per cooperative launch with grid barriers between phases:
    # same set, round count and trace as the oracle, over several solves per handle,
    # with a round limit, and for a batch
    T = tcmis_mod()
    for name in ("er10k", "grid24", "rmat12"):
        g = gen.workload(name, seed=3)
        k = oracle.keys(g.row_ptr, 6)
        want, rounds, trace = expected(g.row_ptr, g.col_idx, k)
        drp, dci = to_dev(g.row_ptr, g.col_idx)
        h = T.mis_build_tiles(drp, dci, **kw(cfg), seed=6,
                              poll_rounds=3, launch="persistent")
        for rep in range(2):
            print(f"case persistent {name} cfg={cfg} rep={rep}", flush=True)
            out, st = T.mis_solve(h)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), want), f"{name} rep {rep}"
            assert np.array_equal(st["trace"], trace) and st["rounds"] == rounds and st["graph"] == 2
        if rounds > 1:
            part, r1, _ = expected(g.row_ptr, g.col_idx, k, max_rounds=rounds - 1)
            out, st = T.mis_solve(h, max_rounds=rounds - 1)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), part) and st["rounds"] == r1
        T.mis_free_tiles(h)
    graphs = [gen.make(*s) for s in gen.batch_spec(12, seed=4, n_min=30, n_max=3000)]
    rp, ci, off = gen.union(graphs)
    drp, dci = to_dev(rp, ci)
    h = T.mis_build_batch(drp, dci, off, **kw(cfg), seed=2,
                          launch="persistent")
    out, st, rounds, sizes = T.mis_solve_union(h)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    for i, g in enumerate(graphs):
        want, r, _ = expected(g.row_ptr, g.col_idx, oracle.keys(g.row_ptr, 2))
        assert np.array_equal(got[off[i]:off[i + 1]], want) and rounds[i] == r, f"batch graph {i}"
    T.mis_free_tiles(h)


BATCH_CONFIGS = [("csr", 0, "none", 0), ("tile", 16, "key", 1), ("tile", 32, "degree", 0), ("tile", 16, "rcm", 1),
                 ("hybrid", 16, "none", 1, -1), ("hybrid", 16, "none", 1, 1)]


def solve_batch(graphs, cfg, seed):
    T = tcmis_mod()
    rp, ci, off = gen.union(graphs)
    drp, dci = to_dev(rp, ci)
    h = T.mis_build_batch(drp, dci, off, **kw(cfg), seed=seed,
                          validate=True, poll_rounds=3)
    out, st, rounds, sizes = T.mis_solve_union(h)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    T.mis_free_tiles(h)
    return got, st, rounds, sizes, off


@pytest.mark.parametrize("cfg", BATCH_CONFIGS, ids=lambda c: "-".join(map(str, c)))
def test_batch_equals_each_graph_alone(cfg):
    # disjoint union with graph-local priorities: every graph's slice, round count
    # and set size equal its own round-synchronous solve
    spec = gen.batch_spec(40, seed=5, n_min=20, n_max=4000)
    graphs = [gen.make(*s) for s in spec]
    graphs.insert(7, gen.er(1, 0, 1))          # a one-vertex graph
    graphs.insert(11, gen.er(0, 0, 1))         # an empty graph
    got, st, rounds, sizes, off = solve_batch(graphs, cfg, seed=11)
    worst = 0
    for i, g in enumerate(graphs):
        want, r, tr = expected(g.row_ptr, g.col_idx, oracle.keys(g.row_ptr, 11))
        assert np.array_equal(got[off[i]:off[i + 1]], want), f"graph {i} {spec[i] if i < len(spec) else ''}"
        assert rounds[i] == r and sizes[i] == int(want.sum()), f"graph {i}"
        worst = max(worst, r)
    assert st["rounds"] == worst and st["n_in"] == int(sizes.sum())


@pytest.mark.parametrize("cfg", [("tile", 16, "key", 1), ("hybrid", 16, "none", 1, 1), ("csr", 0, "none", 0)],
                         ids=lambda c: "-".join(map(str, c)))
def test_batch_eq1_rule_uses_each_graphs_own_average(cfg):
    # Eq. 1's average degree is each graph's own in a batch: graph g's keys are the
    # oracle's keys of graph g alone
    T = tcmis_mod()
    graphs = [gen.make(*s) for s in gen.batch_spec(16, seed=9, n_min=50, n_max=5000)]
    rp, ci, off = gen.union(graphs)
    drp, dci = to_dev(rp, ci)
    h = T.mis_build_batch(drp, dci, off, seed=4, key_rule="eq1", validate=True, **kw(cfg))
    out, st, rounds, sizes = T.mis_solve_union(h)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    T.mis_free_tiles(h)
    for i, g in enumerate(graphs):
        want, r, _ = expected(g.row_ptr, g.col_idx, oracle.keys_rule(g.row_ptr, 4, "eq1"))
        assert np.array_equal(got[off[i]:off[i + 1]], want) and rounds[i] == r, f"graph {i}"


def test_batch_of_prebuilt_handles():
    # handles built one by one (different sizes, families and dense-block thresholds,
    # an empty graph and a single vertex among them) solved together without any
    # concatenation: every graph's set and round count equal the oracle's, the same
    # handles solve alone to the same sets, and a non-hybrid handle is refused
    T = tcmis_mod()
    spec = gen.batch_spec(24, seed=9, n_min=50, n_max=30000)
    graphs = [gen.make(*sp) for sp in spec] + [gen.grid(9, 10, 11, 0.01, 4), gen.er(0, 0, 1), gen.er(1, 0, 1)]
    dense = [-1, 1, 9, 4]
    hs, keep = [], []
    for i, g in enumerate(graphs):
        drp, dci = to_dev(g.row_ptr, g.col_idx)
        keep.append((drp, dci))
        hs.append(T.mis_build_tiles(drp, dci, path="hybrid", dense_min=dense[i % 4], seed=11))
    torch.cuda.synchronize()
    outs, st, rounds, sizes = T.mis_solve_batch(hs)
    torch.cuda.synchronize()
    print(f"case handles batch: {len(hs)} graphs, rounds {st['rounds']}", flush=True)
    for i, g in enumerate(graphs):
        want, r, _ = expected(g.row_ptr, g.col_idx, oracle.keys(g.row_ptr, 11))
        assert np.array_equal(outs[i].cpu().numpy()[: g.n], want), f"graph {i} {spec[i] if i < len(spec) else ''}"
        assert rounds[i] == r and sizes[i] == int(want.sum()), f"graph {i}"
        if i % 5 == 0:
            alone, st1 = T.mis_solve(hs[i])
            assert np.array_equal(alone.cpu().numpy(), want[: g.n]) and st1["rounds"] == r
    assert st["rounds"] == int(rounds.max()) and st["n_in"] == int(sizes.sum())
    # a second solve of the same handles with the same scratch: identical
    outs2, _, rounds2, _ = T.mis_solve_batch(hs)
    assert all(torch.equal(a, b) for a, b in zip(outs, outs2)) and np.array_equal(rounds, rounds2)
    drp, dci = keep[0]
    other = T.mis_build_tiles(drp, dci, path="csr", seed=11)
    with pytest.raises(T.MisError) as ei:
        T.mis_solve_batch([hs[0], other])
    assert ei.value.code == T.MIS_EINVAL
    for h in hs + [other]:
        T.mis_free_tiles(h)


def test_batch_rejects_cross_edges():
    T = tcmis_mod()
    rp, ci = csr_from_edges(6, [(0, 1), (2, 3), (3, 4)])
    drp, dci = to_dev(rp, ci)
    T.mis_build_batch(drp, dci, [0, 2, 6], validate=True)      # fine: no edge crosses
    with pytest.raises(T.MisError) as ei:
        T.mis_build_batch(drp, dci, [0, 3, 6], validate=True)  # edge 2-3 joins the graphs
    assert ei.value.code == T.MIS_EINVAL


def test_autotune_picks_a_valid_config_and_caches_it():
    T = tcmis_mod()
    T.mis_autotune_clear()
    for name in ("er10k", "rmat14"):
        g = gen.workload(name, seed=2)
        drp, dci = to_dev(g.row_ptr, g.col_idx)
        opts, cached = T.mis_autotune(drp, dci, seed=4)
        print(f"case autotune {name} -> {opts['path']} T={opts['tile']} {opts['reorder']} "
              f"bpc={opts['blocks_per_cu']} cached={cached}", flush=True)
        assert not cached
        assert opts["path"] in ("tile", "csr", "hybrid") and opts["blocks_per_cu"] in (4, 8, 16)
        if opts["path"] == "tile":
            assert opts["tile"] in (16, 32) and opts["reorder"] in ("key", "none", "degree", "rcm")
        if opts["path"] == "hybrid":
            assert opts["tile"] == 16 and opts["dense_min"] in (-1, 4, 9, 16)
        again, cached = T.mis_autotune(drp, dci, seed=4)
        assert cached and again == opts
        h = T.mis_build_tiles(drp, dci, validate=True, **opts)
        out, st = T.mis_solve(h)
        torch.cuda.synchronize()
        want, rounds, trace = expected(g.row_ptr, g.col_idx, oracle.keys(g.row_ptr, 4))
        assert np.array_equal(out.cpu().numpy(), want) and st["rounds"] == rounds
        assert np.array_equal(st["trace"], trace)
        T.mis_free_tiles(h)
    # a fixed path is kept
    opts, _ = T.mis_autotune(drp, dci, path="csr", seed=4)
    assert opts["path"] == "csr" and opts["tile"] == 0


def test_autotune_batch():
    T = tcmis_mod()
    graphs = [gen.make(*s) for s in gen.batch_spec(24, seed=8, n_min=50, n_max=3000)]
    rp, ci, off = gen.union(graphs)
    drp, dci = to_dev(rp, ci)
    opts, _ = T.mis_autotune(drp, dci, off, seed=3)
    h = T.mis_build_batch(drp, dci, off, validate=True, **opts)
    out, st, rounds, sizes = T.mis_solve_union(h)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    T.mis_free_tiles(h)
    for i, g in enumerate(graphs):
        want, r, _ = expected(g.row_ptr, g.col_idx, oracle.keys(g.row_ptr, 3))
        assert np.array_equal(got[off[i]:off[i + 1]], want) and rounds[i] == r, f"graph {i}"


def _oracle_slices(rp_h, ci_h, off, seed, rule="degree", threads=16):
    """Oracle in/out vector and rounds of every graph of a union, graphs in parallel
    (the oracle's C calls release the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor

    def one(gi):
        va, vb = int(off[gi]), int(off[gi + 1])
        ea, eb = int(rp_h[va]), int(rp_h[vb])
        grp = rp_h[va:vb + 1] - ea
        gci = ci_h[ea:eb] - va
        st, r, _ = oracle.roundsync(grp, gci, oracle.keys_rule(grp, seed, rule))
        return (st == oracle.IN).astype(np.uint8), r

    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(one, range(len(off) - 1)))


@pytest.mark.slow
def test_batch4096_full_against_oracle():
    # the full 4,096-graph batch workload (log-uniform 500..200,000 vertices, half
    # Erdos-Renyi, half R-MAT; 2.2e9 adjacency entries) as ONE hybrid handle: every
    # graph's slice and round count equal the oracle's solve of that graph alone
    T = tcmis_mod()
    spec = gen.batch_spec(4096, seed=1)
    rp_h, ci_h, off = gen.batch_union(spec)
    print(f"case batch4096 n={off[-1]} nnz={ci_h.size}", flush=True)
    drp, dci = to_dev(rp_h, ci_h)
    h = T.mis_build_batch(drp, dci, off, path="hybrid", seed=1)
    out, st, rounds, sizes = T.mis_solve_union(h)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    T.mis_free_tiles(h)
    del drp, dci
    torch.cuda.empty_cache()
    want = _oracle_slices(rp_h, ci_h, off, 1)
    for gi, (w, r) in enumerate(want):
        assert np.array_equal(got[off[gi]:off[gi + 1]], w), f"graph {gi} {spec[gi]}"
        assert rounds[gi] == r and sizes[gi] == int(w.sum()), f"graph {gi}"
    assert st["rounds"] == max(r for _, r in want)


@pytest.mark.slow
def test_serving_pool_full_against_oracle():
    # every graph of the serving workload's request pool (log-uniform 1e3..4e6
    # vertices, Erdos-Renyi / R-MAT / 3D grid) through a continuous-batching session,
    # admitted all at once as far as the arena allows: each result equals the oracle
    T = tcmis_mod()
    spec = gen.serve_spec(48, seed=1)
    rp_h, ci_h, off = gen.batch_union(spec)
    want = _oracle_slices(rp_h, ci_h, off, 1)
    pool = []
    for i in range(len(spec)):
        va, vb = int(off[i]), int(off[i + 1])
        ea, eb = int(rp_h[va]), int(rp_h[vb])
        pool.append((torch.from_numpy(rp_h[va:vb + 1] - ea).pin_memory(),
                     torch.from_numpy(ci_h[ea:eb] - va).pin_memory(), vb - va))
    r = lambda x: (x + 255) // 256 * 256
    foot = max(r(T.mis_build_bytes(p[2], p[1].numel())) + r((p[2] + 1) * 8) + r(p[1].numel() * 4) + r(p[2])
               for p in pool)
    sess = T.Session(arena_bytes=3 * foot, max_live=8, rounds_per_step=4)
    outs = {i: torch.zeros(max(p[2], 1), dtype=torch.uint8).pin_memory() for i, p in enumerate(pool)}
    pending, done = list(range(len(pool))), {}
    while pending or sess.query()[0] > 0:
        while pending and sess.admit(pool[pending[0]][0], pool[pending[0]][1], tag=pending[0],
                                     host_out=outs[pending[0]][: pool[pending[0]][2]]):
            print(f"admit pool graph {pending[0]} n={pool[pending[0]][2]}", flush=True)
            pending.pop(0)
        for d in sess.progress(wait=True):
            assert d["status"] == 0
            done[d["tag"]] = d
    sess.close()
    for i, (w, rr) in enumerate(want):
        assert np.array_equal(outs[i].numpy()[: pool[i][2]], w), f"pool graph {i} {spec[i]}"
        assert done[i]["rounds"] == rr, f"pool graph {i}"
