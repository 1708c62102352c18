"""Benchmark: MIS Medges/s per graph on one MI355X, hybrid tile path vs CSR path.

One step = one pass of the hot path on the R-MAT scale-22 graph (n = 4,194,304,
|E| = 33,554,432, a,b,c,d = .57,.19,.19,.05, random relabelling) resident in HBM:
priority keys, the orientation of every edge towards its higher-priority end, the
dense 16-row blocks as bit tiles and the rest as entry lists (mis_build_tiles, hybrid
path), then the rounds of candidate / exclusion kernels until every vertex is
decided (mis_solve).  value = |E| (undirected, counted once) / step time.  The
device workspace and the output vector are allocated once, before the timed steps,
and passed to every build and solve (as a serving caller does).

Also reported: solve-only throughput (structure built once), the build's stages,
the all-tile path (every edge in reordered bit tiles) and the scalar CSR path on the
same graph, per-kernel HIP-event timings, the roofline of the step's dominant
kernel, and the CPU oracle and sequential greedy timed on this host.

"configs": the 10,000-vertex Erdos-Renyi graph (hybrid and CSR paths) and the 256^3
7-point mesh with 1% long-range pairs (hybrid, CSR, and the all-tile path at 16x16 and
32x32 tiles in natural and RCM order, with tile density and the exclusion kernel's
fraction of the HBM roofline); every leg's set is compared with the first leg's.

"dynamic": batches of 1,000, 10,000 and 100,000 random edge edits (half deletions, half
insertions) on a dynamic handle of the benchmark graph and of the 256^3 mesh, each applied with its local
repair, against a full solve of the edited handle (same set required).

"batch": 4,096 independent graphs (sizes log-uniform over 500..200,000 vertices,
half Erdos-Renyi with average degree 4..32, half R-MAT with 8..24) solved as one
block-diagonal batch (mis_build_batch + mis_solve_union) against one graph per
build+solve; graphs/s and Medges/s.

"serving": a pool of requests (log-uniform 1e3..4e6 vertices, Erdos-Renyi / R-MAT /
3D grid) in pinned host memory; Poisson arrivals at 0.5, 0.8, 1.0 and 1.2 times
the measured one-at-a-time capacity; the continuous-batching session against the
same session limited to one live request (FCFS, one graph per launch); graphs/s
and p50/p99 latency from arrival to result in host memory (H2D, build, solve, D2H).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload rmat22]
                       [--batch-graphs 4096] [--serve-requests 2000] [--no-batch] [--no-serve]
                       [--no-configs] [--no-tune] [--no-dynamic] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def measured_traffic(a, kernel):
    """HBM bytes per launch of `kernel` from its committed counter record
    (profiles/<kernel>_<workload>_traffic.json: rocprofv3 FETCH_SIZE / WRITE_SIZE,
    each scaled by the counter's reading for a copy of known size), or None when the
    record is missing, was taken on another configuration, or the kernel sources
    changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{a.workload}_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if (rec.get("workload"), rec.get("seed"), rec.get("dense_min")) != (a.workload, a.seed, a.dense_min):
        return None
    for name, digest in rec.get("source_sha256", {}).items():
        src = os.path.join(ROOT, "paper_2605_29604_amd", "csrc", name)
        if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != digest:
            return None
    return int(rec["traffic_bytes_per_launch"])


def stored_quality(a):
    """MIS sizes of the benchmark graph under the sequential min-degree greedy heuristic and
    the greedy pass in key order, stored by tests/golden/make_quality.py (seed-1 graph,
    default keys of seed 1), or None for another workload."""
    path = os.path.join(ROOT, "tests", "golden", "rmat22_quality.json")
    if a.workload != "rmat22" or a.seed != 1 or not os.path.exists(path):
        return None
    return json.load(open(path))


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="rmat22")
    p.add_argument("--seed", type=int, default=1)
    p.add_argument("--tile", type=int, default=16)
    p.add_argument("--reorder", default="key")
    p.add_argument("--orient", type=int, default=1)
    p.add_argument("--dense-min", type=int, default=0, help="hybrid path's dense-block threshold (0 = default)")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--no-batch", action="store_true")
    p.add_argument("--no-serve", action="store_true")
    p.add_argument("--batch-graphs", type=int, default=4096)
    p.add_argument("--serve-requests", type=int, default=2000)
    p.add_argument("--serve-pool", type=int, default=48)
    p.add_argument("--serve-live", type=int, default=8)
    p.add_argument("--no-tune", action="store_true")
    p.add_argument("--no-configs", action="store_true", help="skip the er10k and grid256 legs")
    p.add_argument("--no-dynamic", action="store_true", help="skip the edge-edit leg")
    return p.parse_args()


def log(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


def pct(x, q):
    return round(float(np.percentile(np.asarray(x), q)), 3) if len(x) else None


def path_leg(torch, tcmis, rp, ci, n, m, cfg, steps, warmup):
    """One configuration on one resident graph: the build + solve step (workspace and
    output allocated once), solve only (structure built once), and one more solve with
    per-kernel HIP events on the solve stream."""
    ws = torch.empty(tcmis.mis_build_bytes(n, int(ci.numel()), **cfg), dtype=torch.uint8, device="cuda")
    out = torch.empty(n, dtype=torch.uint8, device="cuda")

    def one():
        h = tcmis.mis_build_tiles(rp, ci, workspace=ws, **cfg)
        _, st = tcmis.mis_solve(h, out=out, trace_cap=0)
        tcmis.mis_free_tiles(h)
        return st

    for _ in range(warmup):
        one()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        st = one()
    torch.cuda.synchronize()
    step = (time.perf_counter() - t) / steps
    h = tcmis.mis_build_tiles(rp, ci, workspace=ws, **cfg)
    for _ in range(2):   # the second solve of a handle captures its round loop (auto launch mode)
        tcmis.mis_solve(h, out=out, trace_cap=0)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        tcmis.mis_solve(h, out=out, trace_cap=0)
    torch.cuda.synchronize()
    solve = (time.perf_counter() - t) / steps
    _, stt = tcmis.mis_solve(h, out=out, timing=True, trace_cap=0)
    tcmis.mis_free_tiles(h)
    rec = {"step_ms": round(step * 1e3, 4), "step_medges_s": round(m / step / 1e6, 1),
           "solve_ms": round(solve * 1e3, 4), "solve_medges_s": round(m / solve / 1e6, 1),
           "rounds": st["rounds"], "kernel_ms": [round(x, 4) for x in stt["kernel_ms"]]}
    if cfg["path"] == "tile":
        t_ = st["tile"]
        ents = int(ci.numel()) // (2 if cfg.get("orient", 1) else 1)
        rec["tiles"] = st["tiles"]
        rec["density_nnz_per_tile"] = round(ents / max(1, st["tiles"]), 3)
        # exclusion kernel against the HBM roofline with the per-solve bytes of the
        # tile stream: T*T/8 bitmap + 4-byte column block per multiplied tile, and the
        # two per-vertex bitmaps once per launch
        u = stt["units"]
        xb = u[3] * (t_ * t_ // 8 + 4) + max(1, stt["launches"]) * (n // 4)
        if stt["kernel_ms"][1] > 0:
            gbs = xb / (stt["kernel_ms"][1] * 1e-3) / 1e9
            rec["exclusion"] = {"alg_bytes": int(xb), "achieved_gbs": round(gbs, 1),
                                "frac": round(gbs / HBM_PEAK_GBS, 4)}
    elif cfg["path"] == "hybrid":
        rec["dense_tiles"] = st["tiles"]
    return rec, out.clone()


def bench_configs(a, torch, gen, tcmis, grid):
    """The other single-graph workloads: the 10,000-vertex Erdos-Renyi graph (hybrid and
    CSR paths; launch-bound at this size) and the 256^3 mesh with 1% long-range pairs
    (hybrid, CSR, and the all-tile path at 16x16 and 32x32 in natural and RCM order,
    with tile density and the exclusion kernel's roofline fraction)."""
    res = {}
    legs = [("hybrid", dict(path="hybrid", seed=a.seed)), ("csr", dict(path="csr", seed=a.seed))]
    cases = [("er10k", gen.workload("er10k", seed=1), list(legs), 20, 5)]
    for t_ in (16, 32):
        for order in ("none", "rcm"):
            legs.append((f"tile{t_}_{'natural' if order == 'none' else order}",
                         dict(path="tile", tile=t_, reorder=order, orient=1, seed=a.seed)))
    cases.append(("grid256", grid, legs, 3, 1))
    for name, g, legs_, steps, warmup in cases:
        rp = torch.from_numpy(g.row_ptr).cuda()
        ci = torch.from_numpy(g.col_idx).cuda()
        rec = {"n": g.n, "edges": g.m}
        first = None
        agree = True
        for leg, cfg in legs_:
            r, o = path_leg(torch, tcmis, rp, ci, g.n, g.m, cfg, steps, warmup)
            if first is None:
                first = o
            else:
                agree = agree and bool(torch.equal(first, o))
            rec[leg] = r
            log(f"{name} {leg}: {r}")
        rec["paths_agree"] = agree
        res[name] = rec
        del rp, ci
        torch.cuda.empty_cache()
    return res


def bench_dynamic(a, torch, tcmis, graphs):
    """Dynamic graphs: batches of random edge edits on a dynamic hybrid handle of each
    graph (half deletions of present edges, half insertions of absent ones), each applied
    with its local repair (mis_update_edges), against a full solve of the edited handle;
    the repaired set must equal that solve's."""
    out = {}
    for name, g in graphs:
        rp = torch.from_numpy(g.row_ptr).cuda()
        ci = torch.from_numpy(g.col_idx).cuda()
        out[name] = dynamic_leg(a, torch, tcmis, name, g, rp, ci)
        del rp, ci
        torch.cuda.empty_cache()
    return out


def dynamic_leg(a, torch, tcmis, name, g, rp, ci):
    cfg = dict(path="hybrid", dense_min=-1, dyn_slack=8, seed=a.seed)
    t0 = time.perf_counter()
    h = tcmis.mis_build_tiles(rp, ci, **cfg)
    out, _ = tcmis.mis_solve(h, trace_cap=0)
    torch.cuda.synchronize()
    res = {"config": "hybrid, entry lists, 8 free slots per row and orientation",
           "build_and_solve_ms": round((time.perf_counter() - t0) * 1e3, 3), "batches": []}
    rph, cih = g.row_ptr, g.col_idx
    rng = np.random.default_rng(7)
    deleted, inserted = set(), set()

    def present(u, v):
        if (u, v) in inserted:
            return True
        if (u, v) in deleted:
            return False
        row = cih[rph[u]:rph[u + 1]]
        i = int(np.searchsorted(row, v))
        return i < row.size and int(row[i]) == v

    for k in (1000, 10000, 100000):
        dels, ins = set(), set()
        while len(dels) < k // 2:
            e = int(rng.integers(cih.size))
            u = int(np.searchsorted(rph, e, side="right")) - 1
            v = int(cih[e])
            p = (min(u, v), max(u, v))
            if p not in dels and p not in deleted:
                dels.add(p)
        while len(ins) < k // 2:
            u, v = int(rng.integers(g.n)), int(rng.integers(g.n))
            p = (min(u, v), max(u, v))
            if u != v and p not in ins and p not in dels and not present(*p):
                ins.add(p)
        pairs = np.array(sorted(dels) + sorted(ins), dtype=np.int32).reshape(-1, 2)
        ops = np.array([0] * len(dels) + [1] * len(ins), dtype=np.int8)
        perm = rng.permutation(len(ops))
        d_pairs = torch.from_numpy(np.ascontiguousarray(pairs[perm])).cuda()
        d_ops = torch.from_numpy(ops[perm]).cuda()
        torch.cuda.synchronize()
        t = time.perf_counter()
        info = tcmis.mis_update_edges(h, d_pairs, d_ops, out)
        torch.cuda.synchronize()
        upd = time.perf_counter() - t
        deleted |= dels - inserted
        inserted = (inserted - dels) | ins
        t = time.perf_counter()
        full, st = tcmis.mis_solve(h, trace_cap=0)
        torch.cuda.synchronize()
        fs = time.perf_counter() - t
        rec = {"edits": len(ops), "update_and_repair_ms": round(upd * 1e3, 3), "repair_rounds": info["rounds"],
               "entries_read": info["entries_read"], "full_solve_ms": round(fs * 1e3, 3),
               "same_set_as_full_solve": bool(torch.equal(full, out)), "mis_size": int(st["n_in"])}
        res["batches"].append(rec)
        log(f"dynamic {name}: {rec}")
    tcmis.mis_free_tiles(h)
    return res


def bench_tune(a, torch, gen, tcmis, rp, ci, grid):
    """The autotuner's pick (path, tile size, order, workgroups per CU) for the R-MAT
    graph and for the 256^3 mesh, with the build + solve time of the pick."""
    out = {}
    tcmis.mis_autotune_clear()
    cases = [(a.workload, rp, ci)]
    cases.append(("grid256", torch.from_numpy(grid.row_ptr).cuda(), torch.from_numpy(grid.col_idx).cuda()))
    for name, r, c in cases:
        t = time.perf_counter()
        opts, cached = tcmis.mis_autotune(r, c, seed=a.seed)
        tune_s = time.perf_counter() - t
        for _ in range(2):
            h = tcmis.mis_build_tiles(r, c, **opts)
            tcmis.mis_solve(h, trace_cap=0)
            tcmis.mis_free_tiles(h)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(3):
            h = tcmis.mis_build_tiles(r, c, **opts)
            tcmis.mis_solve(h, trace_cap=0)
            tcmis.mis_free_tiles(h)
        torch.cuda.synchronize()
        step = (time.perf_counter() - t) / 3
        edges = c.numel() // 2
        out[name] = {"pick": {k: opts[k] for k in ("path", "tile", "reorder", "orient", "blocks_per_cu", "dense_min")},
                     "tune_s": round(tune_s, 3), "step_ms": round(step * 1e3, 4),
                     "step_medges_s": round(edges / step / 1e6, 1)}
        log(f"autotune {name}: {out[name]}")
    del cases
    torch.cuda.empty_cache()
    return out


def bench_batch(a, torch, gen, tcmis):
    """The 4,096-graph mix as one block-diagonal hybrid batch (64-bit entry offsets: one
    handle, every round kernel covering all graphs) vs one graph per build + solve.
    The step (build + solve) is timed with direct launches; solve-only is timed again
    with the round loop replayed as a captured hipGraph (the handle's second solve on)."""
    t0 = time.perf_counter()
    spec = gen.batch_spec(a.batch_graphs, seed=1)
    rp_h, ci_h, off = gen.batch_union(spec)
    log(f"batch: {len(spec)} graphs, n={off[-1]} nnz={ci_h.size} generated in {time.perf_counter() - t0:.1f}s")
    cfg = dict(path="hybrid", dense_min=a.dense_min, seed=a.seed)
    rp = torch.from_numpy(rp_h).cuda()
    ci = torch.from_numpy(ci_h).cuda()
    ws = torch.empty(tcmis.mis_build_batch_bytes(rp.numel() - 1, ci.numel(), off, **cfg), dtype=torch.uint8,
                     device="cuda")
    out = torch.empty(rp.numel() - 1, dtype=torch.uint8, device="cuda")

    def batched():
        t = time.perf_counter()
        h = tcmis.mis_build_batch(rp, ci, off, workspace=ws, launch="direct", **cfg)
        _, st, r, _ = tcmis.mis_solve_union(h, out=out, trace_cap=0)
        tcmis.mis_free_tiles(h)
        return time.perf_counter() - t, int(st["rounds"]), r

    batched()
    torch.cuda.synchronize()
    reps = [batched() for _ in range(3)]
    b_s = float(np.median([r[0] for r in reps]))
    g_rounds = reps[-1][2]
    # solve only, the round loop captured once and replayed
    h = tcmis.mis_build_batch(rp, ci, off, workspace=ws, launch="graph", **cfg)
    tcmis.mis_solve_union(h, out=out, trace_cap=0)
    torch.cuda.synchronize()
    ts = []
    for _ in range(3):
        t = time.perf_counter()
        _, st_g, _, _ = tcmis.mis_solve_union(h, out=out, trace_cap=0)
        ts.append(time.perf_counter() - t)
    g_solve_s = float(np.median(ts))
    graph_flag = st_g["graph"]
    tcmis.mis_free_tiles(h)
    # one graph per build + solve, on per-graph device copies of the same CSR
    singles = []
    for gi in range(len(spec)):
        va, vb = int(off[gi]), int(off[gi + 1])
        ea, eb = int(rp_h[va]), int(rp_h[vb])
        singles.append((rp[va:vb + 1] - ea, ci[ea:eb] - va))
    torch.cuda.synchronize()
    one_ws = torch.empty(max(tcmis.mis_build_bytes(r.numel() - 1, c.numel(), **cfg) for r, c in singles),
                         dtype=torch.uint8, device="cuda")
    one_out = torch.empty(max(r.numel() - 1 for r, _ in singles), dtype=torch.uint8, device="cuda")

    def one_by_one(k):
        done_t = []
        t = time.perf_counter()
        for rps, cis in singles[:k]:
            hh = tcmis.mis_build_tiles(rps, cis, workspace=one_ws, **cfg)
            tcmis.mis_solve(hh, out=one_out[: rps.numel() - 1], trace_cap=0)
            tcmis.mis_free_tiles(hh)
            done_t.append(time.perf_counter() - t)
        return time.perf_counter() - t, done_t

    one_by_one(64)
    torch.cuda.synchronize()
    o_s, o_done = one_by_one(len(singles))
    # every 16th graph of the batch equals the same graph solved alone
    same = True
    for gi in range(0, len(singles), 16):
        rps, cis = singles[gi]
        hh = tcmis.mis_build_tiles(rps, cis, workspace=one_ws, **cfg)
        alone, _ = tcmis.mis_solve(hh, out=one_out[: rps.numel() - 1], trace_cap=0)
        tcmis.mis_free_tiles(hh)
        same &= bool(torch.equal(alone, out[int(off[gi]):int(off[gi + 1])]))
    edges = int(ci_h.size) // 2
    res = {"graphs": len(spec), "vertices": int(off[-1]), "edges": edges, "handles": 1,
           "config": f"hybrid, dense_min {a.dense_min}",
           "batched": {"s": round(b_s, 4), "graphs_s": round(len(spec) / b_s, 1),
                       "medges_s": round(edges / b_s / 1e6, 1), "rounds": reps[-1][1],
                       "graph_rounds_p50": pct(g_rounds, 50), "graph_rounds_max": int(np.max(g_rounds)),
                       "latency_ms": round(b_s * 1e3, 3),
                       "note": "one launch group: every graph finishes with the batch"},
           "batched_solve_graph_replay": {"s": round(g_solve_s, 4), "graph_flag": graph_flag,
                                          "medges_s": round(edges / g_solve_s / 1e6, 1)},
           "one_graph_per_launch": {"s": round(o_s, 4), "graphs_s": round(len(singles) / o_s, 1),
                                    "medges_s": round(edges / o_s / 1e6, 1),
                                    "p50_ms": pct(np.array(o_done) * 1e3, 50),
                                    "p99_ms": pct(np.array(o_done) * 1e3, 99)},
           "speedup": round(o_s / b_s, 2), "batch_equals_alone_sampled": same}
    del singles, one_ws, one_out, ws, out, rp, ci
    torch.cuda.empty_cache()
    return res


def bench_serve(a, torch, gen, tcmis):
    """Continuous-batching session vs FCFS one-at-a-time on the same Poisson traces."""
    t0 = time.perf_counter()
    spec = gen.serve_spec(a.serve_pool, seed=1)
    rp_h, ci_h, off = gen.batch_union(spec)
    pool = []
    for i in range(len(spec)):
        va, vb = int(off[i]), int(off[i + 1])
        ea, eb = int(rp_h[va]), int(rp_h[vb])
        rp = torch.from_numpy(rp_h[va:vb + 1] - ea).pin_memory()
        ci = torch.from_numpy(ci_h[ea:eb] - va).pin_memory()
        pool.append((rp, ci, vb - va))
    del rp_h, ci_h
    log(f"serving pool: {len(pool)} graphs, mean n={np.mean([p[2] for p in pool]):.0f}, "
        f"made in {time.perf_counter() - t0:.1f}s")
    r = lambda x: (x + 255) // 256 * 256
    foot = max(r(tcmis.mis_build_bytes(p[2], p[1].numel())) + r((p[2] + 1) * 8) + r(p[1].numel() * 4) + r(p[2])
               for p in pool)
    arena = torch.empty(max(2 * foot, min(foot * 2 * a.serve_live, 96 << 30)), dtype=torch.uint8, device="cuda")
    nmax = max(p[2] for p in pool)
    rng = np.random.default_rng(12345)
    picks = rng.integers(0, len(pool), size=a.serve_requests)
    ref = {}

    def run(max_live, arrivals):
        sess = tcmis.Session(arena=arena, max_live=max_live, rounds_per_step=4)
        bufs = [torch.empty(nmax, dtype=torch.uint8).pin_memory() for _ in range(max_live)]
        free = list(range(max_live))
        owner, lat, mismatch = {}, [], 0
        nxt, done_n = 0, 0
        t = time.perf_counter()
        while done_n < len(arrivals):
            now = time.perf_counter() - t
            while nxt < len(arrivals) and arrivals[nxt] <= now and free:
                p = pool[picks[nxt]]
                b = free[-1]
                if not sess.admit(p[0], p[1], tag=nxt, host_out=bufs[b][: p[2]]):
                    break
                free.pop()
                owner[nxt] = b
                nxt += 1
            for d in sess.progress(wait=False):
                i = d["tag"]
                lat.append(time.perf_counter() - t - arrivals[i])
                b = owner.pop(i)
                res = bufs[b][: pool[picks[i]][2]]
                k = int(picks[i])
                if k not in ref:
                    ref[k] = res.clone()
                elif not torch.equal(ref[k], res):
                    mismatch += 1
                free.append(b)
                done_n += 1
        span = time.perf_counter() - t
        sess.close()
        lat_ms = np.array(lat) * 1e3
        return {"graphs_s": round(len(arrivals) / span, 1), "p50_ms": pct(lat_ms, 50), "p99_ms": pct(lat_ms, 99),
                "mean_ms": round(float(lat_ms.mean()), 3)}, mismatch

    # capacity of one request at a time (all requests queued at t = 0)
    ncap = min(400, a.serve_requests)
    run(1, np.zeros(min(32, ncap)))
    cap_res, _ = run(1, np.zeros(ncap))
    capacity = cap_res["graphs_s"]
    log(f"serving: one-at-a-time capacity {capacity} graphs/s")
    points, mism = [], 0
    for rel in (0.5, 0.8, 1.0, 1.2):
        rate = rel * capacity
        arrivals = np.cumsum(np.random.default_rng(int(rel * 100)).exponential(1.0 / rate, a.serve_requests))
        mix, m1 = run(a.serve_live, arrivals)
        fcfs, m2 = run(1, arrivals)
        mism += m1 + m2
        points.append({"load": rel, "rate_per_s": round(rate, 1), "continuous": mix, "fcfs_one_at_a_time": fcfs})
        log(f"serving load {rel}: continuous {mix} | fcfs {fcfs}")
    del arena
    torch.cuda.empty_cache()
    return {"requests_per_point": a.serve_requests, "pool": len(pool),
            "pool_mean_n": round(float(np.mean([p[2] for p in pool])), 1), "max_live": a.serve_live,
            "capacity_one_at_a_time_graphs_s": capacity, "points": points,
            "mix_equals_alone": mism == 0, "latency": "arrival to result in pinned host memory"}


def cpu_leg(fn, reps=3):
    """Median of `reps` timings of fn() (seconds) on this host's cores."""
    ts = []
    for _ in range(reps):
        t = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t)
    return float(np.median(ts))


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}); the solver does not shard a graph "
              "or a batch across GPUs", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2605_29604_amd import gen, tcmis

    tcmis.lib()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    g = gen.workload(a.workload, seed=1)
    gen_s = time.perf_counter() - t0
    log(f"workload {a.workload}: n={g.n} |E|={g.m} generated in {gen_s:.1f}s")
    rp = torch.from_numpy(g.row_ptr).to(dev)
    ci = torch.from_numpy(g.col_idx).to(dev)
    torch.cuda.synchronize()

    hyb_cfg = dict(path="hybrid", dense_min=a.dense_min, seed=a.seed)
    tile_cfg = dict(path="tile", tile=a.tile, reorder=a.reorder, orient=a.orient, seed=a.seed)
    csr_cfg = dict(path="csr", seed=a.seed)

    def time_steps(cfg, steps, warmup):
        # workspace and output allocated once; every step builds and solves into them
        ws = torch.empty(tcmis.mis_build_bytes(g.n, int(ci.numel()), **cfg), dtype=torch.uint8, device=dev)
        out = torch.empty(g.n, dtype=torch.uint8, device=dev)

        def one():
            h = tcmis.mis_build_tiles(rp, ci, workspace=ws, **cfg)
            o, st = tcmis.mis_solve(h, out=out, trace_cap=0)
            tcmis.mis_free_tiles(h)
            return o, st

        for _ in range(warmup):
            one()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            o, st = one()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        return dt, o.clone(), st

    def time_solve(cfg, steps, warmup):
        h = tcmis.mis_build_tiles(rp, ci, **cfg)
        for _ in range(max(warmup, 2)):   # the second solve captures the round loop (auto launch mode)
            tcmis.mis_solve(h)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            out, st = tcmis.mis_solve(h)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        # one more solve with per-kernel HIP events on the solve stream
        _, stt = tcmis.mis_solve(h, timing=True)
        nbytes = h.bytes()
        tcmis.mis_free_tiles(h)
        return dt, out, st, stt, nbytes

    def build_stages(cfg, reps):
        # per-stage HIP-event durations of the build (same stream as its kernels)
        ws = torch.empty(tcmis.mis_build_bytes(g.n, int(ci.numel()), **cfg), dtype=torch.uint8, device=dev)
        acc = None
        for _ in range(reps + 1):
            h = tcmis.mis_build_tiles(rp, ci, workspace=ws, timing=True, **cfg)
            ms = tcmis.mis_build_times(h)
            tcmis.mis_free_tiles(h)
            if acc is None:
                acc = [0.0] * len(ms)   # the first build warms up and is not counted
                continue
            acc = [x + y for x, y in zip(acc, ms)]
        return [x / reps for x in acc]

    # ---- the hybrid path (headline): end-to-end steps (timed region = K steps), solve only
    step_s, out_h, st_h = time_steps(hyb_cfg, a.steps, a.warmup)
    solve_s, out_h2, st_h2, stt_h, hyb_mem = time_solve(hyb_cfg, max(a.steps, 10), a.warmup)
    stages = build_stages(hyb_cfg, 5)
    # ---- every edge in bit tiles (the reordered all-tile path)
    t_step_s, out_t, st_t = time_steps(tile_cfg, a.steps, a.warmup)
    t_solve_s, _, _, stt_t, tile_mem = time_solve(tile_cfg, max(a.steps, 10), a.warmup)
    # ---- the scalar CSR path
    csr_step_s, out_csr, st_csr = time_steps(csr_cfg, a.steps, a.warmup)
    csr_solve_s, _, _, stt_c, _ = time_solve(csr_cfg, max(a.steps, 10), a.warmup)

    same = bool(torch.equal(out_h, out_csr) and torch.equal(out_h, out_t) and torch.equal(out_h, out_h2))
    m = g.m
    hyb_names = ["keys and dense-block sample", "dense blocks"]
    res = {
        "metric": "MIS Medges/s per graph at 1 GPU (tile vs CSR); batched graphs/s + p50/p99",
        "value": round(m / step_s / 1e6, 3),
        "unit": "Medges/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(step_s * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"{a.workload} R-MAT scale 22, avg degree 16, random relabelling"
                   if a.workload == "rmat22" else a.workload,
                   "n": g.n, "edges": m, "path": "hybrid", "tile": 16, "dense_min": a.dense_min,
                   "step": "keys + dense-block tiles, then the rounds (round 1 on the CSR, later rounds on the "
                           "oriented rows of the vertices round 1 left undecided); CSR resident in HBM"},
        "hybrid": {"step_ms": round(step_s * 1e3, 4), "solve_ms": round(solve_s * 1e3, 4),
                   "solve_medges_s": round(m / solve_s / 1e6, 3),
                   "build_ms": round((step_s - solve_s) * 1e3, 4),
                   "build_stages_ms": {k: round(v, 4) for k, v in zip(hyb_names, stages[: len(hyb_names)])},
                   "rounds": st_h["rounds"], "dense_tiles": st_h["tiles"], "device_bytes": hyb_mem,
                   "kernel_ms": [round(x, 4) for x in stt_h["kernel_ms"]], "units": stt_h["units"],
                   "alg_bytes": stt_h["alg_bytes"]},
        "tile": {"step_ms": round(t_step_s * 1e3, 4), "solve_ms": round(t_solve_s * 1e3, 4),
                 "solve_medges_s": round(m / t_solve_s / 1e6, 3), "build_ms": round((t_step_s - t_solve_s) * 1e3, 4),
                 "config": f"tile {a.tile}, reorder {a.reorder}, orient {a.orient}",
                 "rounds": st_t["rounds"], "tiles": st_t["tiles"], "tile_bytes": st_t["tile_bytes"],
                 "density_nnz_per_tile": round((g.nnz / (2 if a.orient else 1)) / max(1, st_t["tiles"]), 3),
                 "device_bytes": tile_mem, "kernel_ms": [round(x, 4) for x in stt_t["kernel_ms"]],
                 "units": stt_t["units"], "alg_bytes": stt_t["alg_bytes"]},
        "csr": {"step_ms": round(csr_step_s * 1e3, 4), "step_medges_s": round(m / csr_step_s / 1e6, 3),
                "solve_ms": round(csr_solve_s * 1e3, 4), "solve_medges_s": round(m / csr_solve_s / 1e6, 3),
                "kernel_ms": [round(x, 4) for x in stt_c["kernel_ms"]], "units": stt_c["units"],
                "alg_bytes": stt_c["alg_bytes"]},
        "speedup_vs_csr_step": round(csr_step_s / step_s, 3),
        "mis_size": int(st_h["n_in"]),
        "paths_agree": same,
    }
    q = stored_quality(a)
    if q is not None:   # set size against the sequential min-degree greedy heuristic
        res["quality"] = {"mis_size": res["mis_size"], "mindeg_greedy_size": q["mindeg_greedy_size"],
                          "ratio_to_mindeg_greedy": round(res["mis_size"] / q["mindeg_greedy_size"], 5),
                          "equals_key_greedy": res["mis_size"] == q["key_greedy_size"],
                          "source": "tests/golden/rmat22_quality.json"}
    # roofline of the step's dominant kernel (the most time in the step), from HIP events
    # on the stream it runs on: the dense-block build or one of the two round
    # kernels (solve).  Algorithmic bytes per unit: 4 per adjacency
    # index read, 16 per row examined (row bounds and key or list slot), 36 per 16x16
    # bit tile multiplied, 24 per dense block examined, and the two per-vertex bitmaps
    # (n/8 bytes each) once per launch; the neighbours' class or status lookups are
    # the per-vertex vectors, not counted per entry.  "gather_inclusive" counts 4 more
    # bytes per entry for them.
    u = stt_h["units"]
    launches = max(1, stt_h["launches"])
    vec = launches * (g.n // 4)
    cands = {
        "hybrid_candidate": (stt_h["kernel_ms"][0], launches, u[0] * 4 + u[1] * 16 + u[4] * 36 + u[6] * 24 + vec,
                             u[0] * 4),
        "hybrid_exclusion": (stt_h["kernel_ms"][1], launches, u[2] * 4 + u[3] * 16 + u[5] * 36 + u[7] * 24 + vec,
                             u[2] * 4),
    }
    if len(stages) > 1 and stages[1] > 0 and st_h["tiles"] > 0:   # the dense-block build streams the
        # column indices and the row pointer once, and writes the tiles
        cands["hybrid_dense_build"] = (stages[1], 1, 4 * g.nnz + 8 * (g.n + 1) + 36 * st_h["tiles"], 0)
    name = max(cands, key=lambda k: cands[k][0])
    tot_ms, nl, nbytes, gather = cands[name]
    avg_ms = tot_ms / nl
    achieved = (nbytes / nl) / (avg_ms * 1e-3) / 1e9
    res["roofline"] = {"kernel": name, "bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                       "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                       "traffic": measured_traffic(a, name),
                       "avg_launch_us": round(avg_ms * 1e3, 3), "launches": nl,
                       "alg_bytes_per_launch": int(nbytes / nl),
                       "gather_inclusive": {"achieved": round(((nbytes + gather) / nl) / (avg_ms * 1e-3) / 1e9, 2),
                                            "note": "plus 4 bytes per entry for the neighbour's class/status word"},
                       "others": {k: {"avg_launch_us": round(v[0] / v[1] * 1e3, 3),
                                      "achieved": round((v[2] / v[1]) / (v[0] / v[1] * 1e-3) / 1e9, 2)
                                      if v[0] > 0 else None} for k, v in cands.items() if k != name}}

    # round-loop launch modes of the same solve (identical results)
    modes = {}
    for launch in ("direct", "graph", "persistent"):
        lt, lo, lst, _, _ = time_solve(dict(hyb_cfg, launch=launch), max(a.steps, 10), a.warmup)
        modes[launch] = {"solve_ms": round(lt * 1e3, 4), "same_set": bool(torch.equal(lo, out_h)),
                         "graph_flag": lst["graph"]}
    res["launch_modes"] = modes
    grid = None
    if not (a.no_tune and a.no_configs and a.no_dynamic):
        t0 = time.perf_counter()
        grid = gen.workload("grid256", seed=1)
        log(f"grid256 generated in {time.perf_counter() - t0:.1f}s")
    if not a.no_configs:
        res["configs"] = bench_configs(a, torch, gen, tcmis, grid)
    if not a.no_tune:
        res["autotune"] = bench_tune(a, torch, gen, tcmis, rp, ci, grid)
    if not a.no_dynamic:
        res["dynamic"] = bench_dynamic(a, torch, tcmis, [(a.workload, g)] + ([("grid256", grid)] if grid else []))
    del grid

    if not a.no_batch:
        res["batch"] = bench_batch(a, torch, gen, tcmis)
    if not a.no_serve:
        res["serving"] = bench_serve(a, torch, gen, tcmis)

    if not a.no_cpu:
        import oracle
        key = oracle.keys(g.row_ptr, a.seed)
        holder = {}

        def rs():
            holder["rs"] = oracle.roundsync(g.row_ptr, g.col_idx, key)

        def gr():
            holder["gr"] = oracle.greedy(g.row_ptr, g.col_idx, key)

        rs_s = cpu_leg(rs)
        gr_s = cpu_leg(gr)
        want = (holder["rs"][0] == oracle.IN).astype(np.uint8)
        res["parity_vs_oracle"] = bool(np.array_equal(out_h.cpu().numpy(), want))
        res["cpu_baseline"] = {"value": round(m / rs_s / 1e6, 3), "unit": "Medges/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"the round-synchronous oracle on the whole {a.workload} graph (keys "
                                         f"precomputed), median of 3 runs of {rs_s:.3f}s, one thread",
                               "host_cores": len(os.sched_getaffinity(0)), "cpu_model": cpu_model(),
                               "sequential_greedy": {"value": round(m / gr_s / 1e6, 3), "unit": "Medges/s",
                                                     "seconds": round(gr_s, 4), "cores": 1,
                                                     "same_set": bool(np.array_equal(holder["gr"], want))}}
    print(json.dumps(res))


if __name__ == "__main__":
    main()
