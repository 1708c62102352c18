"""A short program for counter runs under rocprofv3: one tile-path (or, with --path
hybrid, hybrid-path) build and solve of a named workload (the CSR resident on the
device), one CSR-path solve, and one device-to-device copy of a known size, whose
FETCH_SIZE / WRITE_SIZE calibrate the counters against bytes actually moved.

    python paper_2605_29604_amd/profile_run.py [--workload rmat22] [--copy-mib 256] [--path hybrid]

With --summarize-stats DIR NAME BENCH_JSON it writes profiles/NAME.md from one
rocprofv3 --kernel-trace --stats run of bench.py (DIR) and that run's JSON line.

With --summarize-kernel RECORD FETCH_DIR WRITE_DIR it writes the per-launch traffic
record of one hybrid-path kernel (RECORD: hybrid_candidate, hybrid_exclusion,
hybrid_dense_build).

With --summarize FETCH_DIR WRITE_DIR (the output folders of one FETCH_SIZE and one
WRITE_SIZE run of this program) it reads the counters instead, on any machine, and
writes the exclusion kernel's per-launch HBM traffic to profiles/ (a JSON record
that bench.py reports while the kernel sources are unchanged, and a short summary).
With --summarize-mfma DIR (one run with the MFMA counters, see the summary it
writes) it does the same for the kernel's int8 matrix-core use, and with
--summarize-stalls DIR for its wait and address-unit shares.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# the sources the exclusion kernel is built from; its record is void once any changes
TRAFFIC_SOURCES = ("solve_tile.hip", "round.hpp", "graph.hpp")

sys.path.insert(0, ROOT)


def _counter(folder: str, name: str, kernel: str):
    """(first device copy's value, values of every dispatch of `kernel`) in KiB."""
    copy, vals = None, []
    with open(os.path.join(folder, "run_counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != name:
                continue
            k, v = r["Kernel_Name"], float(r["Counter_Value"])
            if "__amd_rocclr_copyBuffer" in k and copy is None:
                copy = v
            elif kernel in k:
                vals.append(v)
    if copy is None or not vals:
        raise SystemExit(f"{folder}: no copy or no {kernel} dispatch with {name}")
    return copy, vals


def _gather_fetch(folder: str):
    """FETCH_SIZE (KiB) of the calibration gather: the first dispatch after the first
    device copy whose kernel is torch's indexing kernel, or None."""
    seen_copy = False
    with open(os.path.join(folder, "run_counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != "FETCH_SIZE":
                continue
            k = r["Kernel_Name"]
            if "__amd_rocclr_copyBuffer" in k:
                seen_copy = True
            elif seen_copy and ("index" in k.lower() or "gather" in k.lower()):
                return float(r["Counter_Value"])
    return None


def _dispatches(folder: str, kernel: str):
    """{dispatch id: (duration ns, {counter: value})} of every dispatch of `kernel`."""
    out = {}
    with open(os.path.join(folder, "run_counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if kernel not in r["Kernel_Name"]:
                continue
            d = out.setdefault(int(r["Dispatch_Id"]),
                               (int(r["End_Timestamp"]) - int(r["Start_Timestamp"]), {}))
            d[1][r["Counter_Name"]] = float(r["Counter_Value"])
    return [out[k] for k in sorted(out)]


def _sources_sha():
    sha = {}
    for name in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2605_29604_amd", "csrc", name), "rb") as fh:
            sha[name] = hashlib.sha256(fh.read()).hexdigest()
    return sha


# MI355X: 8 XCDs, 256 compute units of 4 SIMDs; dense int8 matrix peak 5.0 POP/s.
# GRBM_GUI_ACTIVE reads as the sum over the XCDs (8 x the clock over a dispatch).
XCDS = 8
SIMDS = 1024
INT8_PEAK_TOPS = 5000.0


def summarize_mfma(a) -> int:
    kernel = f"k_tile_excl<{a.tile}>"
    rows = _dispatches(a.summarize_mfma, kernel)
    if not rows:
        raise SystemExit(f"{a.summarize_mfma}: no {kernel} dispatch")
    per = []
    for ns, c in rows:
        ops = c.get("SQ_INSTS_VALU_MFMA_MOPS_I8", 0.0) * 512.0
        busy = c.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0)
        gui = c.get("GRBM_GUI_ACTIVE", 0.0)
        per.append({"us": ns / 1e3, "mfma_i8": c.get("SQ_INSTS_VALU_MFMA_I8", 0.0), "ops": ops, "busy_cycles": busy,
                    "gui_active": gui, "tops": ops / ns / 1e3 if ns else 0.0})
    ops = sum(p["ops"] for p in per)
    ns = sum(p["us"] for p in per) * 1e3
    busy = sum(p["busy_cycles"] for p in per)
    gui = sum(p["gui_active"] for p in per)
    util = busy / (gui / XCDS * SIMDS) if gui else 0.0   # MFMA-busy share of SIMD cycles
    tops = ops / ns / 1e3 if ns else 0.0
    rec = {"kernel": "tile_exclusion_mfma", "symbol": kernel, "workload": a.workload, "seed": 1, "tile": a.tile,
           "reorder": a.reorder, "orient": a.orient, "dispatches": per, "mfma_util": util, "int8_tops": tops,
           "int8_peak_tops": INT8_PEAK_TOPS, "frac_of_peak": tops / INT8_PEAK_TOPS, "source_sha256": _sources_sha()}
    base = os.path.join(ROOT, "profiles", f"tile_exclusion_{a.workload}_mfma")
    with open(base + ".json", "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    lines = "\n".join(f"| {i + 1} | {p['us']:.1f} | {p['mfma_i8']:.0f} | {p['ops'] / 1e9:.2f} | {p['tops']:.1f} |"
                       for i, p in enumerate(per))
    md = f"""# {a.workload}: int8 matrix-core use of the tile exclusion kernel

Command (one counter pass, run from /tmp; REPO = the repository root, OUT = a directory for the output):

```
rocprofv3 --pmc SQ_VALU_MFMA_BUSY_CYCLES SQ_INSTS_VALU_MFMA_MOPS_I8 SQ_INSTS_VALU_MFMA_I8 SQ_INSTS_MFMA \\
    GRBM_GUI_ACTIVE --kernel-trace --output-format csv -d $OUT/pmc_mfma -o run -- \\
    python3 $REPO/paper_2605_29604_amd/profile_run.py
python3 paper_2605_29604_amd/profile_run.py --summarize-mfma $OUT/pmc_mfma
```

Each `v_mfma_i32_16x16x64_i8` is 32,768 integer operations (SQ_INSTS_VALU_MFMA_MOPS_I8 counts them / 512).

| Round | µs | MFMA i8 | G int ops | TOPS |
|---:|---:|---:|---:|---:|
{lines}

Over the solve: {tops:.1f} TOPS, {100 * tops / INT8_PEAK_TOPS:.2f}% of the {INT8_PEAK_TOPS:.0f} TOPS dense int8 peak;
MFMA busy {100 * util:.2f}% of SIMD cycles (busy cycles over GUI-active cycles per XCD x 1024 SIMDs).
The products are matrix-vector: the B operand repeats one candidate vector in all 16 columns, so 1/16 of
these operations is the algorithm's work.  The kernel is bound by memory latency and address processing,
not by the matrix cores.

`{os.path.basename(base)}.json` holds these figures with the SHA-256 of the kernel sources they were taken
on; `bench.py` reports them (`roofline.mfma`) only while those sources are unchanged.
"""
    with open(base + ".md", "w") as fh:
        fh.write(md)
    print(f"{base}.json: {tops:.1f} TOPS, util {100 * util:.2f}%")
    return 0


def summarize_stalls(a) -> int:
    """Where the exclusion kernel's waves spend their time: the share of wave cycles
    spent waiting (SQ_WAIT_ANY / SQ_WAVE_CYCLES) and the busy share of the texture
    address units (TA_BUSY_avr over the GUI-active cycles of one XCD)."""
    kernel = f"k_tile_excl<{a.tile}>"
    rows = _dispatches(a.summarize_stalls, kernel)
    if not rows:
        raise SystemExit(f"{a.summarize_stalls}: no {kernel} dispatch")
    per = []
    for ns, c in rows:
        wc, wait = c.get("SQ_WAVE_CYCLES", 0.0), c.get("SQ_WAIT_ANY", 0.0)
        gui, ta = c.get("GRBM_GUI_ACTIVE", 0.0), c.get("TA_BUSY_avr", 0.0)
        per.append({"us": ns / 1e3, "waves": c.get("SQ_WAVES", 0.0), "wait_share": wait / wc if wc else 0.0,
                    "ta_busy_share": ta / (gui / XCDS) if gui else 0.0, "wave_cycles": wc, "wait_any": wait,
                    "ta_busy_avr": ta, "gui_active": gui})
    tot_ns = sum(p["us"] for p in per)
    wait = sum(p["wait_any"] for p in per) / max(1.0, sum(p["wave_cycles"] for p in per))
    ta = sum(p["ta_busy_share"] * p["us"] for p in per) / tot_ns if tot_ns else 0.0
    base = os.path.join(ROOT, "profiles", f"tile_exclusion_{a.workload}_stalls")
    rec = {"kernel": "tile_exclusion_mfma", "symbol": kernel, "workload": a.workload, "seed": 1, "tile": a.tile,
           "reorder": a.reorder, "orient": a.orient, "dispatches": per, "wait_share": wait, "ta_busy_share": ta,
           "source_sha256": _sources_sha()}
    with open(base + ".json", "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    lines = "\n".join(f"| {i + 1} | {p['us']:.1f} | {p['waves']:.0f} | {100 * p['wait_share']:.1f}% | "
                       f"{100 * p['ta_busy_share']:.1f}% |" for i, p in enumerate(per))
    md = f"""# {a.workload}: what bounds the tile exclusion kernel

Command (one counter pass, run from /tmp; REPO = the repository root, OUT = a directory for the output):

```
rocprofv3 --pmc SQ_WAVES SQ_WAVE_CYCLES SQ_WAIT_ANY GRBM_GUI_ACTIVE TA_BUSY_avr --kernel-trace \\
    --output-format csv -d $OUT/pmc_stalls -o run -- python3 $REPO/paper_2605_29604_amd/profile_run.py
python3 paper_2605_29604_amd/profile_run.py --summarize-stalls $OUT/pmc_stalls
```

Wait share = SQ_WAIT_ANY / SQ_WAVE_CYCLES (wave cycles spent waiting, on memory almost entirely here);
TA busy = TA_BUSY_avr (busy cycles averaged over the texture address units) over the GUI-active cycles of
one XCD (GRBM_GUI_ACTIVE reads as the sum over the 8 XCDs).

| Round | µs | waves | wait share | TA busy |
|---:|---:|---:|---:|---:|
{{lines}}

Over the solve (time-weighted): waves wait {{100 * wait:.1f}}% of their cycles and the address units are busy
{{100 * ta:.1f}}% of the time.  The kernel reads 0.16 of the HBM roofline's bytes per second: it is bound by
the latency of its dependent gathers (chunk descriptor, column index, column state, bitmap) and by address
processing of the divergent column-state gathers (64 different lines per instruction), not by bandwidth.
"""
    md = md.replace("{lines}", lines).replace("{100 * wait:.1f}", f"{100 * wait:.1f}").replace(
        "{100 * ta:.1f}", f"{100 * ta:.1f}")
    with open(base + ".md", "w") as fh:
        fh.write(md)
    print(f"{base}.json: wait {100 * wait:.1f}%, TA busy {100 * ta:.1f}%")
    return 0


def summarize_build(a) -> int:
    """HBM bytes of every kernel of one build + solve (the same two counter runs as the
    exclusion kernel's traffic record), scaled like it, with each kernel's duration
    from the runs' kernel trace."""
    import re
    fdir, wdir = a.summarize_build
    cf, _ = _counter(fdir, "FETCH_SIZE", f"k_tile_excl<{a.tile}>")
    cw, _ = _counter(wdir, "WRITE_SIZE", f"k_tile_excl<{a.tile}>")
    copy_kib = a.copy_mib * 1024.0
    sf, sw = copy_kib / cf, copy_kib / cw

    def per_kernel(folder, counter):
        out = {}
        with open(os.path.join(folder, "run_counter_collection.csv")) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                m = re.search(r"(k_\w+(<[^>]*>)?)", r["Kernel_Name"])
                if not m:
                    continue
                ns = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
                out.setdefault(m.group(1), []).append((float(r["Counter_Value"]), ns))
        return out

    fk, wk = per_kernel(fdir, "FETCH_SIZE"), per_kernel(wdir, "WRITE_SIZE")
    rows = []
    for k, lst in fk.items():
        f_kib, ns = max(lst)                       # the tile path's largest dispatch
        w_kib = max(v for v, _ in wk.get(k, [(0.0, 0)]))
        mb = (f_kib * sf + w_kib * sw) * 1024 / 1e6
        rows.append((mb, k, f_kib * sf * 1024 / 1e6, w_kib * sw * 1024 / 1e6, ns / 1e3))
    rows.sort(reverse=True)
    lines = "\n".join(f"| `{k}` | {fm:.0f} | {wm:.0f} | {us:.0f} | {mb / us:.2f} |"
                       for mb, k, fm, wm, us in rows[:14] if us > 0)
    md = f"""# {a.workload}: HBM traffic of the build and solve kernels

From the same two counter passes as `tile_exclusion_{a.workload}_traffic.md` (REPO = the repository root,
OUT = a directory for the output; run from /tmp):

```
rocprofv3 --pmc FETCH_SIZE --kernel-trace --output-format csv -d $OUT/pmc_fetch -o run -- \\
    python3 $REPO/paper_2605_29604_amd/profile_run.py
rocprofv3 --pmc WRITE_SIZE --kernel-trace --output-format csv -d $OUT/pmc_write -o run -- \\
    python3 $REPO/paper_2605_29604_amd/profile_run.py
python3 paper_2605_29604_amd/profile_run.py --summarize-build $OUT/pmc_fetch $OUT/pmc_write
```

FETCH_SIZE scaled by {sf:.4f} and WRITE_SIZE by {sw:.4f} (a {a.copy_mib} MiB copy); for each kernel its largest
dispatch (the exclusion kernel: round 1), with that dispatch's duration under the counter pass.

| Kernel | fetched MB | written MB | µs | TB/s |
|---|---:|---:|---:|---:|
{{lines}}

`k_entries` moves about 5 GB (its 67 M random 4-byte new-id gathers each bring a 64-byte line) at close to
the 8 TB/s HBM peak: it is bound by the bytes those gathers move, 16 times the bytes they use.
"""
    md = md.replace("{lines}", lines)
    path = os.path.join(ROOT, "profiles", f"{a.workload}_build_traffic.md")
    with open(path, "w") as fh:
        fh.write(md)
    print(path)
    return 0


def summarize(a) -> int:
    kernel = f"k_tile_excl<{a.tile}>"
    fdir, wdir = a.summarize
    cf, fetch = _counter(fdir, "FETCH_SIZE", kernel)
    cw, write = _counter(wdir, "WRITE_SIZE", kernel)
    if len(fetch) != len(write):
        raise SystemExit("the two runs dispatched the kernel a different number of times")
    moved = a.copy_mib * 1024.0
    ff, wf = moved / cf, moved / cw
    per = [(f * ff + w * wf) * 1024.0 for f, w in zip(fetch, write)]
    # a random 4-byte gather: FETCH_SIZE bytes it reads beyond its index stream
    gk = _gather_fetch(fdir)
    gather = None
    if gk is not None:
        line = (gk * 1024.0 - a.gathers * 8 / ff) / a.gathers
        gather = {"gathers": a.gathers, "array_mib": a.gather_mib, "fetch_kib": gk,
                  "fetch_bytes_per_gather": line, "scaled_bytes_per_gather": line * ff}
    sha = _sources_sha()
    rec = {"kernel": "tile_exclusion_mfma", "symbol": kernel, "workload": a.workload, "seed": 1, "tile": a.tile,
           "reorder": a.reorder, "orient": a.orient, "dispatches": len(per), "fetch_kib": fetch, "write_kib": write,
           "copy_mib": a.copy_mib, "copy_fetch_kib": cf, "copy_write_kib": cw, "fetch_factor": ff,
           "write_factor": wf, "traffic_bytes_per_dispatch": per, "traffic_bytes_per_launch": sum(per) / len(per),
           "source_sha256": sha}
    base = os.path.join(ROOT, "profiles", f"tile_exclusion_{a.workload}_traffic")
    with open(base + ".json", "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    rows = "\n".join(f"| {i + 1} | {f:.1f} | {w:.1f} | {b / 1e6:.1f} MB |"
                     for i, (f, w, b) in enumerate(zip(fetch, write, per)))
    md = f"""# {a.workload}: HBM traffic of the tile exclusion kernel (FETCH_SIZE / WRITE_SIZE)

Commands (two passes, one counter each, run from /tmp; REPO = the repository root, OUT = a directory for
the output):

```
rocprofv3 --pmc FETCH_SIZE --kernel-trace --output-format csv -d $OUT/pmc_fetch -o run -- \\
    python3 $REPO/paper_2605_29604_amd/profile_run.py
rocprofv3 --pmc WRITE_SIZE --kernel-trace --output-format csv -d $OUT/pmc_write -o run -- \\
    python3 $REPO/paper_2605_29604_amd/profile_run.py
python3 paper_2605_29604_amd/profile_run.py --summarize $OUT/pmc_fetch $OUT/pmc_write
```

`profile_run.py` copies {a.copy_mib} MiB device to device, then builds and solves {a.workload} on the tile path
(T={a.tile}, {a.reorder} order, orient={a.orient}, direct launches) and on the CSR path.

Calibration (the {a.copy_mib} MiB copy): FETCH_SIZE reads {cf:.1f} KiB, WRITE_SIZE {cw:.1f} KiB for {moved:.0f} KiB
moved each way, so FETCH_SIZE is scaled by {ff:.4f} and WRITE_SIZE by {wf:.4f}.

| Round | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes (scaled) |
|---:|---:|---:|---:|
{rows}

Average per launch: {sum(per) / len(per) / 1e6:.2f} MB.

`{os.path.basename(base)}.json` holds these figures with the SHA-256 of the kernel sources they were taken on;
`bench.py` reports `roofline.traffic` only while those sources are unchanged.
"""
    with open(base + ".md", "w") as fh:
        fh.write(md)
    print(f"{base}.json: {len(per)} launches, {sum(per) / len(per) / 1e6:.2f} MB per launch")
    return 0


# the hybrid path's kernels with a traffic record: record name -> (kernel symbol, sources)
HYBRID_KERNELS = {
    "hybrid_candidate": ("k_hyb_p1", ("hyb.hip", "round.hpp", "graph.hpp")),
    "hybrid_exclusion": ("k_hyb_p2", ("hyb.hip", "round.hpp", "graph.hpp")),
    "hybrid_dense_build": ("k_dense_build", ("hyb.hip", "graph.hpp")),
}


def summarize_kernel(a) -> int:
    """Per-launch HBM traffic of one hybrid-path kernel (all its dispatches in one
    build + solve of profile_run.py --path hybrid), FETCH_SIZE and WRITE_SIZE each
    scaled by what the counter reads for the copy of known size."""
    record, fdir, wdir = a.summarize_kernel
    symbol, sources = HYBRID_KERNELS[record]
    cf, fetch = _counter(fdir, "FETCH_SIZE", symbol)
    cw, write = _counter(wdir, "WRITE_SIZE", symbol)
    if len(fetch) != len(write):
        raise SystemExit("the two runs dispatched the kernel a different number of times")
    moved = a.copy_mib * 1024.0
    ff, wf = moved / cf, moved / cw
    per = [(f * ff + w * wf) * 1024.0 for f, w in zip(fetch, write)]
    # a random 4-byte gather: FETCH_SIZE bytes it reads beyond its index stream
    gk = _gather_fetch(fdir)
    gather = None
    if gk is not None:
        line = (gk * 1024.0 - a.gathers * 8 / ff) / a.gathers
        gather = {"gathers": a.gathers, "array_mib": a.gather_mib, "fetch_kib": gk,
                  "fetch_bytes_per_gather": line, "scaled_bytes_per_gather": line * ff}
    sha = {}
    for name in sources:
        with open(os.path.join(ROOT, "paper_2605_29604_amd", "csrc", name), "rb") as fh:
            sha[name] = hashlib.sha256(fh.read()).hexdigest()
    rec = {"kernel": record, "symbol": symbol, "workload": a.workload, "seed": 1, "dense_min": a.dense_min,
           "dispatches": len(per), "fetch_kib": fetch, "write_kib": write, "copy_mib": a.copy_mib,
           "copy_fetch_kib": cf, "copy_write_kib": cw, "fetch_factor": ff, "write_factor": wf,
           "traffic_bytes_per_dispatch": per, "traffic_bytes_per_launch": sum(per) / len(per),
           "gather_calibration": gather, "source_sha256": sha}
    base = os.path.join(ROOT, "profiles", f"{record}_{a.workload}_traffic")
    with open(base + ".json", "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    rows = "\n".join(f"| {i + 1} | {f:.1f} | {w:.1f} | {b / 1e6:.2f} MB |"
                     for i, (f, w, b) in enumerate(zip(fetch, write, per)))
    gtext = ""
    if gather is not None:
        gtext = (f"\n\nGather calibration: {a.gathers} random 4-byte reads from a {a.gather_mib} MiB array (far larger "
                 f"than the\nInfinity Cache) read {gather['fetch_bytes_per_gather']:.1f} bytes of FETCH_SIZE each beyond "
                 f"their index stream\n({gather['scaled_bytes_per_gather']:.1f} bytes after the copy's factor): what one "
                 f"isolated gather that misses every cache costs\nin these counters.")
    md = f"""# {a.workload}: HBM traffic of `{symbol}` (FETCH_SIZE / WRITE_SIZE)

Commands (two passes, one counter each, run from /tmp; REPO = the repository root, OUT = a directory for
the output):

```
rocprofv3 --pmc FETCH_SIZE --kernel-trace --output-format csv -d $OUT/pmc_fetch -o run -- \\
    python3 $REPO/paper_2605_29604_amd/profile_run.py --path hybrid
rocprofv3 --pmc WRITE_SIZE --kernel-trace --output-format csv -d $OUT/pmc_write -o run -- \\
    python3 $REPO/paper_2605_29604_amd/profile_run.py --path hybrid
python3 paper_2605_29604_amd/profile_run.py --summarize-kernel {record} $OUT/pmc_fetch $OUT/pmc_write
```

`profile_run.py --path hybrid` copies {a.copy_mib} MiB device to device, then builds and solves {a.workload} on the
hybrid path (default dense-block threshold, direct launches).

Calibration (the {a.copy_mib} MiB copy): FETCH_SIZE reads {cf:.1f} KiB, WRITE_SIZE {cw:.1f} KiB for {moved:.0f} KiB
moved each way, so FETCH_SIZE is scaled by {ff:.4f} and WRITE_SIZE by {wf:.4f}.

| Dispatch | FETCH_SIZE KiB | WRITE_SIZE KiB | bytes (scaled) |
|---:|---:|---:|---:|
{rows}

Average per launch: {sum(per) / len(per) / 1e6:.2f} MB.  These counters count lines moved between the L2
and the memory fabric, which includes hits in the 256 MB Infinity Cache, so they bound HBM traffic from
above.{gtext}  `{os.path.basename(base)}.json` holds the figures with the SHA-256 of the kernel's sources;
`bench.py` reports them (`roofline.traffic`) only while those sources are unchanged.
"""
    with open(base + ".md", "w") as fh:
        fh.write(md)
    print(f"{base}.json: {len(per)} launches, {sum(per) / len(per) / 1e6:.2f} MB per launch")
    return 0


def _short(name: str) -> str:
    name = name.replace("tcmis::(anonymous namespace)::", "").replace("void ", "")
    return name.split("(")[0]


def summarize_stats(a) -> int:
    """Kernel statistics of one `rocprofv3 --kernel-trace --stats` run of bench.py (the
    hybrid path's default workload): the per-kernel table, one build + solve step from
    the trace, and the roofline kernel's average launch from the trace beside the one
    bench.py measured with HIP events in the same command (its JSON line)."""
    folder, name, bench_json = a.summarize_stats
    with open(os.path.join(folder, "run_kernel_stats.csv")) as fh:
        stats = list(csv.DictReader(fh))
    with open(os.path.join(folder, "run_kernel_trace.csv")) as fh:
        trace = sorted(csv.DictReader(fh), key=lambda r: int(r["Start_Timestamp"]))
    bench = {}
    with open(bench_json) as fh:
        for line in fh:
            if line.startswith("{"):
                bench = json.loads(line)
    rows = "\n".join(f"| `{_short(r['Name'])}` | {int(r['Calls'])} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['Percentage']):.2f} |" for r in stats[:40])
    # one step: from the second k_keys launch to the first report copy after it
    keys = [i for i, r in enumerate(trace) if _short(r["Kernel_Name"]) == "k_keys"]
    step = []
    if len(keys) > 1:
        for r in trace[keys[1]:]:
            step.append(r)
            if "copyBuffer" in r["Kernel_Name"] and len(step) > 1:
                break
    t0 = int(step[0]["Start_Timestamp"]) if step else 0
    t1 = int(step[-1]["End_Timestamp"]) if step else 0
    busy = sum(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in step)
    srows = "\n".join(f"| `{_short(r['Kernel_Name'])}` | {int(r['Grid_Size_X'])} | "
                      f"{(int(r['End_Timestamp']) - int(r['Start_Timestamp'])) / 1e3:.1f} |" for r in step)
    roof = bench.get("roofline", {})
    sym = {"hybrid_candidate": "k_hyb_p1", "hybrid_exclusion": "k_hyb_p2", "hybrid_dense_build": "k_dense_build"}
    k = roof.get("kernel", "")
    durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in trace
            if k in sym and _short(r["Kernel_Name"]).startswith(sym[k])]
    cmp_line = ""
    if durs:
        cmp_line = (f"The roofline kernel `{k}` (`{sym[k]}`, every round): {len(durs)} launches in the trace, "
                    f"{sum(durs) / len(durs):.1f} µs on average; bench.py's HIP-event figure in the same "
                    f"command (one timed solve, {roof.get('launches')} launches): {roof.get('avg_launch_us')} µs.")
    md = f"""# {bench.get('config', {}).get('workload', a.workload)}: kernel statistics of the benchmark run (hybrid path)

Command (run from /tmp; REPO = the repository root, OUT = a directory for the output):

```
rocprofv3 --kernel-trace --stats --output-format csv -d $OUT/stats -o run -- \\
    python3 $REPO/bench.py --steps 3 --warmup 1 --no-cpu --no-batch --no-serve --no-tune \\
        --no-configs --no-dynamic > $OUT/bench.json
python3 paper_2605_29604_amd/profile_run.py --summarize-stats $OUT/stats {name} $OUT/bench.json
```

The run times build + solve steps of the hybrid path, solve-only repeats, one solve with per-kernel HIP
events, the all-tile and CSR paths the same way, and the three launch modes, so call counts are multiples
of the repeats.  Durations from the kernel trace; the benchmark's own line (step {bench.get('ms_per_step')} ms
under the profiler) is measured again without it at the end of every round.

| Kernel | Calls | Avg µs | Total ms | % |
|---|---:|---:|---:|---:|
{rows}

{cmp_line}

## One build + solve step from the trace

The second hybrid build + solve of the trace, from `k_keys` to the solve's report copy: {len(step)}
launches, {busy / 1e3:.1f} µs of kernel time in a span of {(t1 - t0) / 1e3:.1f} µs.

| Kernel | Grid (threads) | µs |
|---|---:|---:|
{srows}
"""
    out = os.path.join(ROOT, "profiles", f"{name}.md")
    with open(out, "w") as fh:
        fh.write(md)
    print(out)
    return 0


def main() -> int:
    p = argparse.ArgumentParser()
    p.add_argument("--workload", default="rmat22")
    p.add_argument("--tile", type=int, default=16)
    p.add_argument("--reorder", default="key")
    p.add_argument("--orient", type=int, default=1)
    p.add_argument("--copy-mib", type=int, default=256)
    p.add_argument("--gather-mib", type=int, default=2048)
    p.add_argument("--gathers", type=int, default=1 << 22)
    p.add_argument("--summarize", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    p.add_argument("--summarize-mfma", metavar="DIR")
    p.add_argument("--summarize-stalls", metavar="DIR")
    p.add_argument("--summarize-build", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    p.add_argument("--summarize-kernel", nargs=3, metavar=("RECORD", "FETCH_DIR", "WRITE_DIR"))
    p.add_argument("--summarize-stats", nargs=3, metavar=("DIR", "NAME", "BENCH_JSON"))
    p.add_argument("--path", default="tile", choices=("tile", "hybrid"))
    p.add_argument("--dense-min", type=int, default=0)
    a = p.parse_args()
    if a.summarize_kernel:
        return summarize_kernel(a)
    if a.summarize_stats:
        return summarize_stats(a)
    if a.summarize:
        return summarize(a)
    if a.summarize_mfma:
        return summarize_mfma(a)
    if a.summarize_stalls:
        return summarize_stalls(a)
    if a.summarize_build:
        return summarize_build(a)
    import torch
    from paper_2605_29604_amd import gen, tcmis

    tcmis.lib()
    g = gen.workload(a.workload, seed=1)
    rp = torch.from_numpy(g.row_ptr).cuda()
    ci = torch.from_numpy(g.col_idx).cuda()
    src = torch.ones(a.copy_mib << 20, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    print(f"copy {a.copy_mib} MiB", flush=True)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    if a.gather_mib > 0:   # random 4-byte gathers of known count from a large array
        big = torch.zeros(a.gather_mib << 18, dtype=torch.int32, device="cuda")
        gen_ = torch.Generator(device="cuda")
        gen_.manual_seed(1)
        idx = torch.randint(0, big.numel(), (a.gathers,), device="cuda", generator=gen_)
        torch.cuda.synchronize()
        print(f"gather {a.gathers} x 4 B from {a.gather_mib} MiB", flush=True)
        picked = big[idx]
        torch.cuda.synchronize()
        del big, idx, picked
    if a.path == "hybrid":
        print("hybrid build + solve", flush=True)
        h = tcmis.mis_build_tiles(rp, ci, path="hybrid", dense_min=a.dense_min, seed=1, launch="direct")
    else:
        print("tile build + solve", flush=True)
        h = tcmis.mis_build_tiles(rp, ci, path="tile", tile=a.tile, reorder=a.reorder, orient=a.orient, seed=1,
                                  launch="direct")
    out, st = tcmis.mis_solve(h, trace_cap=0)
    torch.cuda.synchronize()
    tcmis.mis_free_tiles(h)
    print("csr build + solve", flush=True)
    h = tcmis.mis_build_tiles(rp, ci, path="csr", seed=1, launch="direct")
    out2, st2 = tcmis.mis_solve(h, trace_cap=0)
    torch.cuda.synchronize()
    tcmis.mis_free_tiles(h)
    same = bool(torch.equal(out, out2))
    print(f"rounds {st['rounds']} set {st['n_in']} {a.path}==csr {same}", flush=True)
    return 0 if same else 1


if __name__ == "__main__":
    sys.exit(main())
