"""A short program for counter runs under rocprofv3: one tile-path build and solve
of a named workload (the CSR resident on the device), one CSR-path solve, and one
device-to-device copy of a known size, whose FETCH_SIZE / WRITE_SIZE calibrate the
counters against bytes actually moved.

    python paper_2605_29604_amd/profile_run.py [--workload rmat22] [--copy-mib 256]
"""
from __future__ import annotations

import argparse
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def main() -> int:
    p = argparse.ArgumentParser()
    p.add_argument("--workload", default="rmat22")
    p.add_argument("--tile", type=int, default=16)
    p.add_argument("--reorder", default="key")
    p.add_argument("--orient", type=int, default=1)
    p.add_argument("--copy-mib", type=int, default=256)
    a = p.parse_args()
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
    print(f"rounds {st['rounds']} set {st['n_in']} tile==csr {same}", flush=True)
    return 0 if same else 1


if __name__ == "__main__":
    sys.exit(main())
