"""Writes rmat22_quality.json: MIS sizes of the R-MAT scale-22 benchmark graph (seed 1)
under two sequential references, computed by the oracle only.

  mindeg_greedy_size  the min-degree greedy heuristic (take a vertex of least remaining
                      degree, remove it and its neighbours, repeat)
  key_greedy_size     the greedy pass in decreasing default-key order, which the
                      round-synchronous rule with the same fixed keys reproduces exactly

The benchmark reports its set size against the first.  Run from the repository
root: python tests/golden/make_quality.py  (about a minute on one core).
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2605_29604_amd import gen  # noqa: E402


def main():
    g = gen.workload("rmat22", seed=1)
    md = oracle.mindeg_greedy(g.row_ptr, g.col_idx)
    kg = oracle.greedy(g.row_ptr, g.col_idx, oracle.keys(g.row_ptr, 1))
    rec = {"workload": "rmat22", "graph_seed": 1, "key_seed": 1, "n": int(g.n), "edges": int(g.m),
           "mindeg_greedy_size": int(md.sum()), "key_greedy_size": int(kg.sum())}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "rmat22_quality.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(rec)


if __name__ == "__main__":
    main()
