"""Writes heuristic_quality.json: the quality study of the priority heuristics of
Section 3.3 on the three single-graph workloads, computed by the oracle only (the
synthetic analogue of the paper's MIS-cardinality comparison; no GPU involved).

For each workload (er10k, rmat22, grid256; graph seed 1) and each key rule
(degree = floor(255 / (1 + deg)), hash = H1, eq1 = Eq. 1 discretised; key seed 1):
the size of the set the round-synchronous rule computes (equal, by the greedy
identity, to the greedy pass in decreasing key order, which is what runs here) and
its number of rounds, against the sequential min-degree greedy heuristic (take a
vertex of least remaining degree, remove it and its neighbours, repeat).

Run from the repository root: python tests/golden/make_heuristic_quality.py
(a few minutes on one core).
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2605_29604_amd import gen  # noqa: E402

WORKLOADS = ["er10k", "rmat22", "grid256"]
RULES = ["degree", "hash", "eq1"]


def study(name):
    g = gen.workload(name, seed=1)
    md = int(oracle.mindeg_greedy(g.row_ptr, g.col_idx).sum())
    row = {"n": int(g.n), "edges": int(g.m), "mindeg_greedy_size": md, "rules": {}}
    for rule in RULES:
        k = oracle.keys_rule(g.row_ptr, 1, rule)
        st, rounds, _ = oracle.roundsync(g.row_ptr, g.col_idx, k)
        size = int((st == oracle.IN).sum())
        row["rules"][rule] = {"size": size, "rounds": int(rounds), "ratio_to_mindeg": round(size / md, 5)}
    return row


def main():
    rec = {"graph_seed": 1, "key_seed": 1, "workloads": {}}
    for name in WORKLOADS:
        rec["workloads"][name] = study(name)
        print(name, rec["workloads"][name], flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "heuristic_quality.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
