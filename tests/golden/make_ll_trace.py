"""Writes tests/golden/ll_trace.json: the FP64 oracle's training
log-likelihood every `every` iterations of the whole run of the paper-shaped
synthetic workloads -- the mixing indicator the paper plots for its
synthetic experiments (Section 4.2.1, the log-likelihood of the chain's
state against time).

Only the oracle and the seeded input generators are used, so the stored
values come from the oracle alone.

Usage: python tests/golden/make_ll_trace.py NAME [NAME ...]
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

OUT = os.path.join(HERE, "ll_trace.json")
EVERY = 100


def oracle_trace(name: str) -> dict:
    wl = workloads.by_name(name)
    cfg = oracle.Config(**wl.fit_kwargs())
    ch = oracle.Chain(cfg, wl.row, wl.col, wl.val, wl.W0, wl.H0)
    t0 = time.time()
    points = [[0, ch.loglik()]]
    while ch.t < wl.T:
        ch.run(min(EVERY, wl.T - ch.t))
        points.append([int(ch.t), ch.loglik()])
        if ch.t % 1000 == 0:
            print(f"[golden] {name}: {ch.t}/{wl.T}, {time.time() - t0:.0f} s", file=sys.stderr, flush=True)
    return {"T": wl.T, "every": EVERY, "nnz": wl.nnz, "points": points,
            "oracle_threads": oracle.threads(), "oracle_seconds": round(time.time() - t0, 1)}


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in names:
        data[name] = oracle_trace(name)
        with open(OUT + ".tmp", "w") as f:
            json.dump(data, f, indent=0, sort_keys=True)
            f.write("\n")
        os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main(sys.argv[1:])
