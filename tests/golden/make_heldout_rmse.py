"""Writes tests/golden/heldout_rmse.json: the FP64 oracle's held-out RMSE of
the posterior-mean predictor after the full run of each named workload.

The predictor is the average of mu_ij over the post-burn-in iterations whose
part contains the cell's block (Monte Carlo averages after burn-in,
Section 4.2.2); the RMSE is unclipped.  Only the oracle and the seeded input
generators are used, so the stored values come from the oracle alone.  The
oracle's results do not depend on its thread count.

Usage: python tests/golden/make_heldout_rmse.py NAME [NAME ...]
(updates the entries for the given workloads, keeps the others).
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

OUT = os.path.join(HERE, "heldout_rmse.json")


def oracle_rmse(name: str) -> dict:
    t0 = time.time()
    wl = workloads.by_name(name)
    t_gen = time.time() - t0
    cfg = oracle.Config(**wl.fit_kwargs())
    ch = oracle.Chain(cfg, wl.row, wl.col, wl.val, wl.W0, wl.H0, wl.hrow, wl.hcol)
    t1 = time.time()
    done = 0
    while done < wl.T:
        n = min(100, wl.T - done)
        ch.run(n)
        done += n
        print(f"[golden] {name}: {done}/{wl.T} iterations, {time.time() - t1:.0f} s", file=sys.stderr, flush=True)
    rmse = ch.heldout_rmse(wl.hval)
    return {"T": wl.T, "burn_in": wl.burn_in, "thin": wl.thin, "n_heldout": int(len(wl.hval)),
            "heldout_rmse": rmse, "train_loglik_end": ch.loglik(), "n_kept": int(ch.n_kept),
            "oracle_threads": oracle.threads(), "oracle_seconds": round(time.time() - t1, 1),
            "generate_seconds": round(t_gen, 1)}


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in names:
        data[name] = oracle_rmse(name)
        print(f"[golden] {name}: RMSE {data[name]['heldout_rmse']:.6f}", file=sys.stderr, flush=True)
        with open(OUT + ".tmp", "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
            f.write("\n")
        os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main(sys.argv[1:])
