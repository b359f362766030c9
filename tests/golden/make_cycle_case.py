"""Writes cycle_case.json: small instances on which the GDP rule (the damped
midpoint reading of eq. 10, Jacobi over all nodes) enters a 2-cycle,
Lam_k = Lam_{k-2}, so that the loop stops with "cycle".  The search is
deterministic (numpy PCG64, seed 0) and calls only the oracle; the stored
expectations (stop iteration, k*) are the oracle's and are re-derived
independently by tests/test_oracle_pins.py.

    python tests/golden/make_cycle_case.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import core  # noqa: E402


def search(want=3, tries=40000):
    rng = np.random.default_rng(0)
    cases = []
    for t in range(tries):
        n = int(rng.integers(4, 9))
        side = int(rng.choice([10, 30, 100, 1000]))
        xy = rng.integers(0, side, (n, 2)).astype(np.int32)
        lam0 = rng.integers(-4 * side, 4 * side, n).astype(np.int64)
        o = core.gdp_solve(xy, lam0=lam0, max_iters=200, handoff_div=0)
        # keep cycles whose k* lies before the cycle's own iterates, so that
        # the best-dual choice of Lam* is exercised
        if o["stop"] == "cycle" and o["kstar"] < o["iters"] - 3:
            cases.append({"coords": xy.tolist(), "lam0": lam0.tolist(), "stop_k": int(o["iters"] - 1),
                          "kstar": int(o["kstar"]), "try": t})
            if len(cases) == want:
                break
    return cases


if __name__ == "__main__":
    cases = search()
    out = {"_about": "GDP 2-cycles found by make_cycle_case.py (oracle only): the loop evaluates "
                     "Lam_0 = lam0, ..., Lam_stop_k and stops there with Lam_stop_k = Lam_{stop_k-2}; "
                     "k* is the first iterate of largest dual bound.",
           "cases": cases}
    with open(os.path.join(HERE, "cycle_case.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("wrote %d cases" % len(cases))
