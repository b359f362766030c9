#!/usr/bin/env python3
"""Benchmark of libf2m on one MI355X: time to a certified F2M optimum (the
headline value, seconds) and the scan's pair-evaluation rates on the complete
graph of n = 100,000 cities with integer coordinates uniform in [0, 10^6)^2
(seeded, synthetic).

One step = one full solve on the GPU: the GDP loop (scan, selection, degree
counts, Lam update, device-side stop test), the exact finish when the
trivial x does not certify, and the certificate.  Coordinates are resident
in HBM before the timed region starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "time-to-certified F2M optimum (s) + pair-evals/s at n=100k; warm vs cold"
# gfx950 VALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one 32-bit op per
# lane per clock without packed math
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# algorithmic work per ordered pair the scan tests: two coordinate
# differences, two products (or FMAs), the bound's add and multiply and one
# compare -- 7 VALU lane-ops
OPS_PER_PAIR = 7.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic(key):
    """HBM bytes per launch from the committed rocprofv3 counters
    (profiles/traffic.json), or None when the kernel source has changed
    since they were taken or the workload differs."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    try:
        with open(os.path.join(here, "profiles", "traffic.json")) as f:
            t = json.load(f)
        with open(os.path.join(here, t["source"]), "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError, KeyError):
        return None
    if sha != t.get("sha256"):
        return None
    return t.get("bytes_per_launch", {}).get(key)


def cpu_baseline(xy, lam, budget_s, iterations):
    """The oracle's plain per-row GDP pass on a sample of rows of the same
    instance at the GPU's final Lam, scaled to the seconds of the GDP
    iterations the GPU ran (the oracle's time for the GDP part of the
    time to a certified optimum)."""
    from oracle import core
    n = len(xy)
    rng = np.random.default_rng(0)
    rows = rng.permutation(n)
    done, t_used, take = 0, 0.0, 16
    while t_used < budget_s and done < n:
        chunk = rows[done:done + take]
        t0 = time.perf_counter()
        core.gdp_rows(xy, lam, chunk)
        t_used += time.perf_counter() - t0
        done += len(chunk)
        rate = done / max(t_used, 1e-9)
        take = int(min(max(16, rate * (budget_s - t_used) * 0.9), n - done)) if t_used < budget_s else 0
        if take <= 0:
            break
    per_iter_s = t_used * n / done
    pairs = n * (n - 1) / 2
    return {"value": per_iter_s * iterations, "unit": "s", "cores": core.num_threads(),
            "kind": "oracle", "cpu": cpu_model(),
            "pair_evals_per_s": pairs / per_iter_s,
            "sample": "%d of %d rows of one GDP iteration (each row evaluates all n-1 columns), %.1f s, "
                      "scaled to %d full iterations (the GPU's count); the exact finish is not included "
                      "(the oracle's min-cost flow is dense)" % (done, n, t_used, iterations)}


def subtour_leg(ctx, f2m, xy_dev, cold, args):
    """F2M plus subtour-elimination rows (the extension of Sec. 5) from the
    certified F2M optimum of the cold solve: one separation (components of
    its trivial x), then the GDP with those rows for --sec-iters iterations
    (one untimed run, then `steps` timed runs from the same start)."""
    import torch
    n = xy_dev.shape[0]
    lam0 = torch.from_numpy(np.asarray(cold["lambda2"], np.int64)).cuda()
    new_row = torch.empty(n, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rows, comps = ctx.sec_separate(xy_dev, None, 0, lam0, None, new_row)
    torch.cuda.synchronize()
    sep_s = time.perf_counter() - t0
    if rows == 0:
        return {"rows": 0, "components": comps, "note": "the F2M optimum is connected: no subtour row"}
    row_of = new_row.reshape(1, n)
    times, g = [], None
    for i in range(1 + max(1, args.steps)):
        lam = lam0.clone()
        mu = torch.zeros(rows, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = ctx.sec_gdp(xy_dev, row_of, rows, lam, mu, max_iters=args.sec_iters, trace=False)
        torch.cuda.synchronize()
        if i > 0:
            times.append(time.perf_counter() - t0)
        log("subtour GDP run %d: %d iterations, %.3f s" % (i, g["iterations"], time.perf_counter() - t0))
    it = g["iterations"]
    per = float(np.mean(times)) / it
    tested = g["pairs_tested"] / it
    return {"workload": "F2M + subtour rows from the F2M optimum of the same instance: one separation, "
                        "then the GDP with those rows, %d iterations at most" % args.sec_iters,
            "rows": rows, "components": comps, "separation_s": sep_s, "iterations": it, "stop": g["stop"],
            "seconds": float(np.mean(times)), "ms_per_iteration": 1e3 * per,
            "dual2_f2m": cold["dual2"], "dual2": g["dual2"], "bound_gain": g["dual2"] / cold["dual2"] - 1.0,
            "pairs_tested_per_iteration": tested, "pairs_tested_frac": tested / (n * (n - 1.0)),
            "scan_lane_ops_per_s_over_iteration": OPS_PER_PAIR * tested / per,
            "note": "the rate divides the scan's algorithmic lane-ops by the whole iteration (scan, node and "
                    "row steps, control): a lower bound of the scan's own; profiles/ holds its kernel times"}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _figures(r):
    """A solve's result without its arrays (scalars and small dicts only)."""
    return {k: v for k, v in r.items() if not isinstance(v, np.ndarray) and v is not None}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=100000)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--instance", choices=("uniform", "clustered"), default="uniform",
                    help="uniform: integer coordinates uniform in [0,10^6)^2; clustered: 200 Gaussian centres, "
                         "sigma 2%% of the side")
    ap.add_argument("--graph", choices=("complete", "knn"), default="complete",
                    help="complete graph, or the 10-nearest-neighbour candidate graph")
    ap.add_argument("--scan", choices=("culled", "full"), default="culled",
                    help="culled: skip column tiles that provably hold no relevant pair (default); "
                         "full: test every ordered pair")
    ap.add_argument("--start", choices=("both", "cold"), default="both",
                    help="both: time the cold start, then the learned warm start (when trained weights exist) and "
                         "the candidate-graph warm start")
    ap.add_argument("--sec-iters", type=int, default=400,
                    help="iterations of the subtour-row GDP leg (0: skip the leg)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a device copy of known size (for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the solver runs on a single MI355X and has no "
              "multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        a = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": a.numel(), "copies": 3}))
        return

    from paper_2011_08170_amd import f2m, instances

    n = args.n
    if args.instance == "uniform":
        xy = instances.uniform(n, 1_000_000, args.seed)
    else:
        xy = instances.clustered(n, 1_000_000, args.seed)
    ctx = f2m.Context(0)
    xy_dev = torch.from_numpy(xy).cuda()
    torch.cuda.synchronize()
    log("workload: n=%d %s [0,1e6)^2 seed=%d graph=%s; warmup %d, steps %d" % (
        n, args.instance, args.seed, args.graph, args.warmup, args.steps))

    theta = None
    if args.start == "both":
        from paper_2011_08170_amd import warm
        if os.path.exists(warm.DEFAULT_WEIGHTS):
            theta = warm.load()
        else:
            log("no trained warm-start weights at %s: cold start only" % warm.DEFAULT_WEIGHTS)

    def leg(name, kw):
        """Warm-up solves, then `steps` timed solves without kernel events
        (the value: HIP event records between launches stall the queue for a
        few microseconds each), then `steps` solves with HIP events around
        every scan and update launch (the roofline's launch durations)."""
        for i in range(args.warmup):
            r = ctx.solve(xy_dev, scan=args.scan, graph=args.graph, **kw)
            log("%s warmup %d: %s, %d iterations, %.3f s" % (name, i, r["status"], r["iterations"],
                                                             r["seconds"]["total"]))
        runs = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            # every solve returns its whole result in host memory; like a
            # caller that is done with one result before the next solve, the
            # bench keeps the arrays of the last solve only
            r = ctx.solve(xy_dev, scan=args.scan, graph=args.graph, **kw)
            runs.append(r if i == args.steps - 1 else _figures(r))
            del r
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        for i, r in enumerate(runs):
            log("%s step %d: %s stop=%s iterations=%d total=%.3f s (warm %.3f, gdp %.3f, finish %.3f, "
                "certify %.3f)" % (name, i, r["status"], r["stop"], r["iterations"], r["seconds"]["total"],
                                   r["seconds"]["warm"], r["seconds"]["gdp"], r["seconds"]["finish"],
                                   r["seconds"]["certify"]))
        timed = []
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for i in range(args.steps):
            r = ctx.solve(xy_dev, time_kernels=True, scan=args.scan, graph=args.graph, **kw)
            timed.append(r if i == args.steps - 1 else _figures(r))
            del r
        torch.cuda.synchronize()
        log("%s: %d solves with kernel events in %.3f s" % (name, args.steps, time.perf_counter() - t1))
        return runs, elapsed, timed

    def summary(plain, elapsed, runs):
        """plain: the timed solves (value, phases); runs: the same solves
        with kernel events (launch durations, roofline)."""
        pairs = n * (n - 1) / 2
        iters = sum(r["iterations"] for r in runs)
        scan_ms = sum(r["scan_ms"] for r in runs)
        launches = sum(r["scan_launches"] for r in runs)
        avg_ms = scan_ms / max(launches, 1)
        rates = None
        if args.graph == "complete":
            # ordered pairs the scan kernel evaluated per launch (culled tiles
            # excluded; a list iteration's entries are evaluated by the update,
            # its scan launch exits at once and counts as a launch with none)
            tested_all = sum(r["scan_pairs"] for r in runs)
            tested = sum(r["scan_by_kind"][k]["pairs"] for r in runs for k in ("full", "build")) / max(launches, 1)
            ops = OPS_PER_PAIR * tested
            achieved = ops / (avg_ms * 1e-3) / 1e12
            kern = ("k_rowscan_w<gdp>" if args.scan == "culled" and runs[-1]["scan_rows"] == 1
                    else "k_rowscan<%d,gdp>" % runs[-1]["scan_rows"])
            by_kind = {}
            for kind in ("full", "build", "list"):
                ms = sum(r["scan_by_kind"][kind]["ms"] for r in runs)
                mu = sum(r["scan_by_kind"][kind]["update_ms"] for r in runs)
                nl = sum(r["scan_by_kind"][kind]["launches"] for r in runs)
                pk = sum(r["scan_by_kind"][kind]["pairs"] for r in runs)
                if nl:
                    # a list iteration's pairs are evaluated by the update
                    # (its scan launch exits at once): rate over the update
                    t = mu if kind == "list" else ms
                    a = OPS_PER_PAIR * pk / nl / (t / nl * 1e-3) / 1e12
                    by_kind[kind] = {"launches": nl, "avg_launch_ms": ms / nl, "avg_update_ms": mu / nl,
                                     "pairs_tested_per_launch": pk / nl, "achieved": a, "frac": a / VALU_PEAK_TOPS,
                                     "rate_over": "update" if kind == "list" else "scan"}
            roof = {"bound": "alu", "kernel": kern, "achieved": achieved,
                    "peak": VALU_PEAK_TOPS, "unit": "T lane-op/s", "frac": achieved / VALU_PEAK_TOPS,
                    "ops_per_pair": OPS_PER_PAIR,
                    "traffic": measured_traffic("complete|%s|%s|%d" % (args.scan, args.instance, n)),
                    "avg_launch_ms": avg_ms, "launches": launches,
                    "pairs_tested_per_launch": tested, "ops_per_launch": ops,
                    "slices": runs[-1]["scan_slices"], "by_kind": by_kind,
                    "update_avg_ms": sum(r["update_ms"] for r in runs) / max(launches, 1),
                    "valu_counter": measured_traffic("valu|complete|%s|%s|%d" % (args.scan, args.instance, n))}
            gdp_ms = scan_ms + sum(r["update_ms"] for r in runs)
            rates = {"tested_pairs_per_s": tested_all / (gdp_ms * 1e-3) if gdp_ms else None,
                     "decided_pairs_per_s": iters * pairs / (gdp_ms * 1e-3) if gdp_ms else None,
                     "note": "tested: ordered pairs the GDP kernels evaluated (the scan's filter, or the "
                             "candidate lists in the update); decided: the n(n-1)/2 unordered pairs each "
                             "iteration settles; both over the scan and update kernels' time"}
        else:
            nnz = runs[-1]["graph_nnz"]
            # per row: rowptr 4, own label 4, Lam in 8, Lam out 8, top-4 Z 32 and labels 16;
            # per entry: column 4, cost 4, Lam 8, label 4
            nbytes = n * 72 + nnz * 20
            achieved = nbytes / (avg_ms * 1e-3) / 1e9
            roof = {"bound": "hbm", "kernel": "k_graph_step", "achieved": achieved, "peak": 8000.0,
                    "unit": "GB/s", "frac": achieved / 8000.0,
                    "traffic": measured_traffic("knn|%s|%d" % (args.instance, n)), "avg_launch_ms": avg_ms,
                    "launches": launches, "bytes_per_launch": nbytes, "nnz": nnz}
        out = {
            "value": elapsed / len(plain),
            "ms_per_step": 1e3 * elapsed / len(plain),
            "pair_rates": rates,
            "time_to_certified_s": elapsed / len(plain),
            "certified": all(r["certified"] for r in plain + runs),
            "certified_complete": all(r["certified_complete"] for r in plain + runs),
            "same_objective_all": len({r["primal2"] for r in plain + runs}) == 1,
            "iterations": [r["iterations"] for r in plain],
            "stop": [r["stop"] for r in plain],
            "objective2": plain[-1]["primal2"],
            "timing_note": "value and phase_s: solves without kernel events; roofline: the same number of "
                           "solves with HIP events around every scan and update launch",
            "phase_s": {k: float(np.mean([r["seconds"][k] for r in plain]))
                        for k in ("setup", "warm", "gdp", "finish", "certify")},
            "finish_detail": {"seconds": {k: float(np.mean([r["finish_seconds"][k] for r in plain]))
                                          for k in ("collect", "build", "flow")},
                              "paths": runs[-1]["finish_paths"], "phases": runs[-1]["finish_phases"],
                              "rounds": runs[-1]["finish_rounds"], "candidates": runs[-1]["finish_candidates"]},
            "roofline": roof,
        }
        return out

    cold_runs, cold_s, cold_timed = leg("cold", {})
    cold = summary(cold_runs, cold_s, cold_timed)
    warm_out = None
    if theta is not None:
        warm_out = summary(*leg("warm", {"mlp_theta": theta}))
        warm_out["same_objective"] = warm_out["objective2"] == cold["objective2"]
        warm_out["speedup_time_to_certified"] = cold["time_to_certified_s"] / warm_out["time_to_certified_s"]
    graph_out = None
    if args.start == "both" and args.graph == "complete":
        g_runs, g_s, g_timed = leg("graph-warm", {"warm": "graph"})
        graph_out = summary(g_runs, g_s, g_timed)
        graph_out["warm_iterations"] = [r["warm_iterations"] for r in g_runs]
        graph_out["note"] = ("Lam_0 from a cold GDP on the 10-nearest-neighbour candidate graph; value counts "
                             "the complete-graph iterations only")
        graph_out["same_objective"] = graph_out["objective2"] == cold["objective2"]
        graph_out["speedup_time_to_certified"] = cold["time_to_certified_s"] / graph_out["time_to_certified_s"]
    sec_out = None
    if args.start == "both" and args.graph == "complete" and args.sec_iters > 0:
        sec_out = subtour_leg(ctx, f2m, xy_dev, cold_runs[-1], args)
    out = {
        "metric": METRIC,
        "value": cold["value"],
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": cold["ms_per_step"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": "F2M GDP, %s graph, n=%d cities %s integer in [0,10^6)^2, seed %d, cold start, %s" % (
                       args.graph, n, args.instance, args.seed,
                       "%s scan" % args.scan if args.graph == "complete" else "k=10"),
                   "n": n, "instance": args.instance, "graph": args.graph, "start": "cold", "scan": args.scan},
    }
    out.update({k: v for k, v in cold.items() if k not in ("value", "ms_per_step")})
    out["warm"] = warm_out
    out["warm_graph"] = graph_out
    out["subtour"] = sec_out
    ctx.close()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(xy, cold_runs[-1]["lambda2_gdp"], args.cpu_seconds,
                                           cold_runs[-1]["iterations"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
