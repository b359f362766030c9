"""Autotuner for the scan launch shape of libf2m.

The GDP scan's launch shape -- rows per lane (1, 2, 4) and the number of
column slices -- changes only the time, never a bit of the result (one owner
per row, an order-free merge of the slices, integer reductions).  The tuner
times a few GDP iterations for each candidate shape on a given instance,
keeps the fastest, and caches it per (device, scan mode, size bucket) in a
JSON file.  Timing uses the library's own HIP events around every scan
launch.

    from paper_2011_08170_amd import f2m, tune
    best = tune.tune(ctx, coords_device, scan="culled")
    r = ctx.solve(coords_device, shape=tune.lookup(n, "culled"))
"""
from __future__ import annotations

import json
import math
import os
import tempfile

import numpy as np

CANDIDATES = {
    "full": [(r, s) for r in (1, 2, 4) for s in (0, 8, 16, 32, 64)],
    "culled": [(r, s) for r in (1, 2) for s in (1, 2, 4, 8, 16)],
}


def bucket(n: int) -> float:
    """Half-octave size bucket."""
    return round(2.0 * math.log2(max(int(n), 2))) / 2.0


def cache_path() -> str:
    return os.environ.get("F2M_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "libf2m", "tune.json"))


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(data: dict, path: str | None = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=os.path.dirname(path), suffix=".tmp")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def device_name() -> str:
    try:
        import torch
        return torch.cuda.get_device_name(0)
    except Exception:   # no device: the key still works for a cache file
        return "unknown"


def key(n: int, scan: str, device: str | None = None) -> str:
    return "%s|%s|%.1f" % (device or device_name(), scan, bucket(n))


def lookup(n: int, scan: str = "culled", path: str | None = None, device: str | None = None):
    """Cached best shape (rows, slices) for this size and mode, or None."""
    e = load_cache(path).get(key(n, scan, device))
    return tuple(e["best"]) if e else None


def measure(ctx, coords, scan: str, shape, iters: int = 6):
    """(ms per scan launch, trace) of `iters` GDP iterations with `shape`."""
    r = ctx.solve(coords, max_iters=iters, handoff_div=0, finish="none", scan=scan, shape=shape,
                  time_kernels=True, trace=True)
    # the first launch uses neighbour seeds; later ones the previous top-4
    return r["scan_ms"] / max(r["scan_launches"], 1), r["trace"]


def tune(ctx, coords, scan: str = "culled", candidates=None, iters: int = 6, path: str | None = None,
         store: bool = True) -> dict:
    """Times every candidate shape on `coords` (a device tensor or host
    array), checks that all give the same trajectory, stores the fastest."""
    cands = list(candidates or CANDIDATES[scan])
    n = int(coords.shape[0])
    timings = {}
    ref = None
    same = True
    for sh in cands:
        measure(ctx, coords, scan, sh, 2)   # warm the shape's code path
        ms, trace = measure(ctx, coords, scan, sh, iters)
        timings["%d,%d" % sh] = ms
        if ref is None:
            ref = trace
        elif not np.array_equal(ref, trace):
            same = False
    best = min(cands, key=lambda sh: timings["%d,%d" % sh])
    out = {"best": list(best), "n": n, "scan": scan, "timings_ms": timings, "identical": same}
    if store and same:
        data = load_cache(path)
        data[key(n, scan)] = out
        save_cache(data, path)
    return out
