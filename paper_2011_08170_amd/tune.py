"""Autotuner for the launch shapes of libf2m.

The GDP scan's launch shape -- rows per lane (1, 2, 4) and the number of
column slices -- and the batched loop's slices per instance and iterations
per replayed graph change only the time, never a bit of the result (one
owner per row, an order-free merge of the slices, integer reductions, stop
decisions on the device).  The tuner times each candidate on a given
instance (or batch), checks that every candidate gives the same trajectory,
and stores the fastest in a cache file that the library itself reads
(`f2m_opts.tuner_cache`): text, one entry per line, tab-separated

    device name, mode, size bucket, rows, slices, chunk

with mode "culled" / "full" for `f2m_solve` and "batch-culled" /
"batch-full" for `f2m_solve_batch` (keyed by the batch's total node count);
0 keeps the library's built-in value.  Timing uses the library's own HIP
events around every scan launch (single solves) or the GDP phase of the
batch.

    from paper_2011_08170_amd import f2m, tune
    tune.tune(ctx, coords_device, scan="culled", path=p)
    r = ctx.solve(coords_device, tuner_cache=p)
"""
from __future__ import annotations

import os
import tempfile

import numpy as np

CANDIDATES = {
    "full": [(r, s) for r in (1, 2, 4) for s in (0, 8, 16, 32, 64)],
    "culled": [(1, 1), (1, 2), (1, 4)] + [(2, s) for s in (1, 2, 4, 8, 16)],
}
# batched loop: (slices per instance, iterations per replayed graph)
BATCH_CANDIDATES = {
    "culled": [(s, c) for s in (1, 2) for c in (4, 8, 16, 32)],
    "full": [(s, c) for s in (2, 4, 8) for c in (4, 8, 16)],
}
HEADER = "# libf2m tuner cache: device\tmode\tsize bucket\trows\tslices\tchunk\n"


def bucket(n: int) -> int:
    """Half-octave size bucket: the integer nearest to 2 log2 n, computed
    exactly as floor(bitlength(n^4) / 2) (the library computes the same)."""
    n = max(int(n), 1)
    return (n ** 4).bit_length() // 2


def cache_path() -> str:
    return os.environ.get("F2M_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "libf2m", "tune.tsv"))


def load_cache(path: str | None = None) -> dict:
    """{(device, mode, bucket): (rows, slices, chunk)}; unreadable lines are
    skipped, as the library skips them."""
    path = path or cache_path()
    out = {}
    try:
        with open(path) as f:
            lines = f.read().splitlines()
    except (OSError, UnicodeDecodeError):
        return out
    for line in lines:
        if line.startswith("#"):
            continue
        fld = line.split("\t")
        if len(fld) < 6:
            continue
        try:
            b, r, s, c = int(fld[2]), int(fld[3]), int(fld[4]), int(fld[5])
        except ValueError:
            continue
        if r not in (0, 1, 2, 4) or s < 0 or not 0 <= c <= 4096:
            continue
        out[(fld[0], fld[1], b)] = (r, s, c)
    return out


def save_cache(data: dict, path: str | None = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=os.path.dirname(os.path.abspath(path)), suffix=".tmp")
    with os.fdopen(fd, "w") as f:
        f.write(HEADER)
        for (dev, mode, b), (r, s, c) in sorted(data.items()):
            if "\t" in dev or "\n" in dev:
                raise ValueError("device name with a tab or newline")
            f.write("%s\t%s\t%d\t%d\t%d\t%d\n" % (dev, mode, b, r, s, c))
    os.replace(tmp, path)


def store(device: str, mode: str, n: int, rows: int, slices: int, chunk: int = 0, path: str | None = None):
    data = load_cache(path)
    data[(device, mode, bucket(n))] = (int(rows), int(slices), int(chunk))
    save_cache(data, path)


def lookup(device: str, n: int, mode: str = "culled", path: str | None = None):
    """Cached (rows, slices, chunk) for this device, mode and size, or None."""
    return load_cache(path).get((device, mode, bucket(n)))


def measure(ctx, coords, scan: str, shape, iters: int = 6):
    """(ms per scan launch, trace) of `iters` GDP iterations with `shape`."""
    r = ctx.solve(coords, max_iters=iters, handoff_div=0, finish="none", scan=scan, shape=shape,
                  time_kernels=True, trace=True)
    # the first launch uses neighbour seeds; later ones the previous top-4
    return r["scan_ms"] / max(r["scan_launches"], 1), r["trace"]


def tune(ctx, coords, scan: str = "culled", candidates=None, iters: int = 6, path: str | None = None,
         save: bool = True) -> dict:
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
        timings[sh] = ms
        if ref is None:
            ref = trace
        elif not np.array_equal(ref, trace):
            same = False
    best = min(cands, key=lambda sh: timings[sh])
    out = {"best": tuple(best), "n": n, "scan": scan, "timings_ms": timings, "identical": same}
    if save and same:
        store(ctx.device_name(), scan, n, best[0], best[1], 0, path)
    return out


def tune_batch(ctx, coords, offsets, scan: str = "culled", candidates=None, path: str | None = None,
               save: bool = True, repeats: int = 2) -> dict:
    """Times the batched GDP loop (no finish) for every (slices, chunk)
    candidate, checks that every candidate gives the same trajectories, and
    stores the fastest under the batch's total node count."""
    cands = list(candidates or BATCH_CANDIDATES[scan])
    total = int(np.asarray(offsets)[-1])
    timings = {}
    ref = None
    same = True
    for sl, ch in cands:
        best_t = None
        for _ in range(repeats + 1):   # the first run warms the shape
            _, res = ctx.solve_batch(coords, offsets, finish="none", trace=True, scan=scan, slices=sl, chunk=ch)
            t = max(r["seconds"]["gdp"] for r in res)
            best_t = t if best_t is None else min(best_t, t)
        timings[(sl, ch)] = best_t
        traces = [r["trace"] for r in res]
        if ref is None:
            ref = traces
        elif not all(np.array_equal(a, b) for a, b in zip(ref, traces)):
            same = False
    best = min(cands, key=lambda c: timings[c])
    out = {"best": tuple(best), "total": total, "scan": scan, "timings_s": timings, "identical": same}
    if save and same:
        store(ctx.device_name(), "batch-" + scan, total, 0, best[0], best[1], path)
    return out
