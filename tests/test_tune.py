"""Autotuner: the cache format on the CPU; on the GPU every candidate launch
shape gives the same trajectory, the tuner stores the fastest, the library
reads the cache itself (f2m_opts.tuner_cache) and a cached shape's
trajectory equals the oracle's."""
import math

import numpy as np
import pytest

from paper_2011_08170_amd import instances as I
from paper_2011_08170_amd import tune


def test_bucket_is_nearest_half_octave():
    # floor(bitlength(n^4) / 2) is the integer nearest to 2 log2 n (no n
    # sits on a boundary: 2 log2 n = b + 1/2 has no integer solution)
    for n in list(range(1, 5000)) + [65535, 65536, 100000, 200000, (1 << 30) - 1]:
        assert tune.bucket(n) == math.floor(2 * math.log2(n) + 0.5), n
    assert tune.bucket(1000) == tune.bucket(1100)
    assert tune.bucket(1000) != tune.bucket(2000)


def test_cache_roundtrip(tmp_path):
    path = str(tmp_path / "t" / "tune.tsv")
    assert tune.load_cache(path) == {}
    tune.store("dev A", "culled", 1024, 1, 4, 0, path)
    tune.store("dev A", "batch-culled", 50000, 0, 2, 16, path)
    assert tune.lookup("dev A", 1024, "culled", path=path) == (1, 4, 0)
    assert tune.lookup("dev A", 1024, "full", path=path) is None
    assert tune.lookup("dev B", 1024, "culled", path=path) is None
    assert tune.lookup("dev A", 50000, "batch-culled", path=path) == (0, 2, 16)
    text = open(path).read()
    assert text.startswith("#") and "dev A\tculled\t20\t1\t4\t0\n" in text
    # lines the library would skip are skipped here too
    with open(path, "a") as f:
        f.write("dev A\tculled\t21\t3\t1\t0\n")      # rows must be 0, 1, 2 or 4
        f.write("dev A\tculled\tx\t1\t1\t0\n")
        f.write("short line\n")
    assert tune.lookup("dev A", 1500, "culled", path=path) is None
    open(path, "w").write("not a cache")
    assert tune.load_cache(path) == {}


def test_candidates_are_valid_shapes():
    for mode, cands in tune.CANDIDATES.items():
        assert cands and all(r in (1, 2, 4) and s >= 0 for r, s in cands)
    for mode, cands in tune.BATCH_CANDIDATES.items():
        assert cands and all(s >= 1 and c >= 1 for s, c in cands)


@pytest.mark.gpu
def test_tuner_shapes_identical_on_gpu(tmp_path):
    torch = pytest.importorskip("torch")
    from paper_2011_08170_amd import f2m
    path = str(tmp_path / "c.tsv")
    with f2m.Context(0) as ctx:
        dev = ctx.device_name()
        assert dev
        xy = torch.from_numpy(I.uniform(20000, 1000000, 3)).cuda()
        for scan in ("culled", "full"):
            out = tune.tune(ctx, xy, scan=scan, iters=3, path=path)
            assert out["identical"], out
            assert tuple(out["best"]) in tune.CANDIDATES[scan]
            assert tune.lookup(dev, 20000, scan, path=path) == tuple(out["best"]) + (0,)
            # the library takes the cached shape itself
            r = ctx.solve(xy, max_iters=3, handoff_div=0, finish="none", scan=scan, tuner_cache=path)
            assert (r["scan_rows"], r["scan_slices"]) == tuple(out["best"]) or out["best"][1] == 0
            if out["best"][1] == 0:
                assert r["scan_rows"] == out["best"][0]
        # the batched solve: every candidate gives the same results; the
        # cached one is taken
        cxy, off = I.batch(6, 500, 3000, 5)
        base = ctx.solve_batch(cxy, off, trace=True)[1]
        bt = tune.tune_batch(ctx, cxy, off, candidates=[(1, 4), (2, 8), (1, 16)], path=path, repeats=1)
        assert bt["identical"], bt
        got = ctx.solve_batch(cxy, off, trace=True, tuner_cache=path)[1]
        for a, b in zip(base, got):
            # every instance has at least two column tiles: its slice count is the cached one
            assert b["scan_slices"] == bt["best"][0]
            assert np.array_equal(a["trace"], b["trace"]) and a["primal2"] == b["primal2"]


@pytest.mark.gpu
@pytest.mark.parametrize("mode,shape", [("culled", (1, 4)), ("culled", (2, 2)), ("full", (2, 4))])
def test_cached_shape_trajectory_equals_oracle(tmp_path, mode, shape):
    torch = pytest.importorskip("torch")
    from oracle import core
    from paper_2011_08170_amd import f2m
    path = str(tmp_path / "c.tsv")
    xy = I.uniform(5000, 1000000, 11)   # 20 column tiles: 1, 2 and 4 slices split them evenly
    with f2m.Context(0) as ctx:
        tune.store(ctx.device_name(), mode, len(xy), shape[0], shape[1], 0, path)
        g = ctx.solve(torch.from_numpy(xy).cuda(), scan=mode, trace=True, finish="none", tuner_cache=path)
    assert (g["scan_rows"], g["scan_slices"]) == shape
    if mode == "culled" and shape[0] == 1:
        assert g["scan_list_uses"] > 0
    o = core.gdp_solve(xy, handoff_div=f2m.HANDOFF_DIV)
    assert g["iterations"] == o["iters"] and g["stop"] == o["stop"] and g["kstar"] == o["kstar"]
    assert np.array_equal(g["trace"], o["trace"])
    assert np.array_equal(g["lambda2_gdp"], o["lam"])
