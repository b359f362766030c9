"""Autotuner: cache handling on the CPU; on the GPU every candidate launch
shape gives the same trajectory and the tuner stores the fastest."""
import numpy as np
import pytest

from paper_2011_08170_amd import instances as I
from paper_2011_08170_amd import tune


def test_bucket_and_key(tmp_path):
    assert tune.bucket(1000) == tune.bucket(1100)
    assert tune.bucket(1000) != tune.bucket(2000)
    assert tune.key(100000, "full", "dev") == "dev|full|%.1f" % tune.bucket(100000)


def test_cache_roundtrip(tmp_path):
    path = str(tmp_path / "t" / "tune.json")
    assert tune.load_cache(path) == {}
    tune.save_cache({"dev|culled|10.0": {"best": [2, 4]}}, path)
    assert tune.lookup(1024, "culled", path=path, device="dev") == (2, 4)
    assert tune.lookup(1024, "full", path=path, device="dev") is None
    open(path, "w").write("not json")
    assert tune.load_cache(path) == {}


def test_candidates_are_valid_shapes():
    for mode, cands in tune.CANDIDATES.items():
        assert cands and all(r in (1, 2, 4) and s >= 0 for r, s in cands)


@pytest.mark.gpu
def test_tuner_shapes_identical_on_gpu(tmp_path):
    torch = pytest.importorskip("torch")
    from paper_2011_08170_amd import f2m
    with f2m.Context(0) as ctx:
        xy = torch.from_numpy(I.uniform(20000, 1000000, 3)).cuda()
        for scan in ("culled", "full"):
            out = tune.tune(ctx, xy, scan=scan, iters=3, path=str(tmp_path / "c.json"))
            assert out["identical"], out
            assert tuple(out["best"]) in tune.CANDIDATES[scan]
            assert tune.lookup(20000, scan, path=str(tmp_path / "c.json")) == tuple(out["best"])
        # the batched solve: every slice count gives the same results
        cxy, off = I.batch(6, 500, 3000, 5)
        base = ctx.solve_batch(cxy, off, trace=True)[1]
        for slices in (2, 5):
            other = ctx.solve_batch(cxy, off, trace=True, slices=slices)[1]
            for a, b in zip(base, other):
                assert np.array_equal(a["trace"], b["trace"]) and a["primal2"] == b["primal2"]
