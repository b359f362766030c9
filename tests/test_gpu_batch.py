"""Batched GDP (many uneven instances, one graph-captured loop) against the
oracle and against independent solves, bit for bit."""
import numpy as np
import pytest

from oracle import core
from paper_2011_08170_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    from paper_2011_08170_amd import f2m
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    c = f2m.Context(0)
    yield c
    c.close()


def small_batch():
    # sizes log-uniform in [200, 3000], half uniform, half clustered, plus
    # the degenerate sizes 3 and 4 and a ragged 257
    xy, off = I.batch(14, 200, 3000, 7)
    parts = [xy[off[i]:off[i + 1]] for i in range(14)]
    parts += [I.uniform(3, 1000, 1), I.uniform(4, 1000, 2), I.uniform(257, 100000, 3)]
    offs = np.zeros(len(parts) + 1, np.int64)
    offs[1:] = np.cumsum([len(p) for p in parts])
    return np.concatenate(parts), offs, parts


def test_batch_matches_oracle(ctx):
    from paper_2011_08170_amd import f2m
    xy, off, parts = small_batch()
    st, res = ctx.solve_batch(xy, off, trace=True)
    assert st == "ok"
    for part, r in zip(parts, res):
        assert r["certified"]
        if len(part) == 3:
            assert r["primal2"] == core.exact_opt2(part)
            continue
        o = core.gdp_solve(part, handoff_div=f2m.HANDOFF_DIV)
        assert r["iterations"] == o["iters"] and r["stop"] == o["stop"] and r["kstar"] == o["kstar"]
        assert np.array_equal(r["trace"], o["trace"])
        assert np.array_equal(r["lambda2_gdp"], o["lam"])
        if len(part) <= 1500:
            assert r["primal2"] == core.exact_opt2(part)
        c = core.certify(part, r["lambda2"], r["edge_u"], r["edge_v"], r["edge_x2"])
        assert c["certified"] and c["primal2"] == r["primal2"]


def test_batch_equals_independent_solves(ctx):
    xy, off = I.batch(10, 1000, 8000, 11)
    for scan in ("culled", "full"):
        st, res = ctx.solve_batch(xy, off, trace=True, scan=scan)
        assert st == "ok"
        for i, r in enumerate(res):
            s = ctx.solve(xy[off[i]:off[i + 1]], trace=True)
            for k in ("trace", "lambda2_gdp", "lambda2", "edge_u", "edge_v", "edge_x2"):
                assert np.array_equal(r[k], s[k]), (scan, i, k)
            assert r["primal2"] == s["primal2"] and r["certified"]


def test_batch_equals_independent_solves_large(ctx):
    # instances big enough that the finish's single-source tail runs by
    # chunks: the batch's finishing threads use one thread each, a single
    # solve several, and the bits must not differ
    parts = [I.uniform(40000, 1000000, 21), I.clustered(50000, 1000000, 22), I.uniform(30000, 1000000, 23)]
    off = np.zeros(len(parts) + 1, np.int64)
    off[1:] = np.cumsum([len(p) for p in parts])
    st, res = ctx.solve_batch(np.concatenate(parts), off)
    assert st == "ok"
    for part, r in zip(parts, res):
        s = ctx.solve(part)
        for k in ("lambda2_gdp", "lambda2", "edge_u", "edge_v", "edge_x2"):
            assert np.array_equal(r[k], s[k]), k
        assert r["primal2"] == s["primal2"] and r["certified"] and s["certified"]


def test_benchmark_size_single_equals_batched(ctx):
    # n = 100000 uniform in [0, 10^6)^2, seed 1, as bench.py times it: the
    # single solve (four waves per 64 rows, candidate lists) and a batch of
    # that one instance (one wave per 64 rows, no lists) run different scan
    # code; the trajectories, Lam and the objective must agree bit for bit
    xy = I.uniform(100000, 1000000, 1)
    off = np.array([0, len(xy)], np.int64)
    st, res = ctx.solve_batch(xy, off, trace=True)
    assert st == "ok"
    s = ctx.solve(xy, trace=True)
    r = res[0]
    for k in ("trace", "lambda2_gdp"):
        assert np.array_equal(r[k], s[k]), k
    assert r["iterations"] == s["iterations"] and r["stop"] == s["stop"]
    assert r["primal2"] == s["primal2"] and r["certified"] and s["certified"]
