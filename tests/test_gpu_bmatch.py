"""Rows with right-hand sides b_v in {1, 2, 3} (the fractional b-matching,
Sec. 3: binary rows, integral b) on the GPU, through the C ABI, against the
oracle: whole GDP trajectories (every record, the stop, k*, Lam*) bit for
bit, the certified optimum equal to the oracle's exact optimum with the same
b, b = 2 everywhere equal to F2M, and the candidate-graph variant."""
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


def degrees(n, seed, lo=1, hi=3):
    return np.random.default_rng(seed).integers(lo, hi + 1, n).astype(np.int32)


@pytest.mark.parametrize("n,seed,handoff,scan", [(1000, 1, 0, "culled"), (1000, 2, 50, "culled"),
                                                 (1000, 3, 0, "full"), (3001, 4, 50, "culled"),
                                                 (257, 5, 0, "culled")])
def test_trajectory_equals_oracle(ctx, n, seed, handoff, scan):
    print("b trajectory n=%d seed=%d handoff=%d %s" % (n, seed, handoff, scan), flush=True)
    xy = I.uniform(n, 100000, 100 + seed)
    b = degrees(n, seed)
    g = ctx.solve(torch.from_numpy(xy).cuda(), degree_b=b, handoff_div=handoff, scan=scan, trace=True,
                  finish="none", max_iters=400)
    o = core.gdp_solve(xy, b=b, handoff_div=handoff, max_iters=400)
    assert g["iterations"] == o["iters"] and g["stop"] == o["stop"] and g["kstar"] == o["kstar"]
    assert np.array_equal(g["trace"], o["trace"])
    assert np.array_equal(g["lambda2_gdp"], o["lam"])


@pytest.mark.parametrize("n,seed,kind", [(40, 1, "uniform"), (150, 2, "uniform"), (300, 3, "clustered"),
                                         (200, 4, "ones"), (200, 5, "threes")])
def test_certified_optimum(ctx, n, seed, kind):
    print("b optimum n=%d seed=%d %s" % (n, seed, kind), flush=True)
    xy = I.clustered(n, 100000, seed, centres=5) if kind == "clustered" else I.uniform(n, 100000, 200 + seed)
    b = {"ones": np.ones(n, np.int32), "threes": np.full(n, 3, np.int32)}.get(kind, degrees(n, seed))
    g = ctx.solve(xy, degree_b=b)
    assert g["certified"]
    assert g["primal2"] == g["dual2"] == core.exact_opt2(xy, b=b)
    c = core.certify(xy, g["lambda2"], g["edge_u"], g["edge_v"], g["edge_x2"], b=b)
    assert c["certified"] and c["primal2"] == g["primal2"] and c["dual2"] == g["dual2"]


def test_b_two_is_f2m(ctx):
    xy = I.uniform(2000, 1000000, 7)
    xy_d = torch.from_numpy(xy).cuda()
    a = ctx.solve(xy_d, trace=True)
    b = ctx.solve(xy_d, trace=True, degree_b=np.full(len(xy), 2, np.int32))
    assert np.array_equal(a["trace"], b["trace"]) and np.array_equal(a["lambda2_gdp"], b["lambda2_gdp"])
    assert a["primal2"] == b["primal2"] and a["certified"] and b["certified"]


def test_graph_trajectory_and_optimum(ctx):
    from paper_2011_08170_amd import f2m
    xy = I.uniform(2000, 100000, 8)
    b = degrees(len(xy), 8)
    xy_d = torch.from_numpy(xy).cuda()
    rowptr, col = f2m.knn_graph(ctx, xy_d, 10)
    g = ctx.solve(xy_d, graph="knn", degree_b=b, trace=True, handoff_div=50)
    o = core.gdp_solve(xy, b=b, handoff_div=50, graph=(rowptr, col))
    assert g["iterations"] == o["iters"] and g["stop"] == o["stop"]
    assert np.array_equal(g["trace"], o["trace"]) and np.array_equal(g["lambda2_gdp"], o["lam"])
    assert g["certified"]
    c = core.certify(xy, g["lambda2"], g["edge_u"], g["edge_v"], g["edge_x2"], graph=(rowptr, col), b=b)
    assert c["certified"] and c["primal2"] == g["primal2"]


def test_degree_errors(ctx):
    from paper_2011_08170_amd import f2m
    xy = I.uniform(50, 1000, 1)
    for bad in (np.zeros(50, np.int32), np.full(50, 4, np.int32)):
        with pytest.raises(f2m.F2MError):
            ctx.solve(xy, degree_b=bad)
