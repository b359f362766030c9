"""GPU parity of the candidate-graph variant (k nearest neighbours,
Sec. 5.3) against the oracle: the graph itself, the GDP trajectory on it,
the restricted optimum and its certificate, and the complete-graph check."""
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


GRAPHS = [
    ("uniform_3000_k10", lambda: I.uniform(3000, 1000000, 1), 10),
    ("clustered_20000_k10", lambda: I.clustered(20000, 1000000, 2), 10),
    ("lattice_ties_k10", lambda: I.lattice_jitter(40, 41, 30, 1, 3), 10),
    ("duplicates_k16", lambda: I.with_duplicates(2500, 20000, 300, 4), 16),
    ("uniform_999_k16", lambda: I.uniform(999, 100000, 5), 16),
]


@pytest.mark.parametrize("name,make,k", GRAPHS, ids=[g[0] for g in GRAPHS])
def test_knn_graph_equals_oracle(ctx, name, make, k):
    from paper_2011_08170_amd import f2m
    xy = make()
    rp, col = f2m.knn_graph(ctx, dev(xy), k)
    orp, ocol = core.knn_graph(xy, k)
    assert np.array_equal(rp, orp) and np.array_equal(col, ocol)


@pytest.mark.parametrize("name,make,k", [("uniform_2000", lambda: I.uniform(2000, 1000000, 7), 10),
                                         ("clustered_3000", lambda: I.clustered(3000, 1000000, 8), 10),
                                         ("lattice_ties", lambda: I.lattice_jitter(30, 31, 30, 2, 9), 16)])
def test_graph_trajectory_equals_oracle(ctx, name, make, k):
    xy = make()
    g = core.knn_graph(xy, k)
    for div in (0, 300):
        o = core.gdp_solve(xy, graph=g, handoff_div=div)
        r = ctx.solve(xy, graph="knn", knn_k=k, trace=True, finish="none", handoff_div=div)
        assert r["iterations"] == o["iters"] and r["stop"] == o["stop"] and r["kstar"] == o["kstar"]
        assert np.array_equal(r["trace"], o["trace"])
        assert np.array_equal(r["lambda2_gdp"], o["lam"])


@pytest.mark.parametrize("seed", [1, 2])
def test_graph_solve_certified_restricted_optimum(ctx, seed):
    xy = I.clustered(900, 1000000, seed, centres=20)
    g = core.knn_graph(xy, 10)
    r = ctx.solve(xy, graph="knn", knn_k=10)
    assert r["certified"] and r["status"] == "ok"
    assert r["primal2"] == r["dual2"] == core.exact_opt2(xy, graph=g)
    c = core.certify(xy, r["lambda2"], r["edge_u"], r["edge_v"], r["edge_x2"], graph=g)
    assert c["certified"]
    full = core.certify(xy, r["lambda2"], r["edge_u"], r["edge_v"], r["edge_x2"])
    assert full["dual2"] == r["dual2_complete"]
    assert full["certified"] == r["certified_complete"]
    assert r["certified_complete"] == (r["primal2"] == core.exact_opt2(xy))


def test_c3_shape_sampled_rows(ctx):
    # n = 200,000 clustered (200 centres, sigma = 2% of the side), k = 10:
    # sampled rows hold their own 10 nearest neighbours, and every other
    # member v has the row among v's 10 nearest
    from paper_2011_08170_amd import f2m
    xy = I.clustered(200000, 1000000, 1)
    rp, col = f2m.knn_graph(ctx, dev(xy), 10)
    n = len(xy)
    assert rp[-1] == len(col) and np.all(np.diff(rp) >= 10)
    rows = np.random.default_rng(3).choice(n, 64, replace=False)
    own = core.knn_rows(xy, 10, rows)
    for r, v in enumerate(rows):
        row = col[rp[v]:rp[v + 1]]
        assert np.all(np.diff(row) > 0)
        assert set(own[r]) <= set(row)
        extra = np.array(sorted(set(row) - set(own[r])), np.int64)
        if extra.size:
            theirs = core.knn_rows(xy, 10, extra)
            assert all(v in theirs[i] for i in range(extra.size))
    r = ctx.solve(xy, graph="knn", knn_k=10)
    assert r["certified"] and r["graph_nnz"] == len(col)


@pytest.mark.parametrize("name,make", [("uniform_2500", lambda: I.uniform(2500, 1000000, 11)),
                                       ("clustered_3000", lambda: I.clustered(3000, 1000000, 12)),
                                       ("lattice_ties", lambda: I.lattice_jitter(35, 36, 30, 2, 13))])
def test_graph_warm_start_equals_oracle(ctx, name, make):
    # the oracle's two stages: a cold GDP on the k = 10 candidate graph, then
    # the complete-graph GDP from its Lam*; the GPU's seeds from the first
    # stage change no bit of the second stage's trajectory
    xy = make()
    g = core.knn_graph(xy, 10)
    og = core.gdp_solve(xy, graph=g, handoff_div=300)
    oc = core.gdp_solve(xy, lam0=og["lam"], handoff_div=300)
    r = ctx.solve(dev(xy), warm="graph", trace=True, handoff_div=300)
    assert r["warm_iterations"] == og["iters"]
    assert r["iterations"] == oc["iters"] and r["stop"] == oc["stop"] and r["kstar"] == oc["kstar"]
    assert np.array_equal(r["trace"], oc["trace"])
    assert np.array_equal(r["lambda2_gdp"], oc["lam"])
    cold = ctx.solve(dev(xy))
    assert r["certified"] and cold["certified"] and r["primal2"] == cold["primal2"]


def test_graph_warm_start_small_n_is_cold(ctx):
    xy = I.uniform(9, 1000, 3)   # n <= knn_k: no candidate graph, a cold start
    r = ctx.solve(dev(xy), warm="graph")
    c = ctx.solve(dev(xy))
    assert r["warm_iterations"] == 0 and r["iterations"] == c["iterations"] and r["primal2"] == c["primal2"]
