"""Pins of the oracle's candidate-graph variant: "the top N closest
neighbors for each node" (Sec. 5.3), union-symmetrised, and the GDP, the
certificate and the exact optimum restricted to that graph."""
import numpy as np
import pytest

from oracle import core, exact
from paper_2011_08170_amd import instances as I


def test_knn_against_lexsort():
    for xy in (I.uniform(300, 2000, 1), I.lattice_jitter(12, 13, 10, 1, 2), I.with_duplicates(200, 100, 30, 3)):
        n = len(xy)
        for k in (1, 4, 10, 16):
            idx = core.knn(xy, k)
            d = ((xy[:, None, :].astype(np.int64) - xy[None, :, :]) ** 2).sum(-1)
            for v in range(0, n, 7):
                u = np.array([w for w in range(n) if w != v])
                order = np.lexsort((u, d[v, u]))
                assert list(idx[v]) == list(u[order[:k]])


def test_knn_graph_structure():
    xy = I.clustered(500, 1000000, 4, centres=10)
    rowptr, col = core.knn_graph(xy, 10)
    n = len(xy)
    idx = core.knn(xy, 10)
    edges = set()
    for v in range(n):
        row = col[rowptr[v]:rowptr[v + 1]]
        assert np.all(np.diff(row) > 0) and v not in row and len(row) >= 10
        assert set(idx[v]) <= set(row)
        edges |= {(v, int(u)) for u in row}
    assert all((u, v) in edges for (v, u) in edges)


@pytest.mark.parametrize("n,k", [(6, 2), (7, 3), (8, 3)])
def test_graph_optimum_brute_force(n, k):
    for seed in range(3):
        xy = I.uniform(n, 500, 1000 + 10 * n + seed)
        g = core.knn_graph(xy, k)
        b = exact.brute_force_opt2(xy, graph=g)
        # None on both sides when no degree-2 x exists on the graph
        assert core.exact_opt2(xy, graph=g) == b


def test_graph_optimum_highs_and_restriction():
    for seed in (1, 2):
        xy = I.clustered(200, 1000000, seed, centres=8)
        g = core.knn_graph(xy, 10)
        og = core.exact_opt2(xy, graph=g)
        assert og == exact.highs_opt2(xy, graph=g)
        assert og >= core.exact_opt2(xy)   # a restriction can only cost more


def test_full_knn_graph_is_the_complete_graph():
    xy = I.uniform(60, 5000, 9)
    g = core.knn_graph(xy, 59)
    a = core.gdp_solve(xy, graph=g)
    b = core.gdp_solve(xy)
    assert np.array_equal(a["trace"], b["trace"]) and np.array_equal(a["lam"], b["lam"])
    assert core.exact_opt2(xy, graph=g) == core.exact_opt2(xy)


def test_graph_rows_against_sort():
    xy = I.uniform(150, 3000, 6)
    g = core.knn_graph(xy, 6)
    rowptr, col = g
    lam = np.random.default_rng(0).integers(0, 800, 150).astype(np.int64)
    r = core.gdp_rows(xy, lam, np.arange(150), graph=g)
    for v in range(150):
        u = col[rowptr[v]:rowptr[v + 1]].astype(np.int64)
        z = np.array([2 * exact.euc2d(xy, v, w) for w in u]) - lam[v] - lam[u]
        order = np.lexsort((u, z))
        assert list(r["z4"][v]) == list(z[order[:4]])
        assert list(r["i4"][v]) == list(u[order[:4]])
        assert r["rowneg"][v] == np.minimum(z, 0).sum()


def test_graph_certificate_of_graph_optimum():
    xy = I.uniform(120, 20000, 3)
    g = core.knn_graph(xy, 8)
    opt2, x2, lam = core.exact_opt2(xy, want_x=True, graph=g)
    eu, ev, ex = core.dense_to_edges(x2)
    c = core.certify(xy, lam, eu, ev, ex, graph=g)
    assert c["certified"] and c["primal2"] == opt2
    # an edge outside the graph is infeasible for the restricted problem
    rowptr, col = g
    v = 0
    outside = [u for u in range(1, 120) if u not in set(col[rowptr[0]:rowptr[1]])][0]
    c2 = core.certify(xy, lam, np.r_[eu, [v]], np.r_[ev, [outside]], np.r_[ex, [1]], graph=g)
    assert not c2["feasible"]
