"""Pins of the oracle's GDP for rows with other right-hand sides: the
fractional b-matching  sum_{e in delta(v)} x_e = b_v, 0 <= x <= 1, with
b_v in {1, 2, 3} (Sec. 3: binary rows, integral b_i, condition 8; the
gradient compares positions b_v and b_v + 1 of the row's sorted adjusted
lengths).  Exact optima from three independent routes, closed forms, the
record fields against a dense numpy evaluation, weak duality, and the
b = 2 case equal to F2M."""
import numpy as np
import pytest

from oracle import core, exact
from paper_2011_08170_amd import instances as I


def dense_Z(xy, lam):
    n = len(xy)
    C = np.array([[exact.euc2d(xy, u, v) if u != v else 0 for v in range(n)] for u in range(n)], dtype=np.int64)
    return 2 * C - lam[:, None] - lam[None, :]


def random_b(n, seed, lo=1, hi=3):
    return np.random.default_rng(seed).integers(lo, hi + 1, n).astype(np.int32)


@pytest.mark.parametrize("n", [4, 5, 6, 7])
def test_exact_optimum_three_ways(n):
    feasible = 0
    for seed in range(6):
        xy = I.uniform(n, 300, 500 + 10 * n + seed)
        b = random_b(n, seed)
        if n == 4:
            b = np.minimum(b, 3)
        bf = exact.brute_force_opt2(xy, b=b)
        sx = exact.simplex_opt2(xy, b=b)
        mc = core.exact_opt2(xy, b=b)
        assert bf == sx == mc, (n, seed, b.tolist(), bf, sx, mc)
        feasible += bf is not None
    assert feasible >= 3


def test_exact_optimum_highs():
    for seed in range(3):
        xy = I.uniform(60, 10000, 900 + seed)
        b = random_b(60, seed)
        assert core.exact_opt2(xy, b=b) == exact.highs_opt2(xy, b=b)


def test_closed_forms():
    # b = 1 on a 6 x 5 lattice of spacing 40: a perfect matching of lattice
    # neighbours costs n/2 * 40 and no degree-1 x can do better
    xy = I.lattice(6, 5, 40)
    n = len(xy)
    assert core.exact_opt2(xy, b=np.ones(n, np.int32)) == 2 * (n // 2) * 40
    # b = 3 on far-apart squares of side 10: each node takes its whole K4
    sq = np.concatenate([I.square4(10) + np.int32(200000 * i) for i in range(3)])
    assert core.exact_opt2(sq, b=np.full(12, 3, np.int32)) == 2 * 3 * (4 * 10 + 2 * 14)
    # b = 1 on far-apart pairs: the pairs themselves
    pairs = np.array([[0, 0], [3, 4], [500000, 0], [500012, 5]], np.int32)
    assert core.exact_opt2(pairs, b=np.ones(4, np.int32)) == 2 * (5 + 13)


def dense_record(xy, lam, b):
    n = len(xy)
    Z = dense_Z(xy, lam)
    rows = np.sort(Z[~np.eye(n, dtype=bool)].reshape(n, n - 1), axis=1)
    zb, zb1 = rows[np.arange(n), b - 1], rows[np.arange(n), b]
    s = zb + zb1
    step = np.sign(s) * ((np.abs(s) + 2) // 4)
    neg, zero = (rows < 0).sum(axis=1), (rows == 0).sum(axis=1)
    iu = np.triu_indices(n, 1)
    return dict(dual2=int((b * lam).sum() + np.minimum(Z[iu], 0).sum()),
                unsat=int(((zb > 0) | (zb1 < 0)).sum()), bad=int((2 * neg + zero != 2 * b).sum()),
                max_step=int(np.abs(step).max()), nonzero=int((step != 0).sum()), sum_lam=int(lam.sum())), step


def test_record_fields_against_dense():
    for seed in range(4):
        xy = I.uniform(50, 2000, 40 + seed)
        b = random_b(50, seed)
        lam = np.random.default_rng(seed).integers(-400, 2500, 50).astype(np.int64)
        want, step = dense_record(xy, lam, b)
        got = core.gdp_iter(xy, lam, b=b)
        assert np.array_equal(got["step"], step)
        for f, v in want.items():
            assert got["rec"][f] == v, (seed, f)


def test_degree_two_is_f2m():
    xy = I.uniform(200, 50000, 7)
    a = core.gdp_solve(xy, handoff_div=50)
    b = core.gdp_solve(xy, handoff_div=50, b=np.full(200, 2, np.int32))
    assert np.array_equal(a["trace"], b["trace"]) and np.array_equal(a["lam"], b["lam"])


def test_weak_duality_and_trivial_certificates():
    hits = 0
    for seed in range(6):
        n = 40
        xy = I.uniform(n, 3000, 70 + seed)
        b = random_b(n, seed)
        opt2 = core.exact_opt2(xy, b=b)
        if opt2 is None:
            continue
        r = core.gdp_solve(xy, b=b, max_iters=400)
        assert np.all(r["trace"][:, 1] <= opt2)
        if r["stop"] == "trivial":
            eu, ev, ex2 = core.trivial_x(xy, r["lam"])
            c = core.certify(xy, r["lam"], eu, ev, ex2, b=b)
            assert c["certified"] and c["primal2"] == opt2
            hits += 1
        # the flow's own duals certify its x for these degrees
        o2, x2, lam = core.exact_opt2(xy, want_x=True, b=b)
        eu, ev, ex2 = core.dense_to_edges(x2)
        c = core.certify(xy, lam, eu, ev, ex2, b=b)
        assert c["certified"] and c["primal2"] == opt2
    assert hits >= 2   # seeds 0 and 2 stop "trivial"


def test_rejects_bad_degrees():
    xy = I.uniform(10, 100, 1)
    with pytest.raises(RuntimeError):
        core.gdp_iter(xy, np.zeros(10, np.int64), b=np.full(10, 4, np.int32))
    with pytest.raises(RuntimeError):
        core.gdp_iter(xy, np.zeros(10, np.int64), b=np.zeros(10, np.int32))
