"""Pins of the oracle's GDP rule (eq. 9, eq. 10 and Sec. 3, with the damped
midpoint reading) and of its certificate (Lagrangian bound of Sec. 2)."""
import numpy as np
import pytest

from oracle import core, exact
from paper_2011_08170_amd import instances as I


def dense_Z(xy, lam):
    n = len(xy)
    C = np.array([[exact.euc2d(xy, u, v) if u != v else 0 for v in range(n)] for u in range(n)],
                 dtype=np.int64)
    Z = 2 * C - lam[:, None] - lam[None, :]
    return Z


def test_step_rounding_table():
    # dLam = sign(s) * floor((|s| + 2) / 4): s/4 rounded half away from zero
    table = {0: 0, 1: 0, 2: 1, 3: 1, 4: 1, 5: 1, 6: 2, 7: 2, 9: 2, 10: 3, 48: 12, 50: 13, 101: 25,
             102: 26}
    for s, d in table.items():
        assert core.step(s) == d
        assert core.step(-s) == -d


def test_worked_square(golden):
    g = golden["square4"]
    xy = np.array(g["coords"], np.int32)
    r = core.gdp_solve(xy)
    assert r["stop"] == g["stop"]
    assert r["iters"] == len(g["lam_trajectory"])
    assert list(r["trace"][:, 1]) == g["dual2"]
    assert list(r["trace"][:, 3]) == g["bad"]
    assert list(r["lam"]) == g["lam_trajectory"][-1]
    eu, ev, ex2 = core.trivial_x(xy, r["lam"])
    got = sorted((int(a), int(b), int(c)) for a, b, c in zip(eu, ev, ex2))
    assert got == sorted(tuple(sorted(e[:2])) + (e[2],) for e in g["x_edges"])
    c = core.certify(xy, r["lam"], eu, ev, ex2)
    assert c["certified"] and c["primal2"] == g["opt2"]


@pytest.mark.parametrize("m", [2, 3, 4])
def test_separated_triangles_certify_in_one_step(m):
    # each node: two triangle sides (c=10) and far edges; from Lam=0 the
    # midpoint lands between the triangle sides and the far edges, so the
    # trivial x is the triangles after one step
    xy = I.triangles(m)
    r = core.gdp_solve(xy)
    assert r["stop"] == "trivial" and r["iters"] == 2
    eu, ev, ex2 = core.trivial_x(xy, r["lam"])
    c = core.certify(xy, r["lam"], eu, ev, ex2)
    assert c["certified"] and c["primal2"] == 60 * m == core.exact_opt2(xy)


def test_rows_against_full_sort():
    # per-row order statistics against numpy's full lexicographic sort
    rnd = np.random.default_rng(3)
    for xy in (I.uniform(40, 300, 1), I.lattice_jitter(6, 7, 20, 1, 2), I.with_duplicates(30, 200, 6, 4)):
        n = len(xy)
        for trial in range(3):
            lam = rnd.integers(-40, 400, n).astype(np.int64)
            Z = dense_Z(xy, lam)
            r = core.gdp_rows(xy, lam, np.arange(n))
            for v in range(n):
                u = np.array([w for w in range(n) if w != v])
                z = Z[v, u]
                order = np.lexsort((u, z))
                assert list(r["z4"][v]) == list(z[order[:4]])
                assert list(r["i4"][v]) == list(u[order[:4]])
                assert r["neg"][v] == (z < 0).sum()
                assert r["zero"][v] == (z == 0).sum()
                assert r["rowneg"][v] == np.minimum(z, 0).sum()
                s = int(z[order[1]] + z[order[2]])
                assert r["step"][v] == int(np.sign(s)) * ((abs(s) + 2) // 4)


def test_iteration_record_against_dense():
    xy = I.uniform(60, 1000, 9)
    lam = np.random.default_rng(1).integers(0, 600, 60).astype(np.int64)
    Z = dense_Z(xy, lam)
    r = core.gdp_iter(xy, lam)["rec"]
    iu = np.triu_indices(60, 1)
    assert r["dual2"] == 2 * lam.sum() + np.minimum(Z[iu], 0).sum()
    assert r["sum_lam"] == lam.sum()


def test_step_sign_follows_degree_deficit():
    # at an unsatisfied node the step moves lambda toward degree 2: Z(2) > 0
    # means fewer than 2 negative edges and the step is positive; Z(3) < 0
    # means 3 or more negative edges and the step is negative
    xy = I.uniform(80, 2000, 4)
    rnd = np.random.default_rng(2)
    for _ in range(5):
        lam = rnd.integers(-500, 1500, 80).astype(np.int64)
        r = core.gdp_rows(xy, lam, np.arange(80))
        z2, z3 = r["z4"][:, 1], r["z4"][:, 2]
        deg2 = 2 * r["neg"] + r["zero"]
        assert np.all(r["step"][z2 > 0] > 0) and np.all(deg2[z2 > 0] <= 3)
        assert np.all(r["step"][z3 < 0] < 0) and np.all(deg2[z3 < 0] >= 6)


def test_weak_duality_along_trajectory():
    for seed in (1, 2):
        n = 20 if seed == 1 else 40
        xy = I.uniform(n, 1000, seed)
        opt2 = exact.simplex_opt2(xy) if seed == 1 else core.exact_opt2(xy)
        r = core.gdp_solve(xy)
        assert np.all(r["trace"][:, 1] <= opt2)
        rnd = np.random.default_rng(seed)
        for _ in range(10):
            lam = rnd.integers(-300, 900, n).astype(np.int64)
            assert core.gdp_iter(xy, lam)["rec"]["dual2"] <= opt2


def test_fixed_point_nodes_satisfied_and_close():
    # the rule's fixed points satisfy Z(2) <= 0 <= Z(3) at every node
    for seed in (1, 2, 3):
        xy = I.uniform(200, 100000, seed)
        r = core.gdp_solve(xy)
        opt2 = core.exact_opt2(xy)
        last = r["trace"][-1]
        assert last[1] <= opt2
        if r["stop"] == "fixed":
            assert last[2] == 0 and last[5] == 0
        assert opt2 - r["trace"][:, 1].max() <= 1e-4 * opt2


def test_label_permutation_equivariance():
    xy = I.uniform(120, 5000, 8)
    perm = np.random.default_rng(0).permutation(120)
    a = core.gdp_solve(xy, max_iters=60)
    b = core.gdp_solve(xy[perm], max_iters=60)
    # every value statistic of the trajectory is label free (the hash is not)
    cols = [1, 2, 3, 4, 5, 7]
    k = min(a["iters"], b["iters"])
    assert np.array_equal(a["trace"][:k, cols], b["trace"][:k, cols])


def test_translation_invariance():
    xy = I.uniform(100, 5000, 5)
    a = core.gdp_solve(xy, max_iters=40)
    b = core.gdp_solve(xy + np.int32(777), max_iters=40)
    assert np.array_equal(a["trace"], b["trace"]) and np.array_equal(a["lam"], b["lam"])


def test_cap_and_best_iterate():
    xy = I.uniform(100, 5000, 5)
    full = core.gdp_solve(xy)
    r = core.gdp_solve(xy, max_iters=5)
    assert r["stop"] == "cap" and r["iters"] == 6
    kbest = int(np.argmax(r["trace"][:, 1]))
    assert r["kstar"] == kbest
    assert np.array_equal(r["trace"], full["trace"][:6])


def test_certificate_rejects_mistakes(golden):
    g = golden["square4"]
    xy = np.array(g["coords"], np.int32)
    lam = np.array(g["lam_trajectory"][-1], np.int64)
    eu, ev, ex2 = core.trivial_x(xy, lam)
    assert core.certify(xy, lam, eu, ev, ex2)["certified"]
    # Lam moved far enough to lower the bound
    bad = lam.copy(); bad[0] += 10
    assert not core.certify(xy, bad, eu, ev, ex2)["certified"]
    # x: flip one value, drop, duplicate, out of range, self loop, x2=3
    f = ex2.copy(); f[0] = 1
    assert not core.certify(xy, lam, eu, ev, f)["feasible"]
    assert not core.certify(xy, lam, eu[1:], ev[1:], ex2[1:])["feasible"]
    assert not core.certify(xy, lam, np.r_[eu, eu[:1]], np.r_[ev, ev[:1]], np.r_[ex2, ex2[:1]])["feasible"]
    o = ev.copy(); o[0] = 4
    assert not core.certify(xy, lam, eu, o, ex2)["feasible"]
    o = ev.copy(); o[0] = eu[0]
    assert not core.certify(xy, lam, eu, o, ex2)["feasible"]
    f = ex2.copy(); f[0] = 3
    assert not core.certify(xy, lam, eu, ev, f)["feasible"]


def test_certificate_rejects_negative_edge_outside_x():
    # a fifth city close to the square: with the square's Lam and a Lam for
    # it that makes a non-solution edge negative, the bound drops below the
    # primal and nothing is certified
    xy = np.array([[0, 0], [10, 0], [10, 10], [0, 10], [5, 5]], np.int32)
    opt2, x2, lam = core.exact_opt2(xy, want_x=True)
    eu, ev, ex2 = core.dense_to_edges(x2)
    assert core.certify(xy, lam, eu, ev, ex2)["certified"]
    # push one node's Lam up so an unused edge at it turns negative
    used = {(int(a), int(b)) for a, b in zip(eu, ev)}
    v = 4
    unused = [u for u in range(5) if u != v and (min(u, v), max(u, v)) not in used]
    Z = dense_Z(xy, lam)
    bump = int(Z[v, unused[0]]) + 1
    lam2 = lam.copy(); lam2[v] += bump
    c = core.certify(xy, lam2, eu, ev, ex2)
    assert c["feasible"] and not c["certified"] and c["dual2"] < c["primal2"]


def test_handoff_stop():
    # stops at the first iterate with #unsatisfied * div <= n; every earlier
    # record has more unsatisfied nodes; the records up to it are the plain
    # run's records
    xy = I.uniform(400, 100000, 3)
    full = core.gdp_solve(xy)
    for div in (20, 100, 400):
        r = core.gdp_solve(xy, handoff_div=div)
        k = r["iters"] - 1
        assert r["stop"] == "handoff" and r["kstar"] == k
        assert r["trace"][k, 2] * div <= 400
        assert np.all(r["trace"][:k, 2] * div > 400)
        assert np.array_equal(r["trace"], full["trace"][:k + 1])
