"""The oracle of the GDP with subtour-elimination rows (oracle/sec.py):
F2M plus rows x(delta(S)) >= 2 with multipliers M_q >= 0 (Sec. 2, eq. 4-5;
the gradient of Sec. 3 on rows with b = 2; the extension named in Sec. 5).

Pins, none of them the oracle checking itself:
* with no subtour row it is the F2M oracle: the same trajectory bit for bit
  as the C oracle (itself pinned in test_oracle_gdp / test_oracle_pins);
* weak duality against an exact-rational LP (oracle.exact, with a surplus
  variable per subtour row) at every iterate and at random (Lam, M >= 0): a
  wrong sign or factor on the subtour term lets the bound pass the LP;
* strong duality where the trivial x certifies: primal = dual = the exact LP
  optimum, also equal to scipy's HiGHS -- pins the 2 sum M term, the
  crossing test and the factor 2;
* a hand-derived case: two far triangles, F2M = the two perimeters, the
  subtour LP = the best tour through both;
* separation: every returned cut is crossed by no edge of x's support.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import core, exact, sec
from paper_2011_08170_amd import instances as I


def first_round(xy):
    """F2M by the oracle's GDP (trivial stop), its x and the subtour rows
    that x violates."""
    r = core.gdp_solve(xy, handoff_div=0)
    if r["stop"] != "trivial":
        return None
    ed = sec.trivial_x(xy, r["lam"], [], [])
    return r, ed, sec.separate(len(xy), ed)


def cases():
    out = []
    for seed in range(40):
        rng = np.random.default_rng(seed)
        n = int(rng.integers(6, 11))
        xy = I.clustered(n, 10000, seed, centres=2) if seed % 2 else I.uniform(n, 10000, seed)
        fr = first_round(xy)
        if fr and fr[2]:
            out.append((seed, xy, fr))
    return out


CASES = cases()


def test_no_rows_is_the_f2m_oracle():
    for n, seed in ((6, 1), (20, 2), (60, 3)):
        xy = I.uniform(n, 100000, seed)
        a = core.gdp_solve(xy, max_iters=500)
        b = sec.gdp_solve(xy, [], max_iters=500)
        assert b["stop"] == a["stop"] and b["iters"] == a["iters"] and b["kstar"] == a["kstar"]
        assert np.array_equal(b["lam"], a["lam"])
        for k, rec in enumerate(b["trace"]):
            row = a["trace"][k]
            assert [rec["dual2"], rec["unsat"], rec["bad"], rec["max_step"], rec["nonzero"], rec["sum_lam"]] == \
                [int(x) for x in row[[1, 2, 3, 4, 5, 7]]]
            assert rec["hash"] == int(row[6]) & ((1 << 64) - 1)


def test_two_far_triangles_by_hand(golden):
    g = golden["two_far_triangles_subtour"]
    xy = np.array(g["xy"], np.int32)
    # F2M: each triangle alone, sides 10, 10 (nint(sqrt(106))) and 10
    assert core.exact_opt2(xy) == g["f2m_opt2"] == 2 * 60
    fr = first_round(xy)
    assert fr is not None and fr[2] == [g["cut"]]
    # one subtour row: the best tour, two sides of each triangle plus the two
    # cheapest crossing edges between path ends: 20 + 20 + 990 + 1000
    lp = exact.simplex_sec_opt2(xy, [g["cut"]])
    assert lp == g["sec_opt2"] == 2 * 2030
    s = sec.gdp_solve(xy, [g["cut"]], lam0=fr[0]["lam"], max_iters=2000)
    assert max(t["dual2"] for t in s["trace"]) <= lp


@pytest.mark.parametrize("seed,xy,fr", CASES[:10], ids=[str(c[0]) for c in CASES[:10]])
def test_weak_duality_along_the_trajectory(seed, xy, fr):
    r, ed, cuts = fr
    lp = exact.simplex_sec_opt2(xy, cuts)
    assert lp is not None and lp >= core.exact_opt2(xy)
    s = sec.gdp_solve(xy, cuts, lam0=r["lam"], max_iters=3000)
    for t in s["trace"]:
        assert Fraction(t["dual2"]) <= lp
        assert t["sum_mu"] >= 0
    assert np.all(s["mu"] >= 0)
    # any Lam and any M >= 0, far from the trajectory
    rng = np.random.default_rng(seed)
    for _ in range(5):
        lam = rng.integers(-5000, 20000, len(xy))
        mu = rng.integers(0, 20000, len(cuts))
        assert Fraction(sec.gdp_iter(xy, lam, cuts, mu)["rec"]["dual2"]) <= lp


def test_strong_duality_where_certified():
    certified = 0
    for seed, xy, (r, ed, cuts) in CASES:
        s = sec.gdp_solve(xy, cuts, lam0=r["lam"], max_iters=3000)
        x = sec.trivial_x(xy, s["lam"], cuts, s["mu"])
        c = sec.certify(xy, s["lam"], cuts, s["mu"], x)
        if not c["certified"]:
            continue
        certified += 1
        lp = exact.simplex_sec_opt2(xy, cuts)
        assert Fraction(c["primal2"]) == Fraction(c["dual2"]) == lp, seed
        assert abs(exact.highs_sec_opt2(xy, cuts) - float(lp)) < 1e-6
    assert certified >= 10


def test_separation_returns_violated_rows():
    for seed, xy, (r, ed, cuts) in CASES[:10]:
        n = len(xy)
        for S in cuts:
            assert 0 not in S and 2 <= len(S) <= n - 2
            ins = set(S)
            assert not any((u in ins) != (v in ins) for (u, v, _) in ed)
        # the same x gives no new row once those are in
        assert sec.separate(n, ed, cuts) == []


def test_second_round_raises_the_bound():
    done = 0
    for seed, xy, (r, ed, cuts) in CASES:
        s = sec.gdp_solve(xy, cuts, lam0=r["lam"], max_iters=3000)
        x = sec.trivial_x(xy, s["lam"], cuts, s["mu"])
        more = sec.separate(len(xy), x, cuts)
        if not more:
            continue
        lp1 = exact.simplex_sec_opt2(xy, cuts)
        lp2 = exact.simplex_sec_opt2(xy, cuts + more)
        assert lp2 >= lp1
        s2 = sec.gdp_solve(xy, cuts + more, lam0=s["lam"], mu0=list(s["mu"]) + [0] * len(more), max_iters=3000)
        assert max(t["dual2"] for t in s2["trace"]) <= lp2
        done += 1
        if done >= 3:
            break
