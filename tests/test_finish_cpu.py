"""The host exact finish of libf2m (f2m_finish.cpp), run on the CPU with a
brute-force pair source, against the oracle's exact optimum.  The result
must be a certificate (primal2 == dual2 on the complete graph) from any
starting Lam: zero, random, or a GDP fixed point."""
import numpy as np
import pytest

from oracle import core
from paper_2011_08170_amd import instances as I
from tests.native import harness


@pytest.fixture(scope="module")
def L(tmp_path_factory):
    return harness.build(tmp_path_factory.mktemp("finish"))


def check(L, xy, lam0):
    lam, eu, ev, ex, st = harness.finish(L, xy, lam0)
    c = core.certify(xy, lam, eu, ev, ex)
    assert c["certified"], (c, st)
    assert c["primal2"] == core.exact_opt2(xy)
    assert np.all(eu < ev)
    # the bulk path (costs, initial flow bits and incidence lists from the
    # source; the pairs as a list or, as the GPU source gives them, as keys)
    # starts from the same state, so it must end in the same bits; so must
    # a workspace that served other instances before
    for bulk, reuse in ((True, False), (2, False), (True, True), (2, True), (False, True)):
        got = harness.finish(L, xy, lam0, bulk=bulk, reuse=reuse)
        for a, b in zip((lam, eu, ev, ex), got[:4]):
            assert np.array_equal(a, b), (bulk, reuse)
        assert got[4] == st
    # the chunked single-source tail serves the excess nodes in another
    # order: another optimum may come out, always certified, and the same
    # one on every run and for any thread count
    par = [harness.finish(L, xy, lam0, bulk=True, reuse=r) for r in (2, 2, 3)]
    c = core.certify(xy, *par[0][:4])
    assert c["certified"] and c["primal2"] == core.exact_opt2(xy), c
    for other in par[1:]:
        for a, b in zip(par[0][:4], other[:4]):
            assert np.array_equal(a, b)
    return st


@pytest.mark.parametrize("n", [3, 4, 5, 7, 12])
def test_small_from_zero(L, n):
    for seed in range(3):
        xy = I.uniform(n, 300, 10 * n + seed)
        check(L, xy, np.zeros(n, np.int64))


def test_from_gdp_fixed_point(L):
    for seed in (1, 2, 3):
        xy = I.uniform(200, 100000, seed)
        r = core.gdp_solve(xy)
        st = check(L, xy, r["lam"])
        assert st["rounds"] <= 4


def test_from_gdp_handoff(L):
    for seed in (4, 5):
        xy = I.uniform(300, 100000, seed)
        r = core.gdp_solve(xy, handoff_div=30)
        assert r["stop"] == "handoff"
        check(L, xy, r["lam"])


def test_from_random_and_ties(L):
    rnd = np.random.default_rng(4)
    for xy in (I.lattice_jitter(8, 9, 20, 2, 1), I.with_duplicates(60, 400, 8, 2), I.lattice(6, 6, 5),
               I.clustered(150, 100000, 3, centres=4)):
        n = len(xy)
        check(L, xy, rnd.integers(-50, 200, n).astype(np.int64))
        check(L, xy, core.gdp_solve(xy)["lam"])


def test_odd_lattice_half_values(L):
    # 3x3 lattice: odd n, so no all-integer 2-factor of unit edges fits
    # every node; the optimum has half values or longer edges
    xy = I.lattice(3, 3, 10)
    check(L, xy, np.zeros(9, np.int64))


def z_order(xy):
    """The instance with its nodes renumbered along a Z-order curve (the
    library hands the finish nodes in such a spatial order)."""
    x = xy[:, 0].astype(np.int64)
    y = xy[:, 1].astype(np.int64)
    key = np.zeros(len(xy), np.int64)
    for b in range(20):
        key |= ((x >> b) & 1) << (2 * b) | ((y >> b) & 1) << (2 * b + 1)
    return xy[np.argsort(key, kind="stable")]


def test_parallel_tail_many_chunks(L):
    # n = 2000 in a spatial order: the parallel tail has several chunks,
    # most searches commit inside their chunk, the rest go to the
    # sequential tail
    rnd = np.random.default_rng(11)
    for xy in (z_order(I.uniform(2000, 100000, 7)), z_order(I.clustered(2000, 100000, 8, centres=6))):
        n = len(xy)
        lam = harness.finish(L, xy, np.zeros(n, np.int64), bulk=True)[0]
        for lam0 in (lam + rnd.integers(-3, 4, n), rnd.integers(0, 3000, n).astype(np.int64)):
            ref = harness.finish(L, xy, lam0, bulk=True)
            cr = core.certify(xy, *ref[:4])
            assert cr["certified"], cr
            par = [harness.finish(L, xy, lam0, bulk=True, reuse=r) for r in (2, 2, 3)]
            c = core.certify(xy, *par[0][:4])
            assert c["certified"] and c["primal2"] == cr["primal2"], c
            for other in par[1:]:
                for a, b in zip(par[0][:4], other[:4]):
                    assert np.array_equal(a, b)


def test_b_matching_degrees(L):
    # rows with right-hand sides b_v in {1, 2, 3} (the b-matching of Sec. 3):
    # both copies of v carry b_v units; certified against the oracle's
    # certificate and exact optimum with the same b, from Lam = 0 and from
    # the oracle's GDP stop
    rnd = np.random.default_rng(21)
    for n, seed in ((5, 1), (9, 2), (40, 3), (200, 4)):
        xy = I.uniform(n, 100000, seed)
        b = rnd.integers(1, 4, n).astype(np.int32)
        opt = core.exact_opt2(xy, b=b)
        for lam0 in (np.zeros(n, np.int64), core.gdp_solve(xy, b=b, handoff_div=50)["lam"]):
            ref = harness.finish(L, xy, lam0, b=b)
            c = core.certify(xy, *ref[:4], b=b)
            assert c["certified"] and c["primal2"] == opt, (n, c)
            got = harness.finish(L, xy, lam0, bulk=True, b=b)
            for x, y in zip(ref[:4], got[:4]):
                assert np.array_equal(x, y)
    # b = 2 everywhere is F2M
    xy = I.uniform(60, 100000, 9)
    a = harness.finish(L, xy, np.zeros(60, np.int64))
    c = harness.finish(L, xy, np.zeros(60, np.int64), b=np.full(60, 2, np.int32))
    for x, y in zip(a[:4], c[:4]):
        assert np.array_equal(x, y)
