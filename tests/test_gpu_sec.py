"""Subtour-elimination rows on the GPU (F2M plus rows x(delta(S)) >= 2 with
multipliers M_q >= 0: Sec. 2 eq. 4-5, Sec. 3 with b = 2, the extension of
Sec. 5), through the C ABI, against the oracle (oracle/sec.py):

* the GDP trajectory -- every record (dual2, unsat, bad, max step, nonzero,
  hash, sum Lam, sum M), the stop, k*, Lam* and M* -- bit for bit: with no
  rows, from the F2M solution with one and two rounds of separated rows,
  and from random (Lam, M) on random layers of rows over several column
  tiles with a ragged tail;
* the separation: the same violated cuts, in the same order;
* the certificate of the trivial x: primal2, dual2, feasibility, tightness;
* the rounds driver: every round's rows, iterations, stop and bound as the
  oracle's rounds give them, the bound below the exact LP optimum with all
  those rows;
* argument errors.
"""
import numpy as np
import pytest

from oracle import core, exact, sec
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


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def layer_of_cuts(n, edges, cuts, base):
    """One round's cuts as a layer: cut j (the side without node 0) is a
    component of the support, or the complement of the component holding
    node 0, which then stands for it (same crossing edges)."""
    row = np.full(n, -1, np.int32)
    comps = sec.components(n, edges)
    for j, S in enumerate(cuts):
        key = tuple(S)
        hit = [C for C in comps if sec.canonical_cut(n, C) == key]
        assert len(hit) == 1
        row[hit[0]] = base + j
    return row


def sets_of(row_of, nrows):
    """The node set of every row id (row order)."""
    out = [None] * nrows
    for layer in np.atleast_2d(row_of):
        for q in np.unique(layer[layer >= 0]):
            out[q] = sorted(np.nonzero(layer == q)[0].tolist())
    return out


def compare_run(g, o, nrows):
    assert g["stop"] == o["stop"] and g["iterations"] == o["iters"] and g["kstar"] == o["kstar"]
    for k, (a, b) in enumerate(zip(g["trace"], o["trace"])):
        assert a["k"] == k
        for f in ("dual2", "unsat", "bad", "max_step", "nonzero", "hash", "sum_lam", "sum_mu"):
            assert a[f] == b[f], (k, f, a[f], b[f])


def run_both(ctx, xy, row_of, nrows, lam0, mu0, max_iters):
    n = len(xy)
    cuts = sets_of(row_of, nrows) if nrows else []
    o = sec.gdp_solve(xy, cuts, lam0=lam0, mu0=mu0, max_iters=max_iters)
    lam = dev(lam0, np.int64)
    mu = dev(mu0 if nrows else np.zeros(1), np.int64)
    g = ctx.sec_gdp(dev(xy, np.int32), dev(row_of, np.int32) if nrows else None, nrows, lam, mu,
                    max_iters=max_iters)
    compare_run(g, o, nrows)
    assert np.array_equal(lam.cpu().numpy(), o["lam"])
    if nrows:
        assert np.array_equal(mu.cpu().numpy()[:nrows], o["mu"])
    return g, o


@pytest.mark.parametrize("n,seed,cap", [(6, 1, 500), (20, 2, 500), (60, 3, 500), (700, 4, 25)])
def test_no_rows_is_f2m(ctx, n, seed, cap):
    print("sec no rows n=%d seed=%d" % (n, seed), flush=True)
    xy = I.uniform(n, 100000, seed)
    run_both(ctx, xy, None, 0, np.zeros(n, np.int64), [], cap)


def f2m_start(xy):
    r = core.gdp_solve(xy, handoff_div=0, max_iters=5000)
    edges = sec.trivial_x(xy, r["lam"], [], [])
    return r["lam"], edges


CASES = [(30, 1, "uniform"), (60, 1, "uniform"), (80, 5, "clustered"), (120, 1, "uniform")]


@pytest.mark.parametrize("n,seed,kind", CASES)
def test_first_round_equals_oracle(ctx, n, seed, kind):
    print("sec round 1 n=%d seed=%d %s" % (n, seed, kind), flush=True)
    xy = I.uniform(n, 100000, seed) if kind == "uniform" else I.clustered(n, 100000, seed, centres=4)
    lam0, edges = f2m_start(xy)
    cuts = sec.separate(n, edges)
    assert cuts
    # the GPU's separation: the same cuts in the same order
    nr = torch.empty(n, dtype=torch.int32, device="cuda")
    new, comps = ctx.sec_separate(dev(xy, np.int32), None, 0, dev(lam0, np.int64), None, nr)
    assert comps == len(sec.components(n, edges))
    got = sets_of(nr.cpu().numpy(), new)
    assert [list(sec.canonical_cut(n, S)) for S in got] == cuts
    # the GDP from the F2M solution with those rows
    row = nr.cpu().numpy().reshape(1, n)
    g, o = run_both(ctx, xy, row, new, lam0, np.zeros(new, np.int64), 3000)
    # a second round
    x = sec.trivial_x(xy, o["lam"], got, o["mu"])
    more = sec.separate(n, x, got)
    nr2 = torch.empty(n, dtype=torch.int32, device="cuda")
    new2, _ = ctx.sec_separate(dev(xy, np.int32), dev(row, np.int32), new, dev(o["lam"], np.int64),
                               dev(o["mu"], np.int64), nr2)
    got2 = sets_of(nr2.cpu().numpy(), new + new2)[new:]
    assert [list(sec.canonical_cut(n, S)) for S in got2] == more
    if new2:
        rows2 = np.stack([row[0], nr2.cpu().numpy()])
        run_both(ctx, xy, rows2, new + new2, o["lam"], np.concatenate([o["mu"], np.zeros(new2, np.int64)]), 3000)


def random_layers(n, nl, rng):
    """nl layers of disjoint random sets (2 .. n/3 nodes each)."""
    rows = np.full((nl, n), -1, np.int32)
    q = 0
    for l in range(nl):
        perm = rng.permutation(n)
        at = 0
        while True:
            k = int(rng.integers(2, max(3, n // 3)))
            if at + k > n - 2:
                break
            rows[l, perm[at:at + k]] = q
            q += 1
            at += k
            if rng.random() < 0.3:
                at += int(rng.integers(1, 5))   # nodes in no row of this layer
    return rows, q


@pytest.mark.parametrize("n,nl,seed,cap", [(12, 1, 1, 200), (40, 3, 2, 100), (300, 2, 3, 20), (600, 5, 4, 12),
                                           (517, 8, 5, 8)])
def test_random_layers_equal_oracle(ctx, n, nl, seed, cap):
    print("sec random layers n=%d layers=%d seed=%d" % (n, nl, seed), flush=True)
    rng = np.random.default_rng(seed)
    xy = I.uniform(n, 100000, 50 + seed) if seed % 2 else I.clustered(n, 100000, seed, centres=6)
    rows, q = random_layers(n, nl, rng)
    lam0 = rng.integers(-2000, 12000, n)
    mu0 = np.where(rng.random(q) < 0.4, 0, rng.integers(0, 3000, q))
    run_both(ctx, xy, rows, q, lam0, mu0, cap)


@pytest.mark.parametrize("n,seed", [(30, 1), (60, 1), (80, 5)])
def test_certificate_equals_oracle(ctx, n, seed):
    xy = I.uniform(n, 100000, seed) if seed != 5 else I.clustered(n, 100000, seed, centres=4)
    lam0, edges = f2m_start(xy)
    nr = torch.empty(n, dtype=torch.int32, device="cuda")
    new, _ = ctx.sec_separate(dev(xy, np.int32), None, 0, dev(lam0, np.int64), None, nr)
    row = nr.cpu().numpy().reshape(1, n)
    cuts = sets_of(row, new)
    rng = np.random.default_rng(seed)
    o = sec.gdp_solve(xy, cuts, lam0=lam0, max_iters=3000)
    for lam, mu in ((o["lam"], o["mu"]), (lam0, np.zeros(new, np.int64)),
                    (o["lam"] + rng.integers(-3, 4, n), o["mu"] + rng.integers(0, 3, new))):
        want = sec.certify(xy, lam, cuts, mu, sec.trivial_x(xy, lam, cuts, mu))
        got = ctx.sec_certify(dev(xy, np.int32), dev(row, np.int32), new, dev(lam, np.int64), dev(mu, np.int64))
        assert got["primal2"] == want["primal2"] and got["dual2"] == want["dual2"]
        assert got["feasible"] == want["feasible"] and got["certified"] == want["certified"]


def test_separation_at_several_tiles(ctx):
    # the support's components over 1500 nodes (six column tiles, a ragged
    # tail) at a Lam that leaves many of them
    n = 1500
    xy = I.clustered(n, 100000, 11, centres=40)
    lam = core.gdp_solve(xy, handoff_div=0, max_iters=60)["lam"]
    nr = torch.empty(n, dtype=torch.int32, device="cuda")
    new, comps = ctx.sec_separate(dev(xy, np.int32), None, 0, dev(lam, np.int64), None, nr)
    Z = sec.z_matrix(sec.cost_matrix(xy), lam, [], [])
    iu = np.triu_indices(n, 1)
    sel = Z[iu] <= 0
    edges = list(zip(iu[0][sel].tolist(), iu[1][sel].tolist(), [0] * int(sel.sum())))
    assert comps == len(sec.components(n, edges))
    got = sets_of(nr.cpu().numpy(), new)
    assert [list(sec.canonical_cut(n, S)) for S in got] == sec.separate(n, edges)


def test_rounds_equal_oracle_rounds(ctx):
    from paper_2011_08170_amd import f2m
    for n, seed in ((10, 3), (11, 8), (40, 2)):
        xy = I.uniform(n, 10000, seed) if n != 40 else I.clustered(n, 10000, seed, centres=3)
        lam0, edges = f2m_start(xy)
        # the oracle's rounds
        lam, mu, cuts, rounds = lam0, np.zeros(0, np.int64), [], []
        for _ in range(4):
            x = sec.trivial_x(xy, lam, cuts, mu)
            more = sec.separate(n, x, cuts)
            if not more:
                break
            s = sec.gdp_solve(xy, cuts + more, lam0=lam, mu0=list(mu) + [0] * len(more), max_iters=3000)
            rounds.append((len(more), s["iters"], s["stop"], s["trace"][s["kstar"]]["dual2"]))
            cuts, lam, mu = cuts + more, s["lam"], s["mu"]
        lamd = dev(lam0, np.int64)
        row_of = torch.full((f2m.SEC_MAX_LAYERS, n), -1, dtype=torch.int32, device="cuda")
        mud = torch.zeros(4 * n, dtype=torch.int64, device="cuda")
        r = ctx.sec_solve(dev(xy, np.int32), lamd, row_of, mud, max_rounds=4, max_iters=3000)
        assert r["rounds"] == len(rounds)
        assert list(zip(r["rows_added"], r["iterations"], r["stop"], r["dual2"])) == rounds
        assert np.array_equal(lamd.cpu().numpy(), lam)
        assert np.array_equal(mud.cpu().numpy()[:len(cuts)], mu)
        if cuts and n <= 12:
            lp = exact.simplex_sec_opt2(xy, cuts)
            assert r["best_dual2"] <= lp


def test_argument_errors(ctx):
    from paper_2011_08170_amd import f2m
    n = 20
    xy = dev(I.uniform(n, 10000, 1), np.int32)
    lam = torch.zeros(n, dtype=torch.int64, device="cuda")
    mu = torch.zeros(4, dtype=torch.int64, device="cuda")
    bad_id = np.full((1, n), -1, np.int32)
    bad_id[0, :3] = 7                       # id >= nrows
    small = np.full((1, n), -1, np.int32)
    small[0, 0] = 0                         # a row of one node
    twice = np.full((2, n), -1, np.int32)
    twice[0, :3] = 0
    twice[1, 5:8] = 0                       # row 0 in two layers
    for rows, q in ((bad_id, 1), (small, 1), (twice, 1)):
        with pytest.raises(f2m.F2MError):
            ctx.sec_gdp(xy, dev(rows, np.int32), q, lam, mu, max_iters=5)
    ok = np.full((1, n), -1, np.int32)
    ok[0, :4] = 0
    neg = torch.tensor([-1], dtype=torch.int64, device="cuda")
    with pytest.raises(f2m.F2MError):
        ctx.sec_gdp(xy, dev(ok, np.int32), 1, lam, neg, max_iters=5)
    # the context still works
    g = ctx.sec_gdp(xy, dev(ok, np.int32), 1, lam, mu[:1], max_iters=5)
    assert g["iterations"] >= 1
