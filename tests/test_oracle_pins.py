"""Pins of the oracle's iteration record and stop rules against quantities
computed here independently: a dense numpy evaluation of the adjusted
lengths (eq. 9 doubled, exact lengths from Python's integer square root),
the published SplitMix64 outputs, and 2-cycles of the rule found by
tests/golden/make_cycle_case.py."""
import json
import os

import numpy as np
import pytest

from oracle import core, exact
from paper_2011_08170_amd import instances as I

HERE = os.path.dirname(os.path.abspath(__file__))
M64 = (1 << 64) - 1


def finaliser(z):
    """SplitMix64's output function, written from its definition."""
    z = ((z ^ (z >> 30)) * 0xbf58476d1ce4e5b9) & M64
    z = ((z ^ (z >> 27)) * 0x94d049bb133111eb) & M64
    return z ^ (z >> 31)


def splitmix64(seed, k, gamma=0x9e3779b97f4a7c15):
    s, out = seed, []
    for _ in range(k):
        s = (s + gamma) & M64
        out.append(finaliser(s))
    return out


def lam_hash(lam):
    """sum_v finaliser(Lam_v xor gamma*(v+1)) mod 2^64 (two's complement Lam)."""
    h = 0
    for v, x in enumerate(lam):
        h = (h + finaliser((int(x) & M64) ^ ((0x9e3779b97f4a7c15 * (v + 1)) & M64))) & M64
    return h


def dense_Z(xy, lam):
    n = len(xy)
    C = np.array([[exact.euc2d(xy, u, v) if u != v else 0 for v in range(n)] for u in range(n)], dtype=np.int64)
    return 2 * C - lam[:, None] - lam[None, :]


def dense_record(xy, lam):
    """Every field of the iteration record at Lam, and the step, from the
    dense matrix of Z (row v: all u != v, sorted as a multiset)."""
    n = len(xy)
    Z = dense_Z(xy, lam)
    off = ~np.eye(n, dtype=bool)
    rows = np.sort(Z[off].reshape(n, n - 1), axis=1)
    z2, z3 = rows[:, 1], rows[:, 2]
    s = z2 + z3
    step = np.sign(s) * ((np.abs(s) + 2) // 4)
    neg = (rows < 0).sum(axis=1)
    zero = (rows == 0).sum(axis=1)
    iu = np.triu_indices(n, 1)
    rec = dict(dual2=int(2 * lam.sum() + np.minimum(Z[iu], 0).sum()),
               unsat=int(((z2 > 0) | (z3 < 0)).sum()),
               bad=int((2 * neg + zero != 4).sum()),
               max_step=int(np.abs(step).max()),
               nonzero=int((step != 0).sum()),
               hash=lam_hash(lam),
               sum_lam=int(lam.sum()))
    return rec, step


def test_splitmix64_reference_outputs():
    g = json.load(open(os.path.join(HERE, "golden", "splitmix64.json")))
    assert splitmix64(g["seed"], len(g["outputs"]), int(g["gamma"], 16)) == g["outputs"]


@pytest.mark.parametrize("name,make,lo,hi", [
    ("uniform", lambda: I.uniform(70, 3000, 11), -500, 3000),
    ("ties", lambda: I.lattice_jitter(6, 8, 30, 0, 3), -50, 150),
    ("dups", lambda: I.with_duplicates(50, 400, 8, 5), -200, 700),
    ("negative_lam", lambda: I.uniform(40, 1000, 12), -4000, -100),
])
def test_record_fields_against_dense(name, make, lo, hi):
    xy = make()
    n = len(xy)
    rnd = np.random.default_rng(n)
    for trial in range(4):
        lam = rnd.integers(lo, hi, n).astype(np.int64)
        if trial == 0:
            lam[:] = 0
        want, step = dense_record(xy, lam)
        got = core.gdp_iter(xy, lam)
        assert np.array_equal(got["step"], step), name
        for f, v in want.items():
            assert got["rec"][f] == v, (name, trial, f)
        assert core.lam_hash(lam) == want["hash"]


def cycle_cases():
    return json.load(open(os.path.join(HERE, "golden", "cycle_case.json")))["cases"]


@pytest.mark.parametrize("case", cycle_cases(), ids=lambda c: "try%d" % c["try"])
def test_cycle_stop(case):
    xy = np.array(case["coords"], np.int32)
    lam = np.array(case["lam0"], np.int64)
    # the rule by dense numpy: Lam_0 .. Lam_K with K the first k >= 2 at
    # which Lam_k = Lam_{k-2} element by element
    lams, recs = [lam.copy()], []
    for k in range(200):
        rec, step = dense_record(xy, lams[-1])
        recs.append(rec)
        assert rec["bad"] > 0 and rec["nonzero"] > 0   # neither trivial nor fixed before the cycle
        if k >= 2 and np.array_equal(lams[k], lams[k - 2]):
            break
        lams.append(lams[-1] + step)
    K = len(recs) - 1
    assert K == case["stop_k"]
    assert not np.array_equal(lams[K], lams[K - 1])   # a genuine 2-cycle, not a fixed point
    duals = [r["dual2"] for r in recs]
    kstar = int(np.argmax(duals))                     # first iterate of largest dual
    assert kstar == case["kstar"]
    o = core.gdp_solve(xy, lam0=case["lam0"], max_iters=200, handoff_div=0)
    assert o["stop"] == "cycle" and o["iters"] == K + 1 and o["kstar"] == kstar
    assert np.array_equal(o["lam"], lams[kstar])
    for k in range(K + 1):
        assert o["trace"][k, 0] == k
        for j, f in enumerate(core.TRACE_FIELDS[1:], start=1):
            want = recs[k][f]
            got = int(o["trace"][k, j]) & M64 if f == "hash" else int(o["trace"][k, j])
            assert got == want, (k, f)
