"""GPU parity: libf2m (HIP, gfx950) against the CPU oracle, bit for bit.

Every comparison is exact: the method is integer arithmetic throughout
(Lam = 2*lambda int64, exact EUC_2D lengths), so the tolerance is zero."""
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


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def gpu_step(ctx, xy, lam):
    n = len(xy)
    out = dict(lam=torch.empty(n, dtype=torch.int64, device="cuda"),
               z4=torch.empty(4 * n, dtype=torch.int64, device="cuda"),
               i4=torch.empty(4 * n, dtype=torch.int32, device="cuda"),
               neg=torch.empty(n, dtype=torch.int32, device="cuda"),
               zero=torch.empty(n, dtype=torch.int32, device="cuda"),
               step=torch.empty(n, dtype=torch.int64, device="cuda"))
    rec = ctx.gdp_step(dev(xy, np.int32), dev(lam, np.int64), out["lam"], out["z4"], out["i4"], out["neg"],
                       out["zero"], out["step"])
    h = {k: v.cpu().numpy() for k, v in out.items()}
    h["z4"] = h["z4"].reshape(n, 4)
    h["i4"] = h["i4"].reshape(n, 4)
    return rec, h


CASES = [
    ("n4", lambda: I.uniform(4, 1000, 1)),
    ("n5", lambda: I.uniform(5, 1000, 2)),
    ("n257", lambda: I.uniform(257, 100000, 3)),
    ("c1_1000", lambda: I.uniform(1000, 100000, 1)),
    ("ragged_3001", lambda: I.uniform(3001, 1000000, 4)),
    ("ties_lattice", lambda: I.lattice_jitter(30, 33, 50, 3, 5)),
    ("dups", lambda: I.with_duplicates(700, 5000, 60, 6)),
    ("clustered_2000", lambda: I.clustered(2000, 1000000, 7)),
    ("full_span", lambda: np.array(I.uniform(600, 1 << 20, 8), dtype=np.int32) - (1 << 19)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_gdp_step_matches_oracle(ctx, name, make):
    xy = make()
    n = len(xy)
    rnd = np.random.default_rng(n)
    for lam in (np.zeros(n, np.int64), rnd.integers(-3000, 9000, n).astype(np.int64)):
        rec, g = gpu_step(ctx, xy, lam)
        o = core.gdp_iter(xy, lam)
        assert np.array_equal(g["z4"], o["z4"]), name
        assert np.array_equal(g["i4"], np.where(o["i4"] < 0, -1, o["i4"])), name
        assert np.array_equal(g["neg"], o["neg"]) and np.array_equal(g["zero"], o["zero"])
        assert np.array_equal(g["step"], o["step"])
        assert np.array_equal(g["lam"], lam + o["step"])
        for f in ("dual2", "unsat", "bad", "max_step", "nonzero", "hash", "sum_lam"):
            assert rec[f] == o["rec"][f], (name, f)


def _boundary_pairs(count, seed):
    """(dx, dy) with 0 <= dx, dy < 2^20 whose length is within 3/4 (in 4 D)
    of a half-integer: 4 D is within 3 of an odd square, where FP32 alone
    could round the wrong way."""
    rng = np.random.default_rng(seed)
    found = []
    dy = np.arange(0, 1 << 20, 419, dtype=np.int64)
    while len(found) < count:
        dx = rng.integers(1 << 18, 1 << 20, 2048, dtype=np.int64)
        d4 = 4 * (dx[:, None] ** 2 + dy[None, :] ** 2)
        o = np.floor(np.sqrt(d4.astype(np.float64))).astype(np.int64) | 1
        dist = np.minimum(np.abs(d4 - o * o), np.abs(d4 - (o - 2) * (o - 2)))
        dist = np.minimum(dist, np.abs(d4 - (o + 2) * (o + 2)))
        ii, jj = np.nonzero(dist <= 3)
        found += [(int(dx[i]), int(dy[j])) for i, j in zip(ii, jj)]
    return found[:count]


def test_exact_rounding_near_half_integers(ctx):
    """EUC_2D rounding (the integer cost of eq. 9) at lengths within 3/4 of a
    half-integer over the full 2^20 span: every Z = 2c at Lam = 0 of five-city
    instances (the origin and four such offsets; all ten pairs are in the
    top four) equals 2 nint(sqrt(D)) with nint from math.isqrt (k with
    (2k-1)^2 <= 4D < (2k+1)^2)."""
    import math
    pairs = _boundary_pairs(24, 5)
    for g in range(0, len(pairs), 4):
        xy = np.array([(0, 0)] + pairs[g:g + 4], dtype=np.int64)
        rec, h = gpu_step(ctx, xy, np.zeros(5, np.int64))
        for v in range(5):
            assert sorted(h["i4"][v].tolist()) == [u for u in range(5) if u != v]
            for j in range(4):
                u = int(h["i4"][v][j])
                d = int(((xy[v] - xy[u]) ** 2).sum())
                assert h["z4"][v][j] == 2 * ((math.isqrt(4 * d) + 1) // 2), (xy[v], xy[u])


@pytest.mark.parametrize("seed,div,scan", [(1, 0, "culled"), (2, 0, "culled"), (3, 0, "full"), (1, 300, "full"),
                                           (2, 50, "culled")])
def test_solve_trajectory_c1(ctx, seed, div, scan):
    # n = 1000, uniform in [0, 10^5)^2: the trajectory, the stop and Lam*
    xy = I.uniform(1000, 100000, seed)
    o = core.gdp_solve(xy, handoff_div=div)
    g = ctx.solve(xy, trace=True, finish="none", handoff_div=div, scan=scan)
    assert g["iterations"] == o["iters"] and g["stop"] == o["stop"] and g["kstar"] == o["kstar"]
    assert np.array_equal(g["trace"], o["trace"])
    assert np.array_equal(g["lambda2_gdp"], o["lam"])


@pytest.mark.parametrize("name,make", [("lattice_ties", lambda: I.lattice_jitter(32, 33, 40, 2, 7)),
                                       ("duplicates", lambda: I.with_duplicates(1500, 20000, 200, 8))])
def test_solve_trajectory_ties_with_lists(ctx, name, make):
    """Tie-heavy instances (jittered lattice; 200 duplicated cities, which
    run 136 iterations into a cycle stop) through the culled scan with
    candidate lists: many list entries share a row's bound, so candidate
    buffers fill up and rows walk their runs instead.  Every record, the
    stop, k* and Lam* equal the oracle's."""
    xy = make()
    o = core.gdp_solve(xy, handoff_div=0)
    g = ctx.solve(xy, trace=True, finish="none", handoff_div=0)
    print(name, "list iterations", g["scan_list_uses"], "builds", g["scan_list_builds"], flush=True)
    assert g["scan_list_uses"] > 0
    assert g["iterations"] == o["iters"] and g["stop"] == o["stop"] and g["kstar"] == o["kstar"]
    assert np.array_equal(g["trace"], o["trace"])
    assert np.array_equal(g["lambda2_gdp"], o["lam"])


@pytest.mark.parametrize("name,make", [("square", lambda: I.square4()), ("tri3", lambda: I.triangles(3)),
                                       ("c1", lambda: I.uniform(1000, 100000, 1)),
                                       ("lattice", lambda: I.lattice_jitter(20, 21, 40, 2, 3)),
                                       ("clustered", lambda: I.clustered(800, 1000000, 2, centres=20))])
def test_solve_certified_optimum(ctx, name, make):
    xy = make()
    g = ctx.solve(xy, trace=True)
    assert g["stop"] in ("trivial", "handoff", "fixed", "cycle")
    assert g["certified"] and g["status"] == "ok", g["status"]
    assert g["primal2"] == g["dual2"] == core.exact_opt2(xy)
    c = core.certify(xy, g["lambda2"], g["edge_u"], g["edge_v"], g["edge_x2"])
    assert c["certified"] and c["primal2"] == g["primal2"]
    from paper_2011_08170_amd import f2m
    o = core.gdp_solve(xy, handoff_div=f2m.HANDOFF_DIV)
    assert np.array_equal(g["trace"], o["trace"])


def test_certify_kernel_matches_oracle(ctx):
    rnd = np.random.default_rng(0)
    for n, seed in [(50, 1), (333, 2), (900, 3)]:
        xy = I.uniform(n, 20000, seed)
        opt2, x2, lam = core.exact_opt2(xy, want_x=True)
        eu, ev, ex = core.dense_to_edges(x2)
        variants = [(lam, eu, ev, ex), (lam + rnd.integers(-5, 6, n), eu, ev, ex),
                    (lam, eu[1:], ev[1:], ex[1:]), (lam, eu, ev, np.where(np.arange(len(ex)) == 0, 3 - ex, ex))]
        for lv, a, b, x in variants:
            o = core.certify(xy, lv, a, b, x)
            g = ctx.certify(dev(xy, np.int32), dev(lv, np.int64), dev(a, np.int32), dev(b, np.int32),
                            dev(x, np.uint8))
            assert g == o


def test_n3_and_errors(ctx):
    from paper_2011_08170_amd import f2m
    g = ctx.solve(np.array([[0, 0], [30, 0], [0, 40]], np.int32))
    assert g["certified"] and g["primal2"] == 240
    with pytest.raises(f2m.F2MError) as e:
        ctx.solve(np.array([[0, 0], [1, 1]], np.int32))
    assert e.value.status == -3
    with pytest.raises(f2m.F2MError) as e:
        ctx.solve(np.array([[0, 0], [1 << 20, 0], [5, 5], [7, 7]], np.int32))
    assert e.value.status == -2


@pytest.mark.parametrize("name,make", [("clustered_5000", lambda: I.clustered(5000, 1000000, 11)),
                                       ("uniform_12289", lambda: I.uniform(12289, 1000000, 12))])
def test_full_and_culled_scans_agree_with_oracle(ctx, name, make):
    # the full scan (every ordered pair) and the culled scan give the same
    # bits; both equal the oracle's first iterations
    xy = make()
    a = ctx.solve(xy, trace=True, finish="none", max_iters=6, scan="full")
    b = ctx.solve(xy, trace=True, finish="none", max_iters=6, scan="culled")
    assert np.array_equal(a["trace"], b["trace"]) and np.array_equal(a["lambda2_gdp"], b["lambda2_gdp"])
    n = len(xy)
    assert a["scan_pairs"] == a["iterations"] * n * (n - 1)
    assert 0 < b["scan_pairs"] < a["scan_pairs"]
    o = core.gdp_solve(xy, max_iters=6)
    assert np.array_equal(a["trace"], o["trace"])
    assert np.array_equal(a["lambda2_gdp"], o["lam"])


def test_device_coords_same_as_host(ctx):
    xy = I.uniform(600, 100000, 9)
    a = ctx.solve(xy, trace=True)
    b = ctx.solve(dev(xy, np.int32), trace=True)
    for k in ("trace", "lambda2", "edge_u", "edge_v", "edge_x2"):
        assert np.array_equal(a[k], b[k])


def test_repeat_bitwise(ctx):
    xy = I.clustered(1500, 1000000, 4)
    a = ctx.solve(xy, trace=True)
    b = ctx.solve(xy, trace=True)
    for k in ("trace", "lambda2", "edge_u", "edge_v", "edge_x2"):
        assert np.array_equal(a[k], b[k])


def test_c2_shape_sampled_rows(ctx):
    # n = 100000 uniform in [0, 10^6)^2, the benchmark's launch shape:
    # sampled rows of one iteration at a cold and a perturbed Lam
    xy = I.uniform(100000, 1000000, 1)
    n = len(xy)
    rows = np.random.default_rng(1).choice(n, 96, replace=False)
    rows = np.concatenate([rows, [0, n - 1]])
    rnd = np.random.default_rng(2)
    for lam in (np.zeros(n, np.int64), rnd.integers(0, 6000, n).astype(np.int64)):
        rec, g = gpu_step(ctx, xy, lam)
        o = core.gdp_rows(xy, lam, rows)
        assert np.array_equal(g["z4"][rows], o["z4"])
        assert np.array_equal(g["i4"][rows], o["i4"])
        assert np.array_equal(g["neg"][rows], o["neg"]) and np.array_equal(g["zero"][rows], o["zero"])
        assert np.array_equal(g["step"][rows], o["step"])
        assert rec["sum_lam"] == int(lam.sum())
        assert rec["hash"] == core.lam_hash(lam)


def test_sliced_culled_scan_with_lists_matches_oracle(ctx):
    # the culled scan split over several column slices keeps a candidate list
    # per slice: the trajectory equals the oracle's and the one-slice run's,
    # and list scans really ran
    from paper_2011_08170_amd import f2m
    xy = I.uniform(8000, 1000000, 21)
    o = core.gdp_solve(xy, handoff_div=f2m.HANDOFF_DIV)
    for shape in ((1, 1), (1, 4), (1, 3)):
        g = ctx.solve(xy, trace=True, finish="none", shape=shape)
        assert g["scan_slices"] == shape[1]
        assert g["scan_list_uses"] > 0 and (g["scan_kind"] == f2m.SCAN_KIND_LIST).sum() == g["scan_list_uses"]
        assert g["iterations"] == o["iters"] and g["stop"] == o["stop"] and g["kstar"] == o["kstar"]
        assert np.array_equal(g["trace"], o["trace"]), shape
        assert np.array_equal(g["lambda2_gdp"], o["lam"]), shape


def test_cycle_stop_matches_oracle(ctx):
    # 2-cycles of the rule (tests/golden/cycle_case.json): the GPU loop stops
    # with "cycle" at the same iteration, with the same largest-dual Lam*
    import json
    import os
    cases = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "cycle_case.json")))["cases"]
    for c in cases:
        xy = np.array(c["coords"], np.int32)
        lam0 = np.array(c["lam0"], np.int64)
        o = core.gdp_solve(xy, lam0=lam0, max_iters=200, handoff_div=0)
        for scan in ("culled", "full"):
            g = ctx.solve(xy, lambda2_init=lam0, trace=True, finish="none", handoff_div=0, max_iters=200,
                          scan=scan)
            assert g["stop"] == "cycle" == o["stop"]
            assert g["iterations"] == o["iters"] == c["stop_k"] + 1 and g["kstar"] == o["kstar"] == c["kstar"]
            assert np.array_equal(g["trace"], o["trace"])
            assert np.array_equal(g["lambda2_gdp"], o["lam"])


def test_resume_from_checkpoint_bitwise(ctx):
    # run to iteration K (cap), resume from lambda2_last with k0 = K and the
    # two previous hashes: records, stop, k*, Lam* and the certified result
    # equal the uninterrupted run's
    xy = I.clustered(6000, 1000000, 31)
    full = ctx.solve(xy, trace=True)
    K = full["iterations"] // 2
    part = ctx.solve(xy, trace=True, max_iters=K, finish="none")
    assert part["stop"] == "cap" and np.array_equal(part["trace"], full["trace"][:K + 1])
    h = (int(full["trace"][K - 1, 6]), int(full["trace"][K - 2, 6]))
    res = ctx.solve(xy, trace=True, lambda2_init=part["lambda2_last"], k0=K, resume_hash=h)
    assert res["stop"] == full["stop"] and res["kstar"] == full["kstar"]
    assert res["iterations"] == full["iterations"] - K
    assert np.array_equal(res["trace"], full["trace"][K:])
    for k in ("lambda2_gdp", "lambda2", "edge_u", "edge_v", "edge_x2"):
        assert np.array_equal(res[k], full[k]), k
    assert res["certified"] and res["primal2"] == full["primal2"]


def test_device_memory_cap(ctx):
    from paper_2011_08170_amd import f2m
    xy = I.uniform(20000, 1000000, 41)
    with f2m.Context(0, max_device_bytes=1 << 20) as small:
        with pytest.raises(f2m.F2MError) as e:
            small.solve(xy)
        assert e.value.status == -4
    # a per-call cap on a context that already holds more also refuses to grow
    g = ctx.solve(xy, max_device_bytes=1 << 40)
    assert g["certified"]


def test_c1_lists_ran(ctx):
    xy = I.uniform(1000, 100000, 1)
    g = ctx.solve(xy, trace=True, finish="none")
    print("C1 list scans", g["scan_list_uses"], "builds", g["scan_list_builds"], flush=True)
    assert g["scan_list_builds"] > 0
