"""Oracle parity at the benchmark-scale configurations, through the C ABI:

* n = 100,000 uniform in [0,10^6)^2: full iteration records of the oracle at
  GPU iterates inside the stretch of candidate-list scans;
* n = 200,000 clustered (200 Gaussian centres, sigma 2% of the side): rows
  of the complete-graph iteration at a cold and at the final Lam, and the
  whole trajectory on the 10-nearest-neighbour candidate graph;
* 512 instances, n log-uniform in [1000, 20000], half uniform, half
  clustered (batch seed 2026): every result re-certified by the oracle and
  16 trajectories (the largest among them) equal to the oracle's;
* the learned warm start at n = 20,000: Lam_0 = round-half-even(2 s y) from
  the library's own features and network, and the trajectory from it.

Every comparison is exact (integer method)."""
import os

import numpy as np
import pytest

from oracle import core
from paper_2011_08170_amd import instances as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
M64 = (1 << 64) - 1


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


def gpu_step(ctx, xy_d, lam):
    n = xy_d.shape[0]
    out = dict(lam=torch.empty(n, dtype=torch.int64, device="cuda"),
               z4=torch.empty(4 * n, dtype=torch.int64, device="cuda"),
               i4=torch.empty(4 * n, dtype=torch.int32, device="cuda"),
               neg=torch.empty(n, dtype=torch.int32, device="cuda"),
               zero=torch.empty(n, dtype=torch.int32, device="cuda"),
               step=torch.empty(n, dtype=torch.int64, device="cuda"))
    rec = ctx.gdp_step(xy_d, dev(lam, np.int64), out["lam"], out["z4"], out["i4"], out["neg"], out["zero"],
                       out["step"])
    h = {k: v.cpu().numpy() for k, v in out.items()}
    h["z4"] = h["z4"].reshape(n, 4)
    h["i4"] = h["i4"].reshape(n, 4)
    return rec, h


def record_row(o):
    r = o["rec"]
    return [r["dual2"], r["unsat"], r["bad"], r["max_step"], r["nonzero"], r["hash"], r["sum_lam"]]


def test_c2_list_scans_against_oracle(ctx):
    from paper_2011_08170_amd import f2m
    xy = I.uniform(100000, 1000000, 1)
    xy_d = dev(xy, np.int32)
    full = ctx.solve(xy_d, trace=True, finish="none")
    kinds = full["scan_kind"]
    listed = np.nonzero(kinds == f2m.SCAN_KIND_LIST)[0]
    assert full["scan_list_uses"] == len(listed) > 0
    assert full["scan_list_builds"] == int((kinds == f2m.SCAN_KIND_BUILD).sum()) > 0
    ks = sorted({int(listed[0]), int(listed[len(listed) // 2]), int(listed[-1])})
    ks = [k for k in ks if k + 1 < full["iterations"]]
    assert ks
    for j, k in enumerate(ks):
        print("C2 list iteration", k, flush=True)
        # Lam_k from a run capped at k (same trajectory up to k)
        part = ctx.solve(xy_d, trace=True, finish="none", max_iters=k)
        assert part["stop"] == "cap" and part["iterations"] == k + 1
        assert np.array_equal(part["trace"], full["trace"][:k + 1])
        lam_k = part["lambda2_last"]
        assert core.lam_hash(lam_k) == int(full["trace"][k, 6]) & M64
        o = core.gdp_iter(xy, lam_k)
        want = record_row(o)
        got = [int(x) for x in full["trace"][k, 1:]]
        got[5] &= M64
        assert got == want, k
        assert core.lam_hash(lam_k + o["step"]) == int(full["trace"][k + 1, 6]) & M64
        if j == 0:
            # the one-iteration entry point at this real iterate
            rec, g = gpu_step(ctx, xy_d, lam_k)
            assert np.array_equal(g["z4"], o["z4"]) and np.array_equal(g["i4"], np.where(o["i4"] < 0, -1, o["i4"]))
            assert np.array_equal(g["neg"], o["neg"]) and np.array_equal(g["zero"], o["zero"])
            assert np.array_equal(g["step"], o["step"]) and np.array_equal(g["lam"], lam_k + o["step"])


def test_c3_clustered_200k(ctx):
    from paper_2011_08170_amd import f2m
    xy = I.clustered(200000, 1000000, 1)
    n = len(xy)
    xy_d = dev(xy, np.int32)
    # complete graph: the final Lam of a solve, then sampled rows of one
    # iteration there and at Lam = 0
    sol = ctx.solve(xy_d, finish="none")
    rows = np.concatenate([np.random.default_rng(5).choice(n, 254, replace=False), [0, n - 1]])
    for lam in (np.zeros(n, np.int64), sol["lambda2_gdp"]):
        rec, g = gpu_step(ctx, xy_d, lam)
        o = core.gdp_rows(xy, lam, rows)
        assert np.array_equal(g["z4"][rows], o["z4"]) and np.array_equal(g["i4"][rows], o["i4"])
        assert np.array_equal(g["neg"][rows], o["neg"]) and np.array_equal(g["zero"][rows], o["zero"])
        assert np.array_equal(g["step"][rows], o["step"])
        assert rec["hash"] == core.lam_hash(lam) and rec["sum_lam"] == int(lam.sum())
    # candidate graph: the CSR's sampled rows against the oracle's k nearest,
    # then the whole GDP trajectory on that graph
    rowptr, col = f2m.knn_graph(ctx, xy_d, 10)
    knn = core.knn_rows(xy, 10, rows)
    for i, v in enumerate(rows):
        mine = set(col[rowptr[v]:rowptr[v + 1]].tolist())
        assert set(knn[i].tolist()) <= mine
    g = ctx.solve(xy_d, graph="knn", trace=True, finish="none")
    o = core.gdp_solve(xy, handoff_div=f2m.HANDOFF_DIV, graph=(rowptr, col))
    assert g["iterations"] == o["iters"] and g["stop"] == o["stop"] and g["kstar"] == o["kstar"]
    assert np.array_equal(g["trace"], o["trace"])
    assert np.array_equal(g["lambda2_gdp"], o["lam"])


def test_c4_batch_512(ctx):
    from paper_2011_08170_amd import f2m
    sizes = I.batch_sizes(512, 1000, 20000, 2026)
    xy, off = I.batch(512, 1000, 20000, 2026)
    assert np.array_equal(np.diff(off), sizes)
    st, res = ctx.solve_batch(xy, off, trace=True)
    assert st == "ok" and len(res) == 512
    parts = [xy[off[i]:off[i + 1]] for i in range(512)]
    for i, (part, r) in enumerate(zip(parts, res)):
        assert r["certified"], i
        c = core.certify(part, r["lambda2"], r["edge_u"], r["edge_v"], r["edge_x2"])
        assert c["certified"] and c["primal2"] == r["primal2"] and c["dual2"] == r["dual2"], i
    big = int(np.argmax(sizes))
    pick = [big] + [int(i) for i in np.random.default_rng(2026).choice(
        [i for i in range(512) if i != big], 15, replace=False)]
    for i in pick:
        o = core.gdp_solve(parts[i], handoff_div=f2m.HANDOFF_DIV)
        r = res[i]
        assert r["iterations"] == o["iters"] and r["stop"] == o["stop"] and r["kstar"] == o["kstar"], i
        assert np.array_equal(r["trace"], o["trace"]), i
        assert np.array_equal(r["lambda2_gdp"], o["lam"]), i


def test_c5_warm_start_lam0_and_trajectory(ctx):
    from paper_2011_08170_amd import f2m, warm
    if not os.path.exists(warm.DEFAULT_WEIGHTS):
        pytest.skip("no trained warm-start weights")
    theta = warm.load()
    xy = I.clustered(20000, 1000000, 3)
    n = len(xy)
    xy_d = dev(xy, np.int32)
    feat = torch.empty((n, 16), dtype=torch.int16, device="cuda")
    scale = ctx.features(xy_d, feat)
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    ctx.mlp_forward(theta, feat, y)
    yh = y.cpu().numpy().astype(np.float64)
    # round half to even of 2 s y in double precision, clamped to 2^37
    lam0 = np.clip(np.rint((2.0 * np.float64(np.float32(scale))) * yh), -(1 << 37), 1 << 37).astype(np.int64)
    g = ctx.solve(xy_d, mlp_theta=theta, trace=True, finish="none")
    u = ctx.solve(xy_d, lambda2_init=lam0, trace=True, finish="none")
    assert np.array_equal(g["trace"], u["trace"]) and np.array_equal(g["lambda2_gdp"], u["lambda2_gdp"])
    assert int(g["trace"][0, 6]) & M64 == core.lam_hash(lam0) and g["trace"][0, 7] == lam0.sum()
    o = core.gdp_solve(xy, lam0=lam0, handoff_div=f2m.HANDOFF_DIV)
    assert g["iterations"] == o["iters"] and g["stop"] == o["stop"] and g["kstar"] == o["kstar"]
    assert np.array_equal(g["trace"], o["trace"])
    assert np.array_equal(g["lambda2_gdp"], o["lam"])
