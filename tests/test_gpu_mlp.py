"""Warm-start network on the GPU against the FP64 reference, and what the
trained network gains: the same certified optimum in fewer iterations."""
import os

import numpy as np
import pytest

from oracle import core, mlp
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


def bf16_to_f64(a16):
    return (a16.astype(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def rel(a, b):
    return np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30)


def test_features_match_reference(ctx):
    xy = I.clustered(3000, 1000000, 2, centres=30)
    d = torch.from_numpy(xy).cuda()
    feat = torch.empty((3000, 16), dtype=torch.int16, device="cuda")
    scale = ctx.features(d, feat)
    idx = core.knn(xy, 16)
    D = ((xy[:, None, :].astype(np.int64) - xy[idx]) ** 2).sum(-1)
    med = np.sort(D.ravel())[(D.size - 1) // 2]
    assert scale == np.float32(np.sqrt(np.float32(med)))
    want = mlp.bf16(np.sqrt(D.astype(np.float32)) * np.float32(1.0 / scale))
    got = bf16_to_f64(feat.cpu().numpy())
    assert np.max(np.abs(got - want) / np.maximum(want, 1e-6)) <= 2 ** -7


def flip_bound(v, err):
    """Largest change of bf16(v) when v moves by at most err (v >= 0): zero
    unless a rounding midpoint (or 0, through the ReLU) lies within err,
    else one bf16 ulp of the larger neighbour (plus err)."""
    v = np.abs(v)
    top = v + err
    e = np.floor(np.log2(np.maximum(top, 1e-300)))
    ulp = 2.0 ** (e - 7)
    q = v / ulp
    near_mid = np.abs((q - np.floor(q)) - 0.5) * ulp <= err + 1e-300
    near_edge = (v <= err) | (np.abs(v - 2.0 ** e) <= err)
    return np.where(near_mid | near_edge, ulp + err, err)


def bf16_bound_terms(theta, X):
    """Element-wise error bound of the GPU forward pass against the FP64
    reference, from the arithmetic.  Products of two bf16 values are exact in
    float32; a float32 sum of m terms errs by at most m 2^-24 times the sum of
    their magnitudes.  The GPU rounds the layer-1 activations to bf16 from
    float32, the reference from float64: an activation changes only where a
    rounding midpoint lies within the layer-1 error (flip_bound)."""
    p = mlp.unpack(theta.astype(np.float64))
    y, c = mlp.forward(theta.astype(np.float64), X)
    W1b = np.abs(mlp.bf16(p["W1"]))
    W2b = np.abs(mlp.bf16(p["W2"]))
    e1 = 17 * 2.0 ** -24 * (np.abs(c["x"]) @ W1b.T + np.abs(p["b1"]))
    dh1 = flip_bound(np.maximum(c["z1"], 0.0), e1)
    e2 = dh1 @ W2b.T + 129 * 2.0 ** -24 * (c["h1b"] @ W2b.T + np.abs(p["b2"]))
    ey = e2 @ np.abs(p["w3"]) + 130 * 2.0 ** -24 * (np.abs(c["h2"]) @ np.abs(p["w3"]) + abs(p["b3"][0]))
    return y, c, p, ey


def test_forward_and_gradient_match_reference(ctx):
    rng = np.random.default_rng(5)
    n = 3000
    theta = mlp.init(7).astype(np.float32)
    X = mlp.bf16(rng.uniform(0.3, 4.0, (n, 16)))
    t = rng.normal(1.2, 0.4, n)
    x16 = ((X.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)).view(np.int16)
    th = torch.from_numpy(theta).cuda()
    fe = torch.from_numpy(x16.copy()).cuda()
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    ctx.mlp_forward(th, fe, y)
    yr, c, p, tol_y = bf16_bound_terms(theta, X)
    gy = y.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(gy - yr) <= tol_y + 1e-6), np.max(np.abs(gy - yr) / tol_y)
    # the bound is tight where no activation can flip
    assert np.median(tol_y / np.maximum(np.abs(yr), 1e-9)) < 1e-2
    grad = torch.empty_like(th)
    loss = ctx.mlp_grad(th, fe, torch.from_numpy(t.astype(np.float32)).cuda(), grad)
    lr_, gr = mlp.loss_and_grad(theta.astype(np.float64), X, t.astype(np.float32).astype(np.float64))
    assert abs(loss - lr_) <= 2.0 * np.mean(np.abs(yr - t) * tol_y) + 1e-6 * lr_
    # element-wise gradient bounds: every gradient entry is a sum over the
    # rows of products of a back-propagated signal and an activation; the
    # signal's own error starts from |dy| <= 2 tol_y / n
    dyb = (2.0 * np.abs(yr - t) + 2.0 * tol_y) / n
    w3 = np.abs(p["w3"])
    m2 = c["z2"] > 0
    m1 = c["z1"] > 0
    a2 = np.outer(dyb, w3) * m2                      # |g2| plus its error
    a1 = (a2 @ np.abs(mlp.bf16(p["W2"]))) * m1       # |g1| plus its error
    k = 2.0 ** -5
    bound = {"w3": k * (c["h2"].T @ dyb) + np.abs(tol_y) @ dyb,
             "b3": np.array([k * dyb.sum()]),
             "W2": k * (a2.T @ c["h1b"]),
             "b2": k * a2.sum(0),
             "W1": k * (a1.T @ np.abs(c["x"])),
             "b1": k * a1.sum(0)}
    g = grad.cpu().numpy().astype(np.float64)
    o = 0
    for name, shape in mlp.SIZES:
        kk = int(np.prod(shape))
        d = np.abs(g[o:o + kk] - gr[o:o + kk])
        b = bound[name].ravel() + 1e-9
        assert np.all(d <= b), (name, float(np.max(d / b)))
        o += kk


def test_warm_start_rounding_and_trajectory(ctx):
    """Lam_0 = round-half-even(2 scale y) of the device's own features and
    network output, bit for bit; the GDP from it equals the oracle's GDP from
    that Lam_0 (every record), and Lam_0 sits within the rounding of the
    FP64 network's prediction."""
    from paper_2011_08170_amd import warm
    if not os.path.exists(WEIGHTS):
        pytest.skip("no trained weights file")
    theta = warm.load(WEIGHTS)
    n = 3000
    xy = I.uniform(n, 1000000, 17)
    d = torch.from_numpy(xy).cuda()
    feat = torch.empty((n, 16), dtype=torch.int16, device="cuda")
    scale = ctx.features(d, feat)
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    ctx.mlp_forward(theta, feat, y)
    yg = y.cpu().numpy()
    lam0 = np.rint(2.0 * np.float64(scale) * yg.astype(np.float64)).astype(np.int64)
    g = ctx.solve(d, mlp_theta=theta, trace=True, finish="none", handoff_div=0, max_iters=300)
    o = core.gdp_solve(xy, lam0=lam0, max_iters=300)
    assert g["iterations"] == o["iters"] and g["stop"] == o["stop"]
    assert np.array_equal(g["trace"], o["trace"])
    # against the FP64 network on the same (device) features
    X = bf16_to_f64(feat.cpu().numpy())
    yr, _, _, tol_y = bf16_bound_terms(theta.cpu().numpy().astype(np.float32), X)
    assert np.all(np.abs(lam0 - 2.0 * scale * yr) <= 0.5 + 2.0 * scale * tol_y + 1e-6)


def test_adamw_matches_reference(ctx):
    rng = np.random.default_rng(2)
    th0 = rng.normal(0, 1, 18817).astype(np.float32)
    g = rng.normal(0, 0.1, 18817).astype(np.float32)
    th = torch.from_numpy(th0.copy()).cuda()
    m = torch.zeros_like(th)
    v = torch.zeros_like(th)
    gt = torch.from_numpy(g).cuda()
    ref, rm, rv = th0.astype(np.float64), np.zeros(18817), np.zeros(18817)
    for step in (1, 2, 3):
        ctx.mlp_adamw(th, gt, m, v, step, 1e-3, 0.01)
        ref, rm, rv = mlp.adamw(ref, g.astype(np.float64), rm, rv, step, 1e-3, wd=0.01)
    # element-wise: float32 arithmetic of three steps, a few ulps of theta
    # plus the rounding of each step's ratio m / (sqrt(v) + eps) (< 2^-16 of lr)
    assert np.all(np.abs(th.cpu().numpy() - ref) <= 2.0 ** -20 * np.abs(ref) + 3 * 1e-3 * 2.0 ** -16)


WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2011_08170_amd",
                       "weights", "warm_mlp.npy")


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained weights file")
@pytest.mark.parametrize("kind", ["uniform", "clustered"])
def test_trained_warm_start_gains(ctx, kind):
    from paper_2011_08170_amd import warm
    theta = warm.load(WEIGHTS)
    xy = I.uniform(20000, 1000000, 3) if kind == "uniform" else I.clustered(20000, 1000000, 3)
    d = torch.from_numpy(xy).cuda()
    cold = ctx.solve(d)
    hot = ctx.solve(d, mlp_theta=theta)
    assert cold["certified"] and hot["certified"]
    assert hot["primal2"] == cold["primal2"]
    assert hot["iterations"] < cold["iterations"]
