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
    yr, _ = mlp.forward(theta.astype(np.float64), X)
    assert rel(y.cpu().numpy(), yr) < 1e-3
    grad = torch.empty_like(th)
    loss = ctx.mlp_grad(th, fe, torch.from_numpy(t.astype(np.float32)).cuda(), grad)
    lr_, gr = mlp.loss_and_grad(theta.astype(np.float64), X, t.astype(np.float32).astype(np.float64))
    assert abs(loss - lr_) <= 1e-3 * lr_
    g = grad.cpu().numpy()
    o = 0
    for name, shape in mlp.SIZES:
        k = int(np.prod(shape))
        assert rel(g[o:o + k], gr[o:o + k]) < 1e-2, name
        o += k


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
    assert rel(th.cpu().numpy(), ref) < 1e-6


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
