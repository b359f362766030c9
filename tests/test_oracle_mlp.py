"""Pins of the FP64 reference of the warm-start network."""
import numpy as np

from oracle import mlp


def test_bf16_rounding_table():
    # bfloat16 keeps 8 significant bits; ties go to even
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -7, -2.5, 3.0e38, 1e-40])
    # 3e38 = 2^127 * 1.7632...: the nearest 8-bit significand is 1 + 98/128
    want = np.array([1.0, 1.0, 1.0 + 2 ** -6, 1.0 + 2 ** -7, -2.5, 2.0 ** 127 * (1 + 98 / 128)])
    got = mlp.bf16(vals)
    assert np.array_equal(got[:6], want)
    assert 0 < got[6] < 1e-40


def test_gradient_finite_differences():
    rng = np.random.default_rng(1)
    theta = mlp.init(3) * 0.7
    X = rng.uniform(0.2, 3.0, (40, 16))
    t = rng.normal(1.5, 0.5, 40)
    loss, g = mlp.loss_and_grad(theta, X, t, round_bf16=False)
    idx = rng.choice(mlp.N_PARAMS, 60, replace=False)
    idx = np.concatenate([idx, [mlp.N_PARAMS - 1, 0, 2048 + 5]])
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.N_PARAMS)
        e[i] = h
        fd = (mlp.loss_and_grad(theta + e, X, t, False)[0] - mlp.loss_and_grad(theta - e, X, t, False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_adamw_first_step():
    # after one step from m = v = 0 the bias-corrected update is
    # lr * g / (|g| + eps) + lr * wd * theta
    th = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -0.1, 0.0])
    new, m, v = mlp.adamw(th, g, np.zeros(3), np.zeros(3), 1, lr=0.01, wd=0.1)
    want = th - 0.01 * (g / (np.abs(g) + 1e-8) + 0.1 * th)
    assert np.allclose(new, want, rtol=0, atol=1e-12)
