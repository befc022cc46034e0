"""Pins of the learned-scorer reference: BF16 rounding, forward pass, gradients, Adam, features."""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp


def test_bf16_round_to_nearest_even():
    v = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, -2.5, 3.0e38])
    r = mlp.bf16_round(v)
    assert r[0] == 1.0
    assert r[1] == 1.0                 # halfway, ties to the even mantissa
    assert r[2] == 1 + 2 ** -6         # halfway, ties to the even mantissa
    assert r[3] == 1 + 2 ** -7         # above halfway rounds up
    assert r[4] == -2.5                # exactly representable
    assert abs(r[5] - 3.0e38) / 3.0e38 < 2 ** -8


def test_forward_closed_form():
    # hidden unit i < 12 copies feature i, layer 2 copies hidden i, output sums: logit = sum relu(f) + b3
    W1 = np.zeros((12, 64)); W1[np.arange(12), np.arange(12)] = 1.0
    W2 = np.zeros((64, 64)); W2[np.arange(12), np.arange(12)] = 1.0
    w3 = np.zeros(64); w3[:12] = 1.0
    theta = mlp.pack(dict(W1=W1, b1=np.zeros(64), W2=W2, b2=np.zeros(64), w3=w3, b3=[0.25]))
    X = np.array([[1.0, -2.0, 3.0] + [0.5] * 9, [-1.0] * 12])
    z, _ = mlp.forward(theta, X)
    assert z[0] == pytest.approx(1.0 + 3.0 + 4.5 + 0.25)
    assert z[1] == pytest.approx(0.25)
    # the C oracle's forward (used inside the tracker) is the same function
    for row in X:
        assert oracle.mlp_logit(theta, row) == pytest.approx(mlp.forward(theta, row[None])[0][0], rel=1e-14)


def random_theta(seed):
    rng = np.random.default_rng(seed)
    return mlp.pack(dict(W1=rng.normal(0, 0.5, (12, 64)), b1=rng.normal(0, 0.1, 64), W2=rng.normal(0, 0.2, (64, 64)),
                         b2=rng.normal(0, 0.1, 64), w3=rng.normal(0, 0.3, 64), b3=rng.normal(0, 0.1, 1)))


def test_c_and_numpy_forward_agree_on_random_nets():
    theta = random_theta(3)
    X = np.random.default_rng(4).normal(size=(50, 12))
    z, _ = mlp.forward(theta, X)
    zc = np.array([oracle.mlp_logit(theta, x) for x in X])
    assert np.allclose(z, zc, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_central_differences(seed):
    theta = random_theta(seed)
    rng = np.random.default_rng(10 + seed)
    X = rng.normal(size=(16, 12))
    y = (rng.uniform(size=16) < 0.5).astype(float)
    _, g = mlp.backward(theta, X, y)
    idx = np.concatenate([rng.choice(768, 40, replace=False), 768 + rng.choice(64, 10, replace=False),
                          832 + rng.choice(4096, 60, replace=False), 4928 + rng.choice(64, 10, replace=False),
                          4992 + rng.choice(64, 20, replace=False), [5056]])
    for i in idx:
        h = 1e-5
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h; tm[i] -= h
        num = (mlp.bce_loss(mlp.forward(tp, X)[0], y) - mlp.bce_loss(mlp.forward(tm, X)[0], y)) / (2 * h)
        assert abs(num - g[i]) <= 1e-7 * max(1e-3, abs(g[i])) + 1e-10, (i, num, g[i])


def test_bce_at_zero_logit_is_log2():
    assert mlp.bce_loss(np.zeros(7), np.array([0, 1, 1, 0, 1, 0, 0])) == pytest.approx(math.log(2.0))


def test_adam_first_step_is_lr_times_sign():
    theta = np.zeros(mlp.N_PARAMS)
    g = np.random.default_rng(5).normal(size=mlp.N_PARAMS)
    t1, m, v = mlp.adam_step(theta, np.zeros_like(g), np.zeros_like(g), g, 1, lr=1e-3)
    # bias-corrected m/sqrt(v) = g/|g| on the first step
    assert np.allclose(t1, -1e-3 * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8), rtol=1e-12)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_features_closed_form():
    # straight track in (x, y): curvature feature zero, chord slopes equal the track slopes
    xd, xm, xu = 100.0, 101.0, 102.0
    f = oracle.features(xd, 1.0, 5.0, xm, 1.5, 5.25, xu, 2.0, 5.5, 2.0, 2.0, 3, 1)
    assert f[0] == pytest.approx((100 - 166) / 81) and f[2] == pytest.approx((102 - 166) / 81)
    assert f[3] == pytest.approx(-0.5 / 2.0) and f[4] == pytest.approx(0.5 / 2.0)
    assert f[5] == pytest.approx(-0.25 / 2.0) and f[6] == pytest.approx(0.25 / 2.0)
    assert f[7] == pytest.approx(0.5) and f[8] == pytest.approx(0.25)
    assert f[9] == pytest.approx(0.0, abs=1e-15)
    assert f[10] == 0.75 and f[11] == 0.25
    # three points on a circle of radius 50: |curvature feature| = 10 * 2 / (2R) ... = 10 / R
    R = 50.0
    pts = [(R * math.cos(a), R * math.sin(a)) for a in (0.0, 0.02, 0.04)]
    f = oracle.features(pts[0][0], pts[0][1], 0, pts[1][0], pts[1][1], 0, pts[2][0], pts[2][1], 0, 2.0, 2.0, 0, 0)
    assert abs(f[9]) == pytest.approx(10.0 / R, rel=1e-9)
