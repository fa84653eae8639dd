"""Pins for the FP64 step-network reference (oracle/mlp.py).

Each test checks the reference against something other than itself: finite
differences, symmetry, special cases with closed forms, Adam's closed-form
first steps, vis-viva, exact decode values and the bfloat16 rounding rule.
"""
import numpy as np
import pytest

from oracle import mlp

MU = 398600.4418


def _theta(seed, bias=0.1):
    t = mlp.init_params(seed)
    p = mlp.unpack(t.copy())
    rng = np.random.default_rng(seed + 100)
    p["b1"][:] = rng.normal(0, bias, mlp.N_HID)
    p["b2"][:] = rng.normal(0, bias, mlp.N_HID)
    p["b3"][:] = 0.3
    return mlp.pack(p)


def _batch(seed, B):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, 1.2, (B, mlp.N_IN)), rng.normal(0, 1, B)


def test_param_count():
    assert mlp.N_PARAMS == 64 * 5 + 64 + 64 * 64 + 64 + 64 + 1 == 4609


def test_gradient_matches_central_differences():
    theta = _theta(1)
    X, t = _batch(2, 7)
    g = mlp.grad(theta, X, t)
    h = 1e-6
    fd = np.empty_like(theta)
    for k in range(theta.size):
        tp = theta.copy()
        tp[k] += h
        tm = theta.copy()
        tm[k] -= h
        fd[k] = (mlp.loss(tp, X, t) - mlp.loss(tm, X, t)) / (2 * h)
    scale = np.abs(g).max()
    assert scale > 1e-3
    np.testing.assert_allclose(g, fd, rtol=0, atol=1e-7 * scale)
    # no parameter group is silently zero
    p = mlp.unpack(g)
    for name in ("W1", "b1", "W2", "b2", "w3", "b3"):
        assert np.abs(p[name]).max() > 0, name


def test_hidden_unit_permutation_invariance():
    theta = _theta(3)
    X, t = _batch(4, 11)
    rng = np.random.default_rng(5)
    p1, p2 = rng.permutation(mlp.N_HID), rng.permutation(mlp.N_HID)
    p = mlp.unpack(theta.copy())
    q = {"W1": p["W1"][p1], "b1": p["b1"][p1], "W2": p["W2"][p2][:, p1],
         "b2": p["b2"][p2], "w3": p["w3"][p2], "b3": p["b3"]}
    theta_q = mlp.pack(q)
    y, _ = mlp.forward(theta, X)
    yq, _ = mlp.forward(theta_q, X)
    np.testing.assert_allclose(yq, y, rtol=1e-13, atol=1e-13)
    g = mlp.unpack(mlp.grad(theta, X, t))
    gq = mlp.unpack(mlp.grad(theta_q, X, t))
    np.testing.assert_allclose(gq["W2"], g["W2"][p2][:, p1], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(gq["W1"], g["W1"][p1], rtol=1e-12, atol=1e-14)


def test_dead_first_layer_gives_constant_output_and_zero_gradient():
    theta = _theta(6)
    p = mlp.unpack(theta.copy())
    p["W1"][:] = 0.0
    p["b1"][:] = -1.0
    theta = mlp.pack(p)
    X, t = _batch(7, 9)
    y, _ = mlp.forward(theta, X)
    expect = np.dot(p["w3"], np.maximum(p["b2"], 0.0)) + p["b3"][0]
    np.testing.assert_allclose(y, expect, rtol=1e-14)
    g = mlp.unpack(mlp.grad(theta, X, t))
    assert np.all(g["W1"] == 0) and np.all(g["b1"] == 0)
    # the output bias gradient is the mean residual times two
    np.testing.assert_allclose(g["b3"][0], 2 * np.mean(y - t), rtol=1e-12)


def test_positive_network_is_affine():
    rng = np.random.default_rng(8)
    p = {"W1": rng.uniform(0.1, 1, (64, 5)), "b1": rng.uniform(0.1, 1, 64),
         "W2": rng.uniform(0.1, 1, (64, 64)), "b2": rng.uniform(0.1, 1, 64),
         "w3": rng.uniform(-1, 1, 64), "b3": np.array([0.7])}
    theta = mlp.pack(p)
    x1, x2 = rng.uniform(0, 1, 5), rng.uniform(0, 1, 5)
    lam = 0.3
    ys, _ = mlp.forward(theta, np.stack([x1, x2, lam * x1 + (1 - lam) * x2]))
    np.testing.assert_allclose(ys[2], lam * ys[0] + (1 - lam) * ys[1], rtol=1e-12)


def test_adam_closed_form_first_steps():
    rng = np.random.default_rng(9)
    theta = rng.normal(0, 1, 50)
    g = rng.normal(0, 1e-2, 50)
    m = np.zeros(50)
    v = np.zeros(50)
    lr, eps = 1e-3, 1e-8
    th = theta
    for step in range(1, 6):
        # bias correction makes every step of a constant gradient lr * g / (|g| + eps)
        new, m, v = mlp.adam(th, m, v, g, step, lr, eps=eps)
        np.testing.assert_allclose(th - new, lr * g / (np.abs(g) + eps), rtol=1e-9)
        th = new
    # a gradient flip at step 2: m_hat = (0.9*0.1*g - 0.1*g)/(1-0.81), v_hat = g^2
    m = np.zeros(50)
    v = np.zeros(50)
    t1, m, v = mlp.adam(theta, m, v, g, 1, lr, eps=0.0)
    t2, m, v = mlp.adam(t1, m, v, -g, 2, lr, eps=0.0)
    mh = (0.9 * 0.1 - 0.1) / (1 - 0.81)
    np.testing.assert_allclose(t1 - t2, lr * mh * np.sign(g), rtol=1e-9)


def test_training_reaches_a_teacher():
    teacher = _theta(10, bias=0.3)
    rng = np.random.default_rng(11)
    X = rng.uniform(0, 1, (256, 5))
    t, _ = mlp.forward(teacher, X)
    theta = mlp.init_params(12)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = mlp.loss(theta, X, t)
    for step in range(1, 401):
        theta, m, v = mlp.adam(theta, m, v, mlp.grad(theta, X, t), step, 3e-3)
    assert mlp.loss(theta, X, t) < l0 / 100


def test_speed_feature_is_vis_viva_at_perigee():
    rng = np.random.default_rng(13)
    a = rng.uniform(6600, 42200, 100)
    e = rng.uniform(0, 0.7, 100)
    inc = rng.uniform(0, np.pi, 100)
    x = mlp.features(a, e, inc, MU)
    rp = a * (1 - e)
    np.testing.assert_allclose(x[:, 3] * mlp.A_SCALE_KM, rp, rtol=1e-15)
    vv = np.sqrt(MU * (2 / rp - 1 / a))
    np.testing.assert_allclose(x[:, 4] * mlp.V_SCALE_KMS, vv, rtol=1e-13)
    # circular: perigee radius = a, speed = sqrt(mu / a)
    xc = mlp.features([42164.0], [0.0], [0.0], MU)
    assert xc[0, 0] == 1.0 and xc[0, 3] == 1.0
    assert abs(xc[0, 4] * 8 - np.sqrt(MU / 42164.0)) < 1e-14


def test_decode_exact_values():
    y = np.array([0.0, 3.0, np.log2(5e-4), 40.0, np.nan, np.inf, -np.inf, -1.0])
    d = mlp.decode(y, 1e-3, 3_600_000)
    assert d.tolist() == [1000, 8000, 1, 3_600_000, 0, 0, 0, 500]
    assert mlp.decode(np.array([5.0]), 1e-3, 0).tolist() == [1]


def test_bf16_rounding_rule():
    u = 2.0 ** -7   # bf16 spacing in [1, 2)
    x = np.array([1.0, 1 + u / 2, 1 + 3 * u / 2, 1 + u / 2 + 2.0 ** -20, -1 - u / 2,
                  3.0e38, 1e-40])
    r = mlp.bf16(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                 # tie to even
    assert r[2] == 1 + 2 * u           # tie to even (upwards)
    assert r[3] == 1 + u               # above the tie
    assert r[4] == -1.0
    assert np.isinf(r[5]) or r[5] == pytest.approx(3.0e38, rel=2 ** -8)
    assert abs(r[6] - 1e-40) <= 2.0 ** -133


def test_bf16_forward_close_to_fp64():
    theta = _theta(14)
    X, _ = _batch(15, 500)
    y, _ = mlp.forward(theta, X)
    yb = mlp.forward_bf16(theta, X)
    assert np.all(np.abs(yb - y) <= 2e-2 * np.maximum(1.0, np.abs(y)))
    assert np.any(yb != y)
