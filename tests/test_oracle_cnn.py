"""Pins of the float64 warm-start network reference (no GPU): brute-force
correlation, identity and zero-layer special cases, central finite
differences of every gradient, and the closed-form first Adam step."""
import math

import numpy as np
import pytest

from oracle import cnn


def small_net(rng, channels=(3, 4, 4, 3)):
    params = []
    for l in range(len(channels) - 1):
        params.append({"w": rng.standard_normal((channels[l + 1], 3, 3, channels[l])) * 0.5,
                       "b": rng.standard_normal(channels[l + 1]) * 0.1})
    return params


def test_conv_matches_explicit_sums():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((5, 4, 3))
    w = rng.standard_normal((2, 3, 3, 3))
    b = rng.standard_normal(2)
    np.testing.assert_allclose(cnn.conv3x3(x, w, b), cnn.conv3x3_loops(x, w, b), rtol=1e-12, atol=1e-12)


def test_delta_kernel_is_identity():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((6, 5, 3))
    w = np.zeros((3, 3, 3, 3))
    for c in range(3):
        w[c, 1, 1, c] = 1.0
    np.testing.assert_array_equal(cnn.conv3x3(x, w, np.zeros(3)), x)


def test_tap_orientation():
    """w[co, t1, t2, ci] with t1 = 2 reads the neighbour at i1 + 1."""
    x = np.zeros((5, 5, 1))
    x[3, 2, 0] = 1.0
    w = np.zeros((1, 3, 3, 1))
    w[0, 2, 1, 0] = 1.0
    out = cnn.conv3x3(x, w, np.zeros(1))
    assert out[2, 2, 0] == 1.0 and out.sum() == 1.0


def test_zero_last_layer_returns_observation():
    rng = np.random.default_rng(2)
    params = cnn.init_params(rng)
    C = rng.standard_normal((8, 7, 3))
    X0, _ = cnn.forward(params, C)
    np.testing.assert_array_equal(X0, C)
    assert sum(p["w"].size + p["b"].size for p in params) == 38755


@pytest.mark.parametrize("seed", [3, 4])
def test_gradients_match_central_differences(seed):
    rng = np.random.default_rng(seed)
    params = small_net(rng)
    C = rng.standard_normal((5, 4, 3))
    Y = rng.standard_normal((5, 4, 3))
    X0, acts = cnn.forward(params, C)
    grads = cnn.backward(params, acts, Y)
    h = 1e-6
    for l, p in enumerate(params):
        for key in ("w", "b"):
            flat = p[key].reshape(-1)
            gflat = grads[l][key].reshape(-1)
            for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp = cnn.mse(cnn.forward(params, C)[0], Y)
                flat[idx] = old - h
                lm = cnn.mse(cnn.forward(params, C)[0], Y)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - gflat[idx]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (l, key, idx, fd, gflat[idx])


def test_input_gradient_of_conv_matches_differences():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((4, 5, 2))
    w = rng.standard_normal((3, 3, 3, 2))
    g = rng.standard_normal((4, 5, 3))
    _, _, dx = cnn.conv3x3_backward(x, w, g)
    h = 1e-6
    for idx in [(0, 0, 0), (2, 3, 1), (3, 4, 0)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (np.sum(g * cnn.conv3x3(xp, w, np.zeros(3))) - np.sum(g * cnn.conv3x3(xm, w, np.zeros(3)))) / (2 * h)
        np.testing.assert_allclose(dx[idx], fd, rtol=1e-7)


def test_first_adam_step_is_signed_learning_rate():
    """With zero moments the first update is lr * g / (|g| + eps)."""
    rng = np.random.default_rng(6)
    params = [{"w": rng.standard_normal(5), "b": rng.standard_normal(2)}]
    grads = [{"w": rng.standard_normal(5), "b": rng.standard_normal(2)}]
    before = [{k: v.copy() for k, v in p.items()} for p in params]
    opt = cnn.Adam(params, lr=1e-2)
    opt.step(params, grads)
    for k in ("w", "b"):
        g = grads[0][k]
        np.testing.assert_allclose(before[0][k] - params[0][k], 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_adam_constant_gradient_moves_by_signed_rate_every_step():
    """With a constant gradient g the bias-corrected moments are exactly g
    and g^2 at every step (m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2), so each
    of the steps moves by lr g / (|g| + eps)."""
    g = np.array([0.5, -2.0, 1e-3, 7.0])
    p = [{"w": np.array([1.0, 2.0, 3.0, 4.0])}]
    opt = cnn.Adam(p, lr=0.05)
    for t in range(1, 6):
        before = p[0]["w"].copy()
        opt.step(p, [{"w": g.copy()}])
        np.testing.assert_allclose(before - p[0]["w"], 0.05 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def test_adam_two_gradients_against_hand_worked_moments():
    """g = 1 then g = 3 on a scalar, lr 0.1, beta1 0.9, beta2 0.999.
    Step 1: m = 0.1, v = 0.001, corrections 0.1 and 0.001: the step is
    0.1 * 1 / (1 + eps).  Step 2: m = 0.9 * 0.1 + 0.1 * 3 = 0.39 and
    v = 0.999 * 0.001 + 0.001 * 9 = 0.009999, corrections 1 - 0.81 = 0.19 and
    1 - 0.998001 = 0.001999, so m_hat = 39/19 and v_hat = 9999/1999."""
    p = [{"w": np.array([0.0])}]
    opt = cnn.Adam(p, lr=0.1)
    opt.step(p, [{"w": np.array([1.0])}])
    np.testing.assert_allclose(p[0]["w"][0], -0.1 / (1.0 + 1e-8), rtol=1e-14)
    np.testing.assert_allclose(opt.m[0]["w"][0], 0.1, rtol=1e-14)
    np.testing.assert_allclose(opt.v[0]["w"][0], 0.001, rtol=1e-14)
    opt.step(p, [{"w": np.array([3.0])}])
    np.testing.assert_allclose(opt.m[0]["w"][0], 0.39, rtol=1e-14)
    np.testing.assert_allclose(opt.v[0]["w"][0], 0.009999, rtol=1e-13)
    step2 = 0.1 * (39.0 / 19.0) / (math.sqrt(9999.0 / 1999.0) + 1e-8)
    np.testing.assert_allclose(p[0]["w"][0], -0.1 / (1.0 + 1e-8) - step2, rtol=1e-13)
    # a different learning rate at step 3 scales only that step
    m3, v3 = 0.9 * 0.39 + 0.1 * (-1.0), 0.999 * 0.009999 + 0.001 * 1.0
    c1, c2 = 1.0 - 0.9 ** 3, 1.0 - 0.999 ** 3
    before = p[0]["w"][0]
    opt.step(p, [{"w": np.array([-1.0])}], lr=0.02)
    np.testing.assert_allclose(before - p[0]["w"][0], 0.02 * (m3 / c1) / (math.sqrt(v3 / c2) + 1e-8), rtol=1e-12)
