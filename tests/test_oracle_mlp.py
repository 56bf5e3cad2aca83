"""Pins for the sketch-rank model oracle: exact GELU values, central finite
differences against the hand-written backward, hand-computed losses, the
first Adam step, and feature values of spectra with a closed form."""
import math

import numpy as np
import pytest

from oracle import mlp


def test_gelu_known_values():
    # GELU(x) = x * Phi(x): Phi(1) = 0.8413447460685429, Phi(-1) = 0.15865525393145707
    np.testing.assert_allclose(mlp.gelu(np.array([0.0, 1.0, -1.0])),
                               [0.0, 0.8413447460685429, -0.15865525393145707], atol=1e-15)
    assert mlp.gelu_grad(np.array([0.0]))[0] == pytest.approx(0.5, abs=1e-16)
    x = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(x), fd, atol=1e-9)


def test_pinball_hand_values():
    # u = t - y = [1, -1]: rho = [0.9 * 1, (0.9 - 1) * -1] = [0.9, 0.1] -> mean 0.5
    assert mlp.pinball(np.array([0.0, 3.0]), np.array([1.0, 2.0])) == pytest.approx(0.5, abs=1e-15)
    assert mlp.pinball(np.array([2.0]), np.array([2.0])) == 0.0


def test_backward_matches_central_differences():
    g = np.random.default_rng(0)
    theta = mlp.init_params(3) + 0.01 * g.standard_normal(mlp.N_PARAMS)
    x = g.standard_normal((7, mlp.N_IN))
    t = g.standard_normal(7) * 3
    # keep every sample away from the kink of the pinball loss
    y, _ = mlp.forward(theta, x)
    t = np.where(np.abs(t - y) < 0.1, t + 0.5, t)
    _, grad = mlp.loss_and_grad(theta, x, t)
    idx = g.choice(mlp.N_PARAMS, 60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.N_PARAMS)
        e[i] = h
        fd = (mlp.loss_and_grad(theta + e, x, t)[0] - mlp.loss_and_grad(theta - e, x, t)[0]) / (2 * h)
        assert grad[i] == pytest.approx(fd, rel=1e-6, abs=1e-10)


def test_first_adam_step_is_signed_lr():
    g = np.array([0.5, -2.0, 1e-3])
    th, m, v = mlp.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=1e-3)
    np.testing.assert_allclose(th, -1e-3 * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_features_closed_form():
    s = 10.0 ** (-np.arange(33, dtype=np.float64))      # L = 33: j_t = t
    f = mlp.features(s, 1024, 2, 1e-8)
    assert f[0] == pytest.approx(10 / 11) and f[1] == 0.5 and f[2] == pytest.approx(0.5)
    want = [max(-1.0, -t / 16.0) for t in range(32)]
    np.testing.assert_allclose(f[3:], want, atol=1e-15)


def test_sketch_rank_rule():
    assert mlp.sketch_rank(math.log2(100.0), 2048, 1024) == 192   # 150 + 32 = 182 -> 192
    assert mlp.sketch_rank(math.log2(1024.0) + 0.01, 2048, 1024) is None
    assert mlp.sketch_rank(9.9, 600, 1024) is None                # k = 1472 > 600 / 4
    assert mlp.sketch_rank(math.log2(320.0), 2048, 1024) == 512   # 480 + 32 -> 512 = n / 4
    assert mlp.sketch_rank(math.log2(330.0), 2048, 1024) is None  # 527 -> 544 > n / 4
    assert mlp.sketch_rank(5.0, 2048, 1024) == 96                 # 48 + 32 = 80 -> 96


def test_init_is_he_uniform_and_deterministic():
    a = mlp.init_params(0)
    b = mlp.init_params(0)
    np.testing.assert_array_equal(a, b)
    w1, b1, w2, b2, w3, b3 = mlp.unpack(a)
    assert np.abs(w1).max() <= math.sqrt(6 / 35) and np.abs(w2).max() <= math.sqrt(6 / 128)
    assert np.all(b1 == 0) and np.all(b2 == 0) and b3[0] == 0
    assert abs(w1.std() - math.sqrt(6 / 35) / math.sqrt(3)) < 0.02
