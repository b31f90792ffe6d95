"""Pins for the CPU reference of the cost model (oracle/mlp.py).

Every function is checked against something other than itself: the forward
pass and the loss against a tiny network worked out by hand, the gradient
against central finite differences and a hand-computed bias gradient, the
normalisation against hand-computed moments, Adam (Kingma and Ba 2015,
Algorithm 1) against a two-step example worked out by hand and its
constant-gradient property, and training against Adam's first-step property
and a network in which only the output bias can move."""

import math

import numpy as np
import pytest

from oracle import mlp


def params(n_in, h, k, seed):
    rng = np.random.default_rng(seed)
    size = 2 * n_in + h * n_in + h + h * h + h + k * h + k
    p = rng.normal(0, 0.5, size)
    p[:n_in] = rng.normal(0, 1, n_in)           # mean
    p[n_in:2 * n_in] = rng.uniform(0.5, 2, n_in)  # inv_std
    return p


# A 2 -> 2 -> 2 -> 2 network with small integer weights, in buffer order:
#   mean = (1, 2), inv_std = (1, 1/2)
#   W1 = [[1, 2], [-1, 1]], b1 = (0, -1)
#   W2 = [[1, 1], [2, -3]], b2 = (1, 0)
#   W3 = [[1, -1], [0, 2]], b3 = (1/2, -1)
HAND = np.array([1, 2, 1, 0.5,
                 1, 2, -1, 1, 0, -1,
                 1, 1, 2, -3, 1, 0,
                 1, -1, 0, 2, 0.5, -1], np.float64)
# Worked by hand:
#   x = (3, 6):  x' = (2, 2);   W1 x' + b1 = (6, -1) -> h1 = (6, 0);
#                W2 h1 + b2 = (7, 12) -> h2 = (7, 12);  y = (7 - 12 + 1/2, 24 - 1)
#   x = (0, 0):  x' = (-1, -1); (-3, -1) -> h1 = (0, 0); (1, 0) -> h2 = (1, 0);  y = (3/2, -1)
#   x = (-1, 6): x' = (-2, 2);  (2, 3) -> h1 = (2, 3); (6, -5) -> h2 = (6, 0);   y = (13/2, -1)
HAND_X = np.array([[3, 6], [0, 0], [-1, 6]], np.float64)
HAND_Y = np.array([[-4.5, 23], [1.5, -1], [6.5, -1]], np.float64)


def test_forward_by_hand():
    # catches a transposed weight matrix, scaling before centring, a missing
    # ReLU on either layer or a bias dropped from any layer
    y, _ = mlp.forward(HAND, HAND_X, 2, 2, 2)
    assert np.array_equal(y, HAND_Y)


def test_loss_and_bias_gradient_by_hand():
    t = HAND_Y + np.array([[0, -3], [-1, 0], [0, 0]])   # residuals (0, 3), (1, 0), (0, 0)
    full = np.ones((3, 2), bool)
    # L = (0 + 9 + 1 + 0 + 0 + 0) / 6
    assert mlp.loss(HAND, HAND_X, t, full, 2, 2, 2) == pytest.approx(10 / 6, rel=1e-15)
    L, g = mlp.loss_grad(HAND, HAND_X, t, full, 2, 2, 2)
    # dL/db3 = (2 / N) * sum of residuals per output = (2/6) * (1, 3)
    assert g[-2:] == pytest.approx([1 / 3, 1.0], rel=1e-15)
    # masked: entry (0, 1) left out -> L = 1 / 5, dL/db3 = (2/5) * (1, 0)
    m = full.copy()
    m[0, 1] = False
    L, g = mlp.loss_grad(HAND, HAND_X, t, m, 2, 2, 2)
    assert L == pytest.approx(0.2, rel=1e-15)
    assert g[-2:] == pytest.approx([0.4, 0.0], abs=1e-15)


@pytest.mark.parametrize("n_in,h,k,b,seed", [(8, 32, 9, 40, 1), (3, 5, 4, 7, 2), (8, 16, 9, 1, 3)])
def test_gradient_matches_finite_differences(n_in, h, k, b, seed):
    rng = np.random.default_rng(seed + 100)
    p = params(n_in, h, k, seed)
    x = rng.normal(0, 2, (b, n_in))
    t = rng.normal(0, 1, (b, k))
    mask = rng.random((b, k)) < 0.5
    mask[0, 0] = True
    L, g = mlp.loss_grad(p, x, t, mask, n_in, h, k)
    assert L == pytest.approx(mlp.loss(p, x, t, mask, n_in, h, k))
    eps = 1e-6
    off = 2 * n_in
    for j in range(g.size):
        q = p.copy(); q[off + j] += eps
        lp = mlp.loss(q, x, t, mask, n_in, h, k)
        q[off + j] -= 2 * eps
        lm = mlp.loss(q, x, t, mask, n_in, h, k)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[j]) <= 1e-6 + 1e-5 * abs(fd), j


def test_normalisation_by_hand():
    # column 0: 2, 4, 6, 8 -> mean 5, deviations -3, -1, 1, 3 -> variance 20/4 = 5
    # column 1: constant 7 -> variance 0 -> inv_std 1
    # column 2: -1, 1, -1, 1 -> mean 0, variance 1
    x = np.array([[2, 7, -1], [4, 7, 1], [6, 7, -1], [8, 7, 1]], np.float64)
    mean, istd = mlp.normalisation(x)
    assert mean == pytest.approx([5, 7, 0], abs=1e-15)
    assert istd == pytest.approx([1 / math.sqrt(5), 1, 1], rel=1e-15)


def test_adam_two_steps_by_hand():
    # lr 0.1, beta (0.9, 0.999), eps 1e-8, w0 = 0, gradients 1 then 3.
    # step 1: m = 0.1, v = 0.001; m_hat = 1, v_hat = 1; w1 = -0.1 / (1 + 1e-8)
    # step 2: m = 0.09 + 0.3 = 0.39, v = 0.000999 + 0.009 = 0.009999;
    #         m_hat = 0.39 / 0.19 = 39/19, v_hat = 0.009999 / 0.001999 = 9999/1999;
    #         w2 = w1 - 0.1 * (39/19) / (sqrt(9999/1999) + 1e-8)
    w, m, v = mlp.adam_step(np.zeros(1), [1.0], np.zeros(1), np.zeros(1), 1, 0.1)
    assert m[0] == pytest.approx(0.1, rel=1e-15) and v[0] == pytest.approx(0.001, rel=1e-13)
    assert w[0] == pytest.approx(-0.09999999900000001, rel=1e-14)
    w, m, v = mlp.adam_step(w, [3.0], m, v, 2, 0.1)
    assert m[0] == pytest.approx(0.39, rel=1e-14) and v[0] == pytest.approx(0.009999, rel=1e-13)
    assert w[0] == pytest.approx(-0.19177811048766837, rel=1e-13)


def test_adam_constant_gradient_steps_by_the_rate():
    # with a constant gradient both bias-corrected moments are exact (g and
    # g^2), so every step moves each weight by lr * |g| / (|g| + eps) against
    # the sign of g; an uncorrected first step would move it sqrt(1000)/10
    # times as far
    g = np.array([2.5, -0.25, 1e-3, -40.0])
    w, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    for t in range(1, 21):
        w, m, v = mlp.adam_step(w, g, m, v, t, 0.01)
        step = 0.01 * np.abs(g) / (np.abs(g) + 1e-8)
        assert w == pytest.approx(-np.sign(g) * step * t, rel=1e-9)


def test_training_first_step_and_frozen_normalisation():
    n_in, h, k = 3, 5, 4
    rng = np.random.default_rng(11)
    p = params(n_in, h, k, 12)
    x = rng.normal(1, 3, (20, n_in))
    t = rng.normal(0, 1, (20, k))
    mask = rng.random((20, k)) < 0.7
    q, losses = mlp.train(p, x, t, mask, n_in, h, k, epochs=1, lr=0.01)
    mean, istd = mlp.normalisation(x)
    assert np.array_equal(q[:n_in], mean) and np.array_equal(q[n_in:2 * n_in], istd)
    p0 = p.copy()
    p0[:n_in], p0[n_in:2 * n_in] = mean, istd
    L0, g0 = mlp.loss_grad(p0, x, t, mask, n_in, h, k)
    # the first loss is taken after the normalisation is set, and Adam's first
    # step moves each trainable weight by lr * |g| / (|g| + eps) against g
    assert losses == [pytest.approx(L0, rel=1e-15)]
    expect = p0[2 * n_in:] - 0.01 * g0 / (np.abs(g0) + 1e-8)
    assert q[2 * n_in:] == pytest.approx(expect, rel=1e-12, abs=1e-15)


def test_training_moves_only_what_has_a_gradient():
    # all weights and hidden biases zero: h1 = h2 = 0 and y = b3 for every
    # sample, so only b3 has a gradient; b3 approaches the masked mean target
    # of each output and nothing else moves
    n_in, h, k = 2, 3, 2
    p = np.zeros(2 * n_in + h * n_in + h + h * h + h + k * h + k)
    x = np.array([[0.0, 1.0], [1.0, 3.0], [2.0, 5.0]])
    t = np.array([[1.0, -2.0], [2.0, -2.0], [3.0, 9.0]])
    mask = np.array([[1, 1], [1, 1], [1, 0]], bool)    # targets' masked means 2 and -2
    q, losses = mlp.train(p, x, t, mask, n_in, h, k, epochs=3000, lr=0.01)
    assert np.all(q[2 * n_in:-k] == 0.0)
    assert q[-k:] == pytest.approx([2.0, -2.0], abs=1e-3)
    # at b3 = masked means the loss is the masked variance: (1 + 0 + 1 + 0 + 0) / 5
    assert losses[-1] == pytest.approx(0.4, abs=1e-4)
