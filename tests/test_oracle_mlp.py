"""Pins for the CPU reference of the cost model: the hand-derived gradient
against central finite differences of the loss, and the forward pass against
a direct per-sample evaluation."""

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


def test_forward_per_sample():
    n_in, h, k = 4, 6, 3
    p = params(n_in, h, k, 7)
    x = np.random.default_rng(8).normal(0, 1, (5, n_in))
    y, _ = mlp.forward(p, x, n_in, h, k)
    mean, istd, w1, b1, w2, b2, w3, b3 = mlp.unpack(p, n_in, h, k)
    for i in range(5):
        xn = [(x[i, d] - mean[d]) * istd[d] for d in range(n_in)]
        h1 = [max(0.0, sum(w1[a, d] * xn[d] for d in range(n_in)) + b1[a]) for a in range(h)]
        h2 = [max(0.0, sum(w2[a, c] * h1[c] for c in range(h)) + b2[a]) for a in range(h)]
        for o in range(k):
            assert y[i, o] == pytest.approx(sum(w3[o, c] * h2[c] for c in range(h)) + b3[o])
