"""CPU (float64) reference of the dispatch cost model -- TEST INFRASTRUCTURE ONLY.

The same network and parameter layout as the library's HIP kernels: for n_in
inputs, h hidden units and k outputs, a flat buffer
    mean[n_in], inv_std[n_in], W1[h][n_in], b1[h], W2[h][h], b2[h], W3[k][h], b3[k]
with x' = (x - mean) * inv_std, h1 = relu(W1 x' + b1), h2 = relu(W2 h1 + b2),
y = W3 h2 + b3, and the masked mean squared error
    L = (1/N) sum_i sum_k mask[i][k] (y[i][k] - t[i][k])^2   (N = set mask entries).
The gradient is derived by hand (chain rule).  Training sets the input
normalisation from the data (mean and population standard deviation of each
input, a standard deviation of zero read as one) and then takes full-batch
Adam steps (Kingma and Ba 2015, Algorithm 1: exponential moment estimates with
bias correction).

Pins (tests/test_oracle_mlp.py): the forward pass and the loss against a tiny
network evaluated by hand; the gradient against central finite differences
and a hand-computed bias gradient; the normalisation against hand-computed
moments; Adam against its constant-gradient property and a two-step example
worked out by hand; training against Adam's first-step property and a network
in which only the output bias can move.
"""

import numpy as np


def unpack(p, n_in, h, k):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    def take(size, shape):
        nonlocal o
        a = p[o:o + size].reshape(shape)
        o += size
        return a
    mean = take(n_in, (n_in,))
    istd = take(n_in, (n_in,))
    w1 = take(h * n_in, (h, n_in))
    b1 = take(h, (h,))
    w2 = take(h * h, (h, h))
    b2 = take(h, (h,))
    w3 = take(k * h, (k, h))
    b3 = take(k, (k,))
    assert o == p.size
    return mean, istd, w1, b1, w2, b2, w3, b3


def forward(p, x, n_in, h, k):
    mean, istd, w1, b1, w2, b2, w3, b3 = unpack(p, n_in, h, k)
    xn = (np.asarray(x, np.float64) - mean) * istd
    a1 = xn @ w1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ w2.T + b2
    h2 = np.maximum(a2, 0.0)
    y = h2 @ w3.T + b3
    return y, (xn, a1, h1, a2, h2)


def loss(p, x, t, mask, n_in, h, k):
    y, _ = forward(p, x, n_in, h, k)
    m = np.asarray(mask, bool)
    r = np.where(m, y - np.asarray(t, np.float64), 0.0)
    return float((r * r).sum() / m.sum())


def loss_grad(p, x, t, mask, n_in, h, k):
    """(L, dL/d(trainable parameters)) in buffer order (everything after the
    normalisation)."""
    _, _, w1, b1, w2, b2, w3, b3 = unpack(p, n_in, h, k)
    y, (xn, a1, h1, a2, h2) = forward(p, x, n_in, h, k)
    m = np.asarray(mask, bool)
    nobs = m.sum()
    r = np.where(m, y - np.asarray(t, np.float64), 0.0)
    L = float((r * r).sum() / nobs)
    dy = 2.0 * r / nobs
    gw3 = dy.T @ h2
    gb3 = dy.sum(0)
    dh2 = (dy @ w3) * (a2 > 0)
    gw2 = dh2.T @ h1
    gb2 = dh2.sum(0)
    dh1 = (dh2 @ w2) * (a1 > 0)
    gw1 = dh1.T @ xn
    gb1 = dh1.sum(0)
    g = np.concatenate([gw1.ravel(), gb1, gw2.ravel(), gb2, gw3.ravel(), gb3])
    return L, g


def normalisation(x):
    """(mean, inv_std) of every input column of x (population moments); a
    column whose variance is zero (below 1e-12) gets inv_std = 1."""
    x = np.asarray(x, np.float64)
    mean = x.mean(0)
    var = ((x - mean) ** 2).mean(0)
    sd = np.where(var > 1e-12, np.sqrt(np.maximum(var, 0.0)), 1.0)
    return mean, 1.0 / sd


def adam_step(w, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t >= 1 (Kingma and Ba 2015, Algorithm 1):
    first and second moment estimates, their bias-corrected values, then
    w - lr * m_hat / (sqrt(v_hat) + eps).  Returns (w, m, v)."""
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return np.asarray(w, np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def train(p, x, t, mask, n_in, h, k, epochs, lr, grads=None):
    """Sets the normalisation of p from x, then `epochs` full-batch Adam steps
    on the masked mean squared error (moments start at zero).  Returns the new
    parameter buffer and the loss before each step; each step's gradient is
    appended to `grads` when a list is given."""
    p = np.array(p, dtype=np.float64)
    mean, istd = normalisation(x)
    p[:n_in] = mean
    p[n_in:2 * n_in] = istd
    w = p[2 * n_in:].copy()
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    losses = []
    for step in range(1, epochs + 1):
        L, g = loss_grad(np.concatenate([p[:2 * n_in], w]), x, t, mask, n_in, h, k)
        losses.append(L)
        if grads is not None:
            grads.append(g)
        w, m, v = adam_step(w, g, m, v, step, lr)
    p[2 * n_in:] = w
    return p, losses
