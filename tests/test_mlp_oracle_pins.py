"""Pins of the surrogate network's FP64 oracle (CPU only).

The backward pass is checked against central finite differences of the loss,
SiLU and its derivative against their closed forms, and the Adam update
against the published recursion evaluated by hand for a scalar parameter.
"""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as Q


def _net(seed, n_in=5, H=7, n_out=4, B=3):
    rng = np.random.default_rng(seed)
    theta = rng.standard_normal(Q.param_count(n_in, H, n_out)) * 0.5
    x = rng.standard_normal((B, n_in))
    t = rng.standard_normal((B, n_out))
    return theta, x, t, (n_in, H, n_out)


def test_param_layout():
    n_in, H, n_out = 33, 512, 16384
    assert Q.param_count(n_in, H, n_out) == 8685056          # 8.69 M parameters
    theta = np.arange(Q.param_count(3, 4, 2), dtype=np.float64)
    W1, b1, W2, b2, W3, b3 = Q.unpack(theta, 3, 4, 2)
    assert W1.shape == (4, 3) and W1[1, 0] == 3 and b1[0] == 12 and W2[0, 1] == 17 and b3[-1] == theta[-1]


def test_silu_closed_forms():
    z = np.array([-30.0, -2.0, -0.5, 0.0, 0.3, 4.0, 30.0])
    assert np.allclose(Q.silu(z), z * 0.5 * (1 + np.tanh(0.5 * z)), rtol=1e-12, atol=1e-14)   # 1 + tanh cancels at z = -30
    assert Q.silu(0.0) == 0.0 and Q.silu_grad(0.0) == 0.5
    h = 1e-6
    fd = (Q.silu(z + h) - Q.silu(z - h)) / (2 * h)
    assert np.allclose(Q.silu_grad(z), fd, rtol=1e-8, atol=1e-10)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_backward_matches_finite_differences(seed):
    theta, x, t, dims = _net(seed)
    L, g, dx = Q.backward(theta, x, t, *dims)
    assert abs(L - Q.loss(theta, x, t, *dims)) < 1e-15
    h = 1e-6
    for k in range(theta.size):
        e = np.zeros_like(theta)
        e[k] = h
        fd = (Q.loss(theta + e, x, t, *dims) - Q.loss(theta - e, x, t, *dims)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), k
    for b in range(x.shape[0]):
        for i in range(x.shape[1]):
            e = np.zeros_like(x)
            e[b, i] = h
            fd = (Q.loss(theta, x + e, t, *dims) - Q.loss(theta, x - e, t, *dims)) / (2 * h)
            assert abs(fd - dx[b, i]) <= 1e-6 * max(1.0, abs(dx[b, i]))


def test_loss_of_exact_fit_is_zero_and_gradient_vanishes():
    theta, x, _, dims = _net(4)
    y, _ = Q.forward(theta, x, *dims)
    L, g, dx = Q.backward(theta, x, y, *dims)
    assert L == 0.0 and np.all(g == 0.0) and np.all(dx == 0.0)


def test_adam_by_hand():
    """Scalar recursion of Kingma & Ba (2015), Algorithm 1, three steps."""
    th, m, v = np.array([1.0]), np.array([0.0]), np.array([0.0])
    grads = [0.5, -0.2, 0.1]
    lr = 1e-2
    want = 1.0
    mm = vv = 0.0
    for s, gval in enumerate(grads, start=1):
        th, m, v = Q.adam_step(th, np.array([gval]), m, v, s, lr)
        mm = 0.9 * mm + 0.1 * gval
        vv = 0.999 * vv + 0.001 * gval * gval
        want -= lr * (mm / (1 - 0.9 ** s)) / (math.sqrt(vv / (1 - 0.999 ** s)) + 1e-8)
        assert abs(th[0] - want) < 1e-15
    # the first step moves every coordinate by lr (times the sign of its gradient)
    t1, _, _ = Q.adam_step(np.zeros(3), np.array([3.0, -1e-3, 7.0]), np.zeros(3), np.zeros(3), 1, 0.1)
    assert np.allclose(t1, [-0.1, 0.1, -0.1], rtol=2e-5)   # eps shifts the smallest gradient by 1e-5
