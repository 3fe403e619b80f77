"""FP64 CPU oracle of the learned surrogate's network (forward, backward, Adam).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call this module; the GPU
library shares no code with it.

The surrogate maps crease parameters and the wavelength to the log-intensity
of the focal-plane ROI.  The paper names the deformations (introduction) but
gives no learned model; the model here is a plain multilayer perceptron

    z1 = W1 x + b1,  h1 = silu(z1)
    z2 = W2 h1 + b2, h2 = silu(z2)
    y  = W3 h2 + b3

with silu(z) = z / (1 + e^{-z}), trained on the mean squared error
``L = sum (y - t)^2 / (B * n_out)`` over a batch of B rows, and updated by Adam
(Kingma & Ba, 2015, Algorithm 1) with beta1 = 0.9, beta2 = 0.999, eps = 1e-8.

Parameters are one flat float vector in the order
``W1 [H, n_in], b1 [H], W2 [H, H], b2 [H], W3 [n_out, H], b3 [n_out]``
(row-major), the same layout the library uses.

Everything is float64 NumPy; the backward pass is the chain rule written out
layer by layer, pinned in the tests against central finite differences.
"""
from __future__ import annotations

import numpy as np

__all__ = ["param_count", "unpack", "silu", "silu_grad", "forward", "loss", "backward", "adam_step",
           "ADAM_BETA1", "ADAM_BETA2", "ADAM_EPS"]

ADAM_BETA1 = 0.9
ADAM_BETA2 = 0.999
ADAM_EPS = 1e-8


def param_count(n_in: int, H: int, n_out: int) -> int:
    return H * n_in + H + H * H + H + n_out * H + n_out


def unpack(theta: np.ndarray, n_in: int, H: int, n_out: int):
    """Views (W1, b1, W2, b2, W3, b3) of the flat parameter vector."""
    theta = np.asarray(theta, dtype=np.float64)
    sizes = [(H, n_in), (H,), (H, H), (H,), (n_out, H), (n_out,)]
    out, o = [], 0
    for s in sizes:
        n = int(np.prod(s))
        out.append(theta[o:o + n].reshape(s))
        o += n
    assert o == theta.size
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    """d/dz [z s(z)] = s(z) (1 + z (1 - s(z))), s the logistic function."""
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta, x, n_in, H, n_out):
    """Returns y [B, n_out] and the cache (z1, h1, z2, h2)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_in, H, n_out)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ W1.T + b1
    h1 = silu(z1)
    z2 = h1 @ W2.T + b2
    h2 = silu(z2)
    y = h2 @ W3.T + b3
    return y, (z1, h1, z2, h2)


def loss(theta, x, t, n_in, H, n_out) -> float:
    y, _ = forward(theta, x, n_in, H, n_out)
    d = y - np.asarray(t, dtype=np.float64)
    return float(np.sum(d * d) / d.size)


def backward(theta, x, t, n_in, H, n_out):
    """(loss, grad of the flat parameters, grad of the inputs)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_in, H, n_out)
    x = np.asarray(x, dtype=np.float64)
    y, (z1, h1, z2, h2) = forward(theta, x, n_in, H, n_out)
    d = y - np.asarray(t, dtype=np.float64)
    L = float(np.sum(d * d) / d.size)
    dy = 2.0 * d / d.size                 # dL/dy
    gW3 = dy.T @ h2
    gb3 = dy.sum(axis=0)
    dh2 = dy @ W3
    dz2 = dh2 * silu_grad(z2)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2
    dz1 = dh1 * silu_grad(z1)
    gW1 = dz1.T @ x
    gb1 = dz1.sum(axis=0)
    dx = dz1 @ W1
    g = np.concatenate([a.ravel() for a in (gW1, gb1, gW2, gb2, gW3, gb3)])
    return L, g, dx


def adam_step(theta, g, m, v, step: int, lr: float):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = ADAM_BETA1 * m + (1.0 - ADAM_BETA1) * g
    v = ADAM_BETA2 * v + (1.0 - ADAM_BETA2) * g * g
    mhat = m / (1.0 - ADAM_BETA1 ** step)
    vhat = v / (1.0 - ADAM_BETA2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + ADAM_EPS), m, v
