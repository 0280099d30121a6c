"""FP64 numpy reference of the surrogate network (forward, loss, gradient).

TEST INFRASTRUCTURE, like the rest of ``oracle/``: only the tests use it.  It
restates the network of ``include/tled_surrogate.h`` in plain numpy double
precision, from the same parameter vector and frequency matrix, so that the GPU
gradients can be checked.  It shares no code with the library.
"""
from __future__ import annotations

import numpy as np


def layout(n_param, n_freq, width, depth, n_out):
    """[(W slice, W shape, b slice)] in the library's parameter order; K0 = padded input width."""
    K0 = ((2 * n_freq + n_param + 31) // 32) * 32
    out, off, fan = [], 0, K0
    for l in range(depth + 1):
        o = width if l < depth else n_out
        out.append((slice(off, off + o * fan), (o, fan), slice(off + o * fan, off + o * fan + o)))
        off += o * fan + o
        fan = width
    return out, K0, off


def features(x, p, B, K0):
    a = 2.0 * np.pi * x @ B.T
    f = np.concatenate([np.sin(a), np.cos(a), p], axis=1)
    return np.concatenate([f, np.zeros((len(x), K0 - f.shape[1]))], axis=1)


def silu(z):
    return z / (1.0 + np.exp(-z))


def forward(theta, x, p, B, cfg):
    lay, K0, _ = layout(**cfg)
    a = features(x, p, B, K0)
    zs, acts = [], [a]
    for l, (ws, wsh, bs) in enumerate(lay):
        z = a @ theta[ws].reshape(wsh).T + theta[bs]
        if l < len(lay) - 1:
            zs.append(z)
            a = silu(z)
            acts.append(a)
        else:
            return z, zs, acts


def loss_and_grad(theta, x, p, target, B, cfg):
    """Mean squared error over samples and outputs and its gradient (FP64)."""
    lay, K0, P = layout(**cfg)
    y, zs, acts = forward(theta, x, p, B, cfg)
    n, no = target.shape
    d = y - target
    loss = float((d * d).sum() / (n * no))
    g = np.zeros(P)
    dz = 2.0 * d / (n * no)
    for l in range(len(lay) - 1, -1, -1):
        ws, wsh, bs = lay[l]
        g[ws] = (dz.T @ acts[l]).ravel()
        g[bs] = dz.sum(0)
        if l > 0:
            da = dz @ theta[ws].reshape(wsh)
            z = zs[l - 1]
            s = 1.0 / (1.0 + np.exp(-z))
            dz = da * s * (1.0 + z * (1.0 - s))
    return loss, g


def grad_magnitude(theta, x, p, target, B, cfg):
    """Per-parameter magnitude of the gradient's terms, sum_n |dz_ni| |a_nj| for weights and
    sum_n |dz_ni| for biases (FP64): the scale against which a low-precision evaluation of the
    same sums is judged element by element."""
    lay, K0, P = layout(**cfg)
    y, zs, acts = forward(theta, x, p, B, cfg)
    n, no = target.shape
    dz = 2.0 * (y - target) / (n * no)
    m = np.zeros(P)
    for l in range(len(lay) - 1, -1, -1):
        ws, wsh, bs = lay[l]
        m[ws] = (np.abs(dz).T @ np.abs(acts[l])).ravel()
        m[bs] = np.abs(dz).sum(0)
        if l > 0:
            da = dz @ theta[ws].reshape(wsh)
            z = zs[l - 1]
            s = 1.0 / (1.0 + np.exp(-z))
            dz = da * s * (1.0 + z * (1.0 - s))
    return m
