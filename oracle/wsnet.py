"""FP64 reference of the per-contact warm-start network and of its training
loss and gradient.

TEST INFRASTRUCTURE ONLY: tests compare the GPU training kernels with these
functions; the product path never imports this module.

Network (the learned warm start of contacts): 7 inputs -> 64 ReLU -> 64 ReLU
-> 3 linear outputs; parameters packed as W1[64][7] b1[64] W2[64][64] b2[64]
W3[3][64] b3[3] (4,867 values).  Training loss over a batch of N records:

    L = (1/N) sum_n sum_k (y_nk - t_nk)^2      (optionally Huber's loss)

Plain definitions in float64 without rounding: the GPU kernels round weights,
inputs, activations and backward deltas to bfloat16 (FP32 accumulation), and
the tests allow for that.
"""
from __future__ import annotations

import numpy as np

IN, HID, OUT = 7, 64, 3
N_PARAMS = HID * IN + HID + HID * HID + HID + OUT * HID + OUT


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    assert w.size == N_PARAMS
    o = 0
    parts = []
    for shape in ((HID, IN), (HID,), (HID, HID), (HID,), (OUT, HID), (OUT,)):
        n = int(np.prod(shape))
        parts.append(w[o:o + n].reshape(shape))
        o += n
    return parts


def forward(w, X):
    """[N, 7] -> [N, 3]"""
    W1, b1, W2, b2, W3, b3 = unpack(w)
    h1 = np.maximum(X @ W1.T + b1, 0.0)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    return h2 @ W3.T + b3


def loss_grad(w, X, T, huber=0.0):
    """Loss and its gradient with respect to the packed parameters, by the
    chain rule through the three layers (ReLU derivative 0 at 0).  With
    huber = h > 0 each squared error e^2 with |e| > h is replaced by
    2 h |e| - h^2 (Huber's loss, written so that it equals e^2 inside)."""
    W1, b1, W2, b2, W3, b3 = unpack(w)
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    N = X.shape[0]
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3.T + b3
    r = y - T
    if huber > 0.0:
        out = np.abs(r) > huber
        L = float(np.where(out, 2.0 * huber * np.abs(r) - huber * huber, r * r).sum() / N)
        dy = 2.0 * np.where(out, huber * np.sign(r), r) / N
    else:
        L = float((r * r).sum() / N)
        dy = 2.0 * r / N
    gW3 = dy.T @ h2
    gb3 = dy.sum(0)
    dz2 = (dy @ W3) * (z2 > 0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return L, g


def adam(w, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba, Algorithm 1) with bias correction;
    step counts from 1.  Returns new (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
