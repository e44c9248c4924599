"""FP64 reference of the pointwise midpoint MLP (TEST INFRASTRUCTURE):
h = tanh(W1 x + b1), y = W2 h + b2, loss = 1/(2N) sum |y - t|^2, with the
gradient by the chain rule and one Adam step (Kingma & Ba), for checking the
GPU kernels.  Parameter order: W1 [32x8], b1 [32], W2 [2x32], b2 [2]."""
from __future__ import annotations

import numpy as np

NIN, NHID, NOUT = 8, 32, 2


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    o = 0
    W1 = w[o:o + NHID * NIN].reshape(NHID, NIN); o += NHID * NIN
    b1 = w[o:o + NHID]; o += NHID
    W2 = w[o:o + NOUT * NHID].reshape(NOUT, NHID); o += NOUT * NHID
    b2 = w[o:o + NOUT]
    return W1, b1, W2, b2


def forward(w, X):
    W1, b1, W2, b2 = unpack(w)
    H = np.tanh(X @ W1.T + b1)
    return H @ W2.T + b2, H


def loss_grad(w, X, Y):
    W1, b1, W2, b2 = unpack(w)
    N = X.shape[0]
    Yp, H = forward(w, X)
    E = (Yp - Y) / N
    loss = 0.5 * np.sum((Yp - Y) ** 2) / N
    gW2 = E.T @ H
    gb2 = E.sum(0)
    dH = E @ W2
    dZ = dH * (1.0 - H * H)
    gW1 = dZ.T @ X
    gb1 = dZ.sum(0)
    return loss, np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2])


def adam(w, g, m, v, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
