"""CPU reference of the ladder network (TEST INFRASTRUCTURE ONLY).

A plain FP64 statement of the network the library trains: 32 -> 128 -> 128 -> 64 with
ReLU after the hidden layers; two losses averaged over the batch: the soft-target
cross entropy -sum_j q_j log softmax(z)_j ("softmax") and the per-output logistic cross
entropy -sum_j [q_j log s(z_j) + (1-q_j) log(1 - s(z_j))] ("sigmoid"); the gradient by
the chain rule; and one Adam step (Kingma & Ba, bias-corrected).  Parameters are one flat vector in the order
W1[128][32], b1[128], W2[128][128], b2[128], W3[64][128], b3[64].
"""
from __future__ import annotations

import numpy as np

SHAPES = [(128, 32), (128,), (128, 128), (128,), (64, 128), (64,)]
N_PARAMS = sum(int(np.prod(s)) for s in SHAPES)


def unpack(p):
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(np.asarray(p[o:o + n], dtype=np.float64).reshape(s))
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in parts])


def forward(p, x):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ W3.T + b3
    return z3, (x, z1, h1, z2, h2)


def softmax(z):
    z = z - z.max(axis=1, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=1, keepdims=True)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def loss(p, x, q, kind="softmax"):
    z3, _ = forward(p, x)
    q = np.asarray(q, dtype=np.float64)
    if kind == "softmax":
        zs = z3 - z3.max(axis=1, keepdims=True)
        logp = zs - np.log(np.exp(zs).sum(axis=1, keepdims=True))
        return float(-(q * logp).sum(axis=1).mean())
    s = sigmoid(z3)
    return float(-(q * np.log(s) + (1 - q) * np.log(1 - s)).sum(axis=1).mean())


def loss_grad(p, x, q, kind="softmax"):
    """Mean loss and its gradient (flat, same order as the parameters)."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    z3, (x, z1, h1, z2, h2) = forward(p, x)
    B = x.shape[0]
    q = np.asarray(q, dtype=np.float64)
    probs = softmax(z3) if kind == "softmax" else sigmoid(z3)
    dz3 = (probs - q) / B
    dW3 = dz3.T @ h2
    db3 = dz3.sum(axis=0)
    dz2 = (dz3 @ W3) * (z2 > 0)
    dW2 = dz2.T @ h1
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (z1 > 0)
    dW1 = dz1.T @ x
    db1 = dz1.sum(axis=0)
    return loss(p, x, q, kind), pack([dW1, db1, dW2, db2, dW3, db3])


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
