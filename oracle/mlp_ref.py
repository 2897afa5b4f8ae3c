"""CPU reference of the pool-policy network (test infrastructure only).

Plain numpy, float64 arithmetic.  With ``rounded=True`` it rounds to bfloat16
(round to nearest even) at the same points as the device kernels: the
weights, the input, each hidden activation after its ReLU, and the gradients
that feed a matrix product (dZ2, dZ1, and dY where it multiplies h2).  With
``rounded=False`` it is the exact network, which the finite-difference pins
check the backward formulas against.
"""
from __future__ import annotations

import numpy as np

IN, H, OUT = 32, 128, 16
oW1 = 0
oB1 = oW1 + IN * H
oW2 = oB1 + H
oB2 = oW2 + H * H
oW3 = oB2 + H
oB3 = oW3 + H * OUT
NPARAMS = oB3 + OUT


def bf16(x):
    """Round float values to the nearest bfloat16 (ties to even)."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def unpack(P):
    P = np.asarray(P, dtype=np.float64)
    return (P[oW1:oB1].reshape(IN, H), P[oB1:oW2], P[oW2:oB2].reshape(H, H), P[oB2:oW3],
            P[oW3:oB3].reshape(H, OUT), P[oB3:oB3 + OUT])


def forward(P, X, nout, rounded=True):
    r = bf16 if rounded else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(P)
    X = np.asarray(X, dtype=np.float64)
    h1 = r(np.maximum(X @ r(W1) + b1, 0.0))
    h2 = r(np.maximum(h1 @ r(W2) + b2, 0.0))
    y = h2 @ r(W3)[:, :nout] + b3[:nout]
    return y, h1, h2


def backward(P, X, dY, nout, rounded=True):
    """(grad vector, dX) of sum(dY * y)."""
    r = bf16 if rounded else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(P)
    X = np.asarray(X, dtype=np.float64)
    _, h1, h2 = forward(P, X, nout, rounded)
    n = X.shape[0]
    dYp = np.zeros((n, OUT))
    dYp[:, :nout] = dY
    dW3 = h2.T @ r(dYp)
    db3 = dYp.sum(0)
    dH2 = dYp[:, :nout] @ r(W3)[:, :nout].T
    dZ2 = r(dH2 * (h2 > 0))
    dW2 = h1.T @ dZ2
    db2 = dZ2.sum(0)
    dH1 = dZ2 @ r(W2).T
    dZ1 = r(dH1 * (h1 > 0))
    dW1 = X.T @ dZ1
    db1 = dZ1.sum(0)
    dX = dZ1 @ r(W1).T
    g = np.zeros(NPARAMS)
    g[oW1:oB1] = dW1.ravel()
    g[oB1:oW2] = db1
    g[oW2:oB2] = dW2.ravel()
    g[oB2:oW3] = db2
    g[oW3:oB3] = dW3.ravel()
    g[oB3:oB3 + OUT] = db3
    return g, dX
