"""FP64 reference of the sampling surrogate's network, for gradient checks.

TEST INFRASTRUCTURE (see the package docstring).  The model is the one the
library trains: for a tuple (f0, f1, f2, base, x) -- features f = (ln a / 2,
ln b / 2, Phi^-1(u) / 3), base = psi(a) - psi(b) + sqrt(psi'(a) + psi'(b))
Phi^-1(u) -- the prediction is

    x_hat = sigmoid(base + w3 . g(W2 g(W1 f + b1) + b2) + b3),
    g(z)  = z * S(z),  S(z) = smoothstep(clamp(z/5 + 1/2, 0, 1)) = u^2 (3 - 2u),

and the loss is the mean squared error of x_hat against x.  The flat parameter
vector is W1 [64][3], b1 [64], W2 [64][64], b2 [64], w3 [64], b3 (4481
values).  Forward and backward are written out plainly in float64.
"""
from __future__ import annotations

import numpy as np

N_PARAMS = 64 * 3 + 64 + 64 * 64 + 64 + 64 + 1


def unpack(P):
    P = np.asarray(P, dtype=np.float64)
    assert P.shape == (N_PARAMS,)
    W1 = P[0:192].reshape(64, 3)
    b1 = P[192:256]
    W2 = P[256:4352].reshape(64, 64)
    b2 = P[4352:4416]
    w3 = P[4416:4480]
    b3 = P[4480]
    return W1, b1, W2, b2, w3, b3


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def g(z):
    u = np.clip(z / 5.0 + 0.5, 0.0, 1.0)
    return z * u * u * (3.0 - 2.0 * u)


def g_prime(z):
    u = np.clip(z / 5.0 + 0.5, 0.0, 1.0)
    return u * u * (3.0 - 2.0 * u) + z * 1.2 * u * (1.0 - u)


def forward(P, T):
    W1, b1, W2, b2, w3, b3 = unpack(P)
    T = np.asarray(T, dtype=np.float64)
    X, base, x = T[:, 0:3], T[:, 3], T[:, 4]
    Z1 = X @ W1.T + b1
    H1 = g(Z1)
    Z2 = H1 @ W2.T + b2
    H2 = g(Z2)
    o = H2 @ w3 + b3
    xh = sigmoid(base + o)
    loss = np.mean((xh - x) ** 2)
    return xh, loss, (X, Z1, H1, Z2, H2, xh, x)


def grad(P, T):
    """Gradient of the mean squared error with respect to the flat parameters."""
    W1, b1, W2, b2, w3, b3 = unpack(P)
    xh, loss, (X, Z1, H1, Z2, H2, xh, x) = forward(P, T)
    n = X.shape[0]
    do = 2.0 * (xh - x) * xh * (1.0 - xh) / n          # dL/do per row
    dw3 = H2.T @ do
    db3 = do.sum()
    dH2 = np.outer(do, w3)
    dZ2 = dH2 * g_prime(Z2)
    dW2 = dZ2.T @ H1
    db2 = dZ2.sum(0)
    dH1 = dZ2 @ W2
    dZ1 = dH1 * g_prime(Z1)
    dW1 = dZ1.T @ X
    db1 = dZ1.sum(0)
    return np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dw3, [db3]]), loss


def round_bf16(P):
    """Weights as the kernels use them: FP32 rounded to the nearest BF16."""
    u = np.asarray(P, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)
