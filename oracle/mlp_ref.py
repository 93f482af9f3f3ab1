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


def _round(v, mode, rng):
    """The value a half-precision operand takes: unchanged (mode None), rounded
    to the nearest FP16 value ('fp16'), or moved by a random relative amount of
    up to 2^-10, one FP16 unit in the last place ('perturb')."""
    if mode is None:
        return v
    if mode == "fp16":
        return v.astype(np.float16).astype(np.float64)
    return v * (1.0 + 2.0 ** -10 * rng.uniform(-1.0, 1.0, v.shape))


def grad(P, T, half=None, rng=None):
    """Gradient of the mean squared error with respect to the flat parameters.

    ``half`` applies ``_round`` where a half-precision kernel would hold an
    operand in FP16: the hidden activations g(Z1) and g(Z2), and dL/dZ2 as
    an operand of dW2 and dL/dH1 (db2 sums it unrounded).  dL/dZ2 is rounded
    scaled by n * 1024, as a kernel keeps it (the per-row derivative times a
    loss scale of 1024), so small values stay clear of FP16's subnormals."""
    W1, b1, W2, b2, w3, b3 = unpack(P)
    T = np.asarray(T, dtype=np.float64)
    X, base, x = T[:, 0:3], T[:, 3], T[:, 4]
    n = X.shape[0]
    Z1 = X @ W1.T + b1
    H1 = _round(g(Z1), half, rng)
    Z2 = H1 @ W2.T + b2
    H2 = _round(g(Z2), half, rng)
    o = H2 @ w3 + b3
    xh = sigmoid(base + o)
    loss = np.mean((xh - x) ** 2)
    do = 2.0 * (xh - x) * xh * (1.0 - xh) / n          # dL/do per row
    dw3 = H2.T @ do
    db3 = do.sum()
    dH2 = np.outer(do, w3)
    dZ2 = dH2 * g_prime(Z2)
    sc = n * 1024.0
    dZ2h = _round(dZ2 * sc, half, rng) / sc
    dW2 = dZ2h.T @ H1
    db2 = dZ2.sum(0)
    dH1 = dZ2h @ W2
    dZ1 = dH1 * g_prime(Z1)
    dW1 = dZ1.T @ X
    db1 = dZ1.sum(0)
    return np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dw3, [db3]]), loss


def grad_envelope(P, T, draws: int = 16, seed: int = 0):
    """Per-parameter spread of the gradient under FP16 operands: the largest
    deviation from the FP16-rounded gradient over ``draws`` gradients whose
    half-precision operands are each moved by up to one FP16 unit in the last
    place (covering a rounding that lands on the other neighbour)."""
    rng = np.random.default_rng(seed)
    g0, _ = grad(P, T, half="fp16")
    env = np.zeros_like(g0)
    for _ in range(draws):
        gp, _ = grad(P, T, half="perturb", rng=rng)
        env = np.maximum(env, np.abs(gp - g0))
    return g0, env


def round_bf16(P):
    """Weights as the kernels use them: FP32 rounded to the nearest BF16."""
    u = np.asarray(P, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)
