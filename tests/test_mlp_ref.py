"""Pin of the FP64 surrogate reference: its analytic gradient against central
finite differences of its own loss (a plainly different computation)."""
import numpy as np

from oracle import mlp_ref


def test_reference_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    P = rng.normal(0, 0.3, mlp_ref.N_PARAMS)
    T = np.column_stack([rng.normal(0, 1, (128, 3)), rng.normal(0, 1, 128), rng.uniform(0, 1, 128)])
    g, loss = mlp_ref.grad(P, T)
    assert np.isclose(loss, mlp_ref.forward(P, T)[1])
    idx = np.concatenate([rng.choice(192, 6, replace=False), 192 + rng.choice(64, 4, replace=False),
                          256 + rng.choice(4096, 10, replace=False), 4352 + rng.choice(64, 4, replace=False),
                          4416 + rng.choice(64, 4, replace=False), [4480]])
    h = 1e-6
    for i in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        fd = (mlp_ref.forward(Pp, T)[1] - mlp_ref.forward(Pm, T)[1]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(fd)) + 1e-10, (i, fd, g[i])


def test_activation_and_bf16_rounding():
    z = np.linspace(-6, 6, 1001)
    # GELU-shaped: identity far right, zero far left, g(0) = 0, close to z * Phi(z)
    assert np.all(mlp_ref.g(z[z >= 2.5]) == z[z >= 2.5]) and np.all(mlp_ref.g(z[z <= -2.5]) == 0)
    from scipy.special import ndtr
    assert np.max(np.abs(mlp_ref.g(z) - z * ndtr(z))) < 0.1
    h = 1e-6
    assert np.allclose(mlp_ref.g_prime(z), (mlp_ref.g(z + h) - mlp_ref.g(z - h)) / (2 * h), atol=1e-6)
    # BF16 keeps 7 explicit significand bits: 1 + 2^-7 is representable,
    # 1 + 2^-8 is a tie that rounds to even (1), 1 + 3 * 2^-8 rounds up
    x = np.array([1.0, 1.0078125, 1.00390625, 1.01171875, -3.14159, 0.0])
    r = mlp_ref.round_bf16(x)
    assert list(r[[0, 1, 2, 3, 5]]) == [1.0, 1.0078125, 1.0, 1.015625, 0.0]
    assert abs(r[4] - x[4]) <= 2 ** -8 * abs(x[4])


def test_fp16_reference_and_envelope():
    # rounding the half-precision operands moves the gradient by a few FP16
    # units relative; the envelope covers that move and is zero only where
    # the gradient itself does not depend on a half-precision operand
    rng = np.random.default_rng(1)
    P = mlp_ref.round_bf16(rng.normal(0, 0.2, mlp_ref.N_PARAMS))
    T = np.column_stack([rng.normal(0, 1, (256, 3)), rng.normal(0, 1, 256), rng.uniform(0, 1, 256)])
    g, _ = mlp_ref.grad(P, T)
    g16, env = mlp_ref.grad_envelope(P, T, draws=8)
    scale = np.abs(g).max()
    assert np.max(np.abs(g16 - g)) <= 2e-2 * scale
    assert np.max(np.abs(g16 - g)) > 0.0
    assert np.all(env >= 0) and np.max(env) <= 2e-2 * scale
    # the rounding-free call is unchanged by the half-precision option's absence
    g2, _ = mlp_ref.grad(P, T, half=None)
    assert np.array_equal(g, g2)
