"""Pins of the float64 MLP oracle: central finite differences of the loss
through every layer, the decode's closed forms, bfloat16 rounding."""
import math

import numpy as np

import qsg_workloads as W
from oracle import mlp


def _batch(B=5, seed=1):
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.normal(size=(B, 6))
    t = rng.random((B, mlp.N_INC)) + 0.05
    t /= t.sum(axis=1, keepdims=True)
    logL = rng.normal(size=B)
    return X, t, logL


def _loss(params, X, t, logL):
    z = mlp.forward(params, X)["out"]
    return mlp.loss_and_grad(z, t, logL)[0]


def test_backward_matches_central_differences():
    p = mlp.init_params(3) * 0.5
    X, t, logL = _batch()
    cache = mlp.forward(p, X)
    loss, dz = mlp.loss_and_grad(cache["out"], t, logL)
    g = mlp.backward(p, cache, dz)
    rng = np.random.Generator(np.random.PCG64(4))
    # every layer's weights and biases, sampled
    offs = [0]
    for k, n in mlp.SIZES:
        offs += [offs[-1] + k * n, offs[-1] + k * n + n]
    idx = np.concatenate([rng.integers(a, b, size=6) for a, b in zip(offs[:-1], offs[1:])])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (_loss(p + e, X, t, logL) - _loss(p - e, X, t, logL)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (i, fd, g[i])


def test_loss_gradient_in_logits_matches_differences():
    rng = np.random.Generator(np.random.PCG64(2))
    z = rng.normal(size=(3, 32))
    _, t, logL = _batch(3)
    loss, g = mlp.loss_and_grad(z, t, logL)
    h = 1e-6
    for b in range(3):
        for l in (0, 7, 30, 31):
            e = np.zeros_like(z)
            e[b, l] = h
            fd = (mlp.loss_and_grad(z + e, t, logL)[0] - mlp.loss_and_grad(z - e, t, logL)[0]) / (2 * h)
            assert abs(fd - g[b, l]) < 1e-7


def test_kl_vanishes_at_the_target():
    rng = np.random.Generator(np.random.PCG64(5))
    z = rng.normal(size=(4, 32))
    t = mlp.softmax(z[:, :31])
    loss, g = mlp.loss_and_grad(z, t, z[:, 31].copy())
    assert abs(loss) < 1e-12 and np.max(np.abs(g)) < 1e-12


def test_zero_logits_decode_to_the_geometric_ladder():
    z = np.zeros((2, 32))
    lad = mlp.decode(z, np.array([2.0, 2.8]), np.array([4.0, 3.6]))
    assert np.allclose(lad[0], W.geometric_ladder(2.0, 4.0, 32), rtol=1e-14)
    assert np.allclose(lad[1], W.geometric_ladder(2.8, 3.6, 32), rtol=1e-14)


def test_decode_is_monotone_with_fixed_end_points():
    rng = np.random.Generator(np.random.PCG64(6))
    z = rng.normal(scale=3.0, size=(16, 32))
    lad = mlp.decode(z, np.full(16, 2.0), np.full(16, 4.0))
    assert np.all(np.diff(lad, axis=1) > 0)
    assert np.allclose(lad[:, 0], 2.0) and np.allclose(lad[:, -1], 4.0)
    # predicted acceptance: equal barrier per gap of exp(z31)/31
    assert np.allclose(mlp.predicted_acceptance(np.full((1, 32), math.log(31 * 0.25))), 0.75)


def test_bf16_rounding_is_nearest_even():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -2.5, 3.140625,
                     1.0 + 2 ** -8 + 2 ** -20])
    got = mlp.to_bf16(vals)
    # bfloat16 keeps 7 fraction bits: spacing 2^-7 near 1
    assert got[0] == 1.0
    assert got[1] == 1.0                  # tie, even neighbour
    assert got[2] == 1.0 + 2 ** -6        # tie between 1+2^-7 and 1+2^-6: even
    assert got[3] == 1.0                  # below half a spacing
    assert got[4] == -2.5 and got[5] == 3.140625
    assert got[6] == 1.0 + 2 ** -7        # just above the tie


def test_adam_first_step_moves_by_lr():
    p = np.zeros(4)
    g = np.array([1.0, -2.0, 0.5, 0.0])
    p1, m, v = mlp.adam(p, g, np.zeros(4), np.zeros(4), 1, 0.01)
    assert np.allclose(p1[:3], -0.01 * np.sign(g[:3]), rtol=1e-6)
    assert p1[3] == 0.0


def test_gelu_is_the_exact_erf_form():
    """GELU(x) = x Phi(x) with Phi the standard normal distribution function:
    table values Phi(1) = 0.8413447460685429, Phi(2) = 0.9772498680518208 and
    the density phi(1) = 0.24197072451914337.  The tanh approximation of
    GELU is 1.5e-4 off at x = 1, the sigmoid form x sigma(1.702 x) 2e-2."""
    phi1, Phi1, Phi2 = 0.24197072451914337, 0.8413447460685429, 0.9772498680518208
    assert abs(mlp.gelu(1.0) - Phi1) < 1e-15
    assert abs(mlp.gelu(-1.0) - (-(1.0 - Phi1))) < 1e-15
    assert abs(mlp.gelu(2.0) - 2 * Phi2) < 1e-15
    assert mlp.gelu(0.0) == 0.0
    # derivative Phi(x) + x phi(x)
    assert abs(mlp.gelu_grad(0.0) - 0.5) < 1e-15
    assert abs(mlp.gelu_grad(1.0) - (Phi1 + phi1)) < 1e-15
    assert abs(mlp.gelu_grad(-1.0) - ((1.0 - Phi1) - phi1)) < 1e-15
