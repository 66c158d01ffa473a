"""Pins of the FP64 surrogate reference: closed forms and finite differences."""
import math

import numpy as np
import pytest

from oracle import mlp_ref


def test_gelu_closed_forms():
    assert mlp_ref.gelu(0.0) == 0.0
    assert mlp_ref.gelu_d(0.0) == pytest.approx(0.5, abs=1e-15)
    # GELU(z) - GELU(-z) = z for the exact (normal CDF) form
    z = np.linspace(-5, 5, 101)
    assert np.allclose(mlp_ref.gelu(z) - mlp_ref.gelu(-z), z, atol=1e-14)
    # Phi(1) = 0.841344746...
    assert mlp_ref.gelu(1.0) == pytest.approx(0.8413447460685429, rel=1e-13)
    h = 1e-6
    assert np.allclose((mlp_ref.gelu(z + h) - mlp_ref.gelu(z - h)) / (2 * h), mlp_ref.gelu_d(z), atol=1e-8)


def test_round_bf16():
    x = np.array([1.0, 1.00390625, 1.005859375, -3.14159265, 1e-3, 65504.0], dtype=np.float32)
    r = mlp_ref.round_bf16(x)
    # bfloat16 keeps 8 significant bits
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == np.float32(1.0078125)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8)


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_finite_differences(seed):
    rng = np.random.default_rng(seed)
    n_in, width, depth = 8, 256, 4
    n = mlp_ref.n_params(n_in, width, depth)
    p = rng.normal(size=n) * 0.05
    X = rng.normal(size=(16, n_in))
    t = rng.normal(size=16)
    loss, g = mlp_ref.loss_and_grad(p, X, t, n_in, width, depth)
    # probe parameters in every block: first/last layer weights, biases, output
    probes = list(rng.integers(0, n, size=40)) + [0, n_in * width, n - 1, n - 2, n - width - 1]
    h = 1e-6
    for i in probes:
        pp = p.copy()
        pm = p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (mlp_ref.loss_and_grad(pp, X, t, n_in, width, depth)[0] -
              mlp_ref.loss_and_grad(pm, X, t, n_in, width, depth)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])
    assert math.isfinite(loss)


def test_parameter_count():
    assert mlp_ref.n_params(8) == 256 * 8 + 256 + 3 * (256 * 256 + 256) + 256 + 1
