"""Pins of the surrogate-network oracle: finite differences for the analytic
gradients, closed forms for GELU and the first Adam step, scipy for the
Spearman correlation."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import mlp


def test_gelu_identities():
    x = np.linspace(-6, 6, 101)
    np.testing.assert_allclose(mlp.gelu(x) - mlp.gelu(-x), x, atol=1e-14)
    assert mlp.gelu(0.0) == 0.0
    assert abs(mlp.gelu(10.0) - 10.0) < 1e-12 and abs(mlp.gelu(-10.0)) < 1e-12
    # Phi(1) = 0.8413447460685429 (standard normal CDF)
    assert abs(mlp.gelu(1.0) - 0.8413447460685429) < 1e-15
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(x), fd, atol=1e-8)


def test_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    n_in, hidden, B = 7, (5, 4), 6
    params = [rng.normal(0, 0.7, s) for s in mlp.shapes(n_in, hidden)]
    X = rng.uniform(-1, 1, (B, n_in))
    t = rng.normal(size=B)
    grads = mlp.backward(params, X, t)
    h = 1e-6
    for pi, p in enumerate(params):
        flat = p.reshape(-1)
        for idx in range(flat.size):
            old = flat[idx]
            flat[idx] = old + h
            lp = mlp.loss(params, X, t)
            flat[idx] = old - h
            lm = mlp.loss(params, X, t)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            g = grads[pi].reshape(-1)[idx]
            assert abs(g - fd) <= 1e-6 * max(1.0, abs(fd)), (pi, idx, g, fd)


def test_adam_first_step_closed_form():
    """After one step m_hat = g and v_hat = g^2: the update is lr g/(|g|+eps)."""
    g = [np.array([0.3, -2.0, 0.0, 1e-3])]
    p = [np.array([1.0, 1.0, 1.0, 1.0])]
    z = [np.zeros(4)]
    newp, m, v = mlp.adam_step(p, g, z, z, 1, lr=0.01)
    np.testing.assert_allclose(newp[0], 1.0 - 0.01 * g[0] / (np.abs(g[0]) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m[0], 0.1 * g[0])
    np.testing.assert_allclose(v[0], 0.001 * g[0] ** 2)


def test_spearman_matches_scipy():
    rng = np.random.default_rng(1)
    a = rng.normal(size=500)
    b = a + rng.normal(scale=0.8, size=500)
    assert abs(mlp.spearman(a, b) - stats.spearmanr(a, b).statistic) < 1e-12
    assert abs(mlp.spearman(a, a) - 1.0) < 1e-12
    assert abs(mlp.spearman(a, -a) + 1.0) < 1e-12


def test_init_params():
    p = mlp.init_params(257, seed=4)
    assert [x.shape for x in p] == [(256, 257), (256,), (256, 256), (256,), (1, 256), (1,)]
    for w, fan in ((p[0], 257), (p[2], 256), (p[4], 256)):
        assert w.dtype == np.float32
        assert np.all(np.abs(w) <= 1 / math.sqrt(fan) + 1e-7)
        assert abs(float(w.mean())) < 0.01 / math.sqrt(fan) * 10
        assert abs(float(w.std()) - 1 / math.sqrt(3 * fan)) < 0.05 / math.sqrt(fan)
    assert all(np.all(b == 0) for b in (p[1], p[3], p[5]))
    q = mlp.init_params(257, seed=4)
    assert all(np.array_equal(x, y) for x, y in zip(p, q))
    r = mlp.init_params(257, seed=5)
    assert not np.array_equal(p[0], r[0])


def test_adam_training_reduces_loss():
    rng = np.random.default_rng(2)
    n_in = 9
    params = [np.asarray(x, np.float64) for x in mlp.init_params(n_in, 0, hidden=(16, 16))]
    X = rng.uniform(-1, 1, (64, n_in))
    t = np.sin(X @ rng.normal(size=n_in))
    m = [np.zeros_like(x) for x in params]
    v = [np.zeros_like(x) for x in params]
    l0 = mlp.loss(params, X, t)
    for step in range(1, 201):
        g = mlp.backward(params, X, t)
        params, m, v = mlp.adam_step(params, g, m, v, step, lr=1e-2)
    assert mlp.loss(params, X, t) < 0.3 * l0


def test_input_stats_closed_forms():
    """Per-gene standardisation of the network's inputs: a two-valued column
    {a, b} (equal counts) has mean (a + b) / 2 and population deviation
    |a - b| / 2; a constant column takes the floor; shifting a column moves
    only its mean and scaling it by c scales its inverse deviation by 1/c;
    the standardised columns have mean 0 and deviation 1."""
    rng = np.random.default_rng(3)
    rows = 1000
    G = rng.uniform(-1, 1, (rows, 6))
    G[:, 0] = np.where(np.arange(rows) % 2 == 0, 0.25, -0.75)    # two values
    G[:, 1] = 0.5                                                # constant
    G[:, 2] = 1e-4 * rng.standard_normal(rows)                   # below the floor
    mean, inv = mlp.input_stats(G)
    assert mean[0] == np.float32(-0.25) and inv[0] == np.float32(2.0)
    assert mean[1] == np.float32(0.5) and inv[1] == np.float32(1.0 / mlp.INPUT_STD_FLOOR)
    assert inv[2] == np.float32(1.0 / mlp.INPUT_STD_FLOOR)
    m2, i2 = mlp.input_stats(np.column_stack([G[:, 3] + 0.125, 0.5 * G[:, 4]]))
    np.testing.assert_allclose(m2[0], mean[3] + 0.125, rtol=1e-6)
    np.testing.assert_allclose(i2[0], inv[3], rtol=1e-6)
    np.testing.assert_allclose(i2[1], 2.0 * inv[4], rtol=1e-6)
    X = mlp.standardize(G, mean, inv).astype(np.float64)
    live = [0, 3, 4, 5]
    np.testing.assert_allclose(X[:, live].mean(axis=0), 0.0, atol=1e-6)
    np.testing.assert_allclose(X[:, live].std(axis=0), 1.0, rtol=1e-5)
    # identity statistics leave the genes as they are
    G32 = G.astype(np.float32)
    assert np.array_equal(mlp.standardize(G32, np.zeros(6, np.float32), np.ones(6, np.float32)), G32)
