"""The plain serial C fitness (oracle/serial.c) against the float64 numpy
oracle and against closed forms.  CPU only."""
import math

import numpy as np
import pytest

from oracle import game as og
from oracle import serial

ERRORS = {0: og.MSE, 1: og.RMSE, 2: og.TMSE, 3: og.TMSE}


@pytest.mark.parametrize("basis", [0, 1, 2, 3])
@pytest.mark.parametrize("degree", [1, 2, 5, 8, 16])
def test_serial_matches_numpy_oracle(basis, degree):
    rng = np.random.default_rng(10 * basis + degree)
    X = rng.uniform(-1, 1, (257, 4)).astype(np.float32)
    t = rng.normal(0, 1, 257).astype(np.float32)
    W = rng.uniform(-1, 1, (5, og.num_genes(basis, 4, degree))).astype(np.float32)
    for ef, R in ((0, 0.0), (1, 0.0), (2, 0.5), (3, 0.3)):
        got = serial.fitness(X, t, W, basis, degree, ef, R)
        ref = og.fitness(X, t, W, basis, degree, ERRORS[ef], R, literal_tmse=(ef == 3))
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-300)


@pytest.mark.parametrize("j", [1, 2, 3, 7, 12])
def test_chebyshev_member_is_cos_j_theta(j):
    """A chromosome whose only gene weights T_j of feature 0, on x = cos(theta)
    with targets cos(j theta): T_j(cos theta) = cos(j theta), so the error is
    zero up to float32 rounding of x and float64 rounding of the recurrence."""
    theta = np.linspace(0.05, 3.0, 101)
    X = np.cos(theta).astype(np.float32)[:, None]
    t = np.cos(j * np.arccos(X[:, 0].astype(np.float64))).astype(np.float32)
    K = og.num_genes(0, 1, 12)
    W = np.zeros((1, K), np.float32)
    W[0, 1 + (j - 1)] = 1.0
    f = serial.fitness(X, t, W, 0, 12)
    assert f[0] < 1e-13


def test_power_basis_polynomial_reproduces_target():
    """Power basis, degree 3: genes (a0, c1, c2, c3) reproduce a0 + c1 x +
    c2 x^2 + c3 x^3 computed here in float64."""
    x = np.linspace(-1, 1, 64).astype(np.float32)
    a0, c = 0.25, (0.5, -0.75, 0.125)
    W = np.array([[a0, *c]], np.float32)
    xd = x.astype(np.float64)
    y = a0 + c[0] * xd + c[1] * xd ** 2 + c[2] * xd ** 3
    f = serial.fitness(x[:, None], y.astype(np.float32), W, 2, 3)
    assert f[0] < 1e-14


def test_bad_arguments_raise():
    X = np.zeros((4, 2), np.float32)
    t = np.zeros(4, np.float32)
    W = np.zeros((1, 5), np.float32)
    with pytest.raises(ValueError):
        serial.fitness(X, t, W, 7, 2)
