"""Pins of the oracle's fitness path against what the paper and mathematics fix.

Each test names what it pins.  None of them re-types the oracle's formula:
they use closed forms, numpy library routines, the paper's worked example,
special cases and invariants.
"""
import os

import numpy as np
import pytest
from numpy.polynomial import chebyshev, legendre, polynomial

from oracle import game
from paper_1304_0597_amd import datagen

BASES = [game.CHEBYSHEV, game.LEGENDRE, game.POWER, game.TRIG]


# ---------------------------------------------------------------- basis tables
@pytest.mark.parametrize("d", [1, 2, 5, 8, 16])
def test_chebyshev_closed_form(d):
    """T_j(cos theta) = cos(j theta), and T_j(+-1) = (+-1)^j."""
    theta = np.linspace(0.0, np.pi, 1001)
    tab = game.basis_table(np.cos(theta), game.CHEBYSHEV, d)[:, 0, :]
    for j in range(1, d + 1):
        np.testing.assert_allclose(tab[:, j - 1], np.cos(j * theta), atol=1e-13 * j * j)
    ends = game.basis_table(np.array([1.0, -1.0]), game.CHEBYSHEV, d)[:, 0, :]
    for j in range(1, d + 1):
        assert ends[0, j - 1] == 1.0 and ends[1, j - 1] == (-1.0) ** j


@pytest.mark.parametrize("basis,ev", [(game.CHEBYSHEV, chebyshev.chebval),
                                      (game.LEGENDRE, legendre.legval),
                                      (game.POWER, polynomial.polyval)])
def test_basis_matches_numpy_polynomial(basis, ev):
    """Each member phi_j equals numpy's evaluation of the unit series e_j."""
    x = np.random.default_rng(1).uniform(-1, 1, 500)
    d = 10
    tab = game.basis_table(x, basis, d)[:, 0, :]
    for j in range(1, d + 1):
        c = np.zeros(j + 1)
        c[j] = 1.0
        np.testing.assert_allclose(tab[:, j - 1], ev(x, c), rtol=1e-12, atol=1e-13)


def test_legendre_endpoints_and_known_value():
    """P_j(1) = 1, P_j(-1) = (-1)^j, P_2(0.5) = -0.125."""
    tab = game.basis_table(np.array([1.0, -1.0, 0.5]), game.LEGENDRE, 6)[:, 0, :]
    np.testing.assert_allclose(tab[0], 1.0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(tab[1], [(-1.0) ** j for j in range(1, 7)], atol=1e-15)
    assert abs(tab[2, 1] + 0.125) < 1e-15


def test_trig_angle_addition_and_pythagoras():
    """cos/sin((j+1)x) from the angle-addition formulas, cos^2 + sin^2 = 1."""
    x = np.random.default_rng(2).uniform(-1, 1, 300)
    d = 9
    tab = game.basis_table(x, game.TRIG, d)
    c, s = tab[:, 0, :], tab[:, 1, :]
    np.testing.assert_allclose(c * c + s * s, 1.0, atol=1e-14)
    for j in range(1, d):
        np.testing.assert_allclose(c[:, j], c[:, j - 1] * c[:, 0] - s[:, j - 1] * s[:, 0], atol=1e-13)
        np.testing.assert_allclose(s[:, j], s[:, j - 1] * c[:, 0] + c[:, j - 1] * s[:, 0], atol=1e-13)


def test_trig_cos_block_is_chebyshev_of_cos():
    """With the sin genes zero, trig on features theta equals Chebyshev on
    features cos(theta) (T_j(cos theta) = cos(j theta))."""
    rng = np.random.default_rng(3)
    N, d, P = 3, 5, 4
    theta = rng.uniform(-1, 1, (50, N))
    t = rng.uniform(-1, 1, 50)
    w_cheb = rng.uniform(-1, 1, (P, N * d + 1))
    w_trig = np.zeros((P, 2 * N * d + 1))
    w_trig[:, 0] = w_cheb[:, 0]
    for i in range(N):
        w_trig[:, 1 + i * 2 * d: 1 + i * 2 * d + d] = w_cheb[:, 1 + i * d: 1 + (i + 1) * d]
    f_trig = game.fitness(theta, t, w_trig, game.TRIG, d)
    f_cheb = game.fitness(np.cos(theta), t, w_cheb, game.CHEBYSHEV, d)
    np.testing.assert_allclose(f_trig, f_cheb, rtol=1e-12)


# ------------------------------------------------------------- layout / model
def _fourier_as_polynomial(X, G, d):
    """Eq. 9's output written as a polynomial in z = exp(i f): a_j cos(j f) +
    b_j sin(j f) is the real part of (a_j - i b_j) z^j, so the model is
    a_0 + sum over features of Re(p(z)) with p(z) = sum_j (a_j - i b_j) z^j,
    evaluated by numpy's polynomial routine.  [NP, P]."""
    X = np.asarray(X, np.float64)
    G = np.atleast_2d(np.asarray(G, np.float64))
    z = np.exp(1j * X)                                   # [NP, N]
    out = np.empty((X.shape[0], G.shape[0]))
    for p in range(G.shape[0]):
        coeffs = np.concatenate([[0.0], G[p, 1:d + 1] - 1j * G[p, d + 1:]])
        out[:, p] = G[p, 0] + polynomial.polyval(z, coeffs).real.sum(axis=1)
    return out


def test_shared_gene_model_is_tied_per_feature_genes():
    """The paper's own polytrigo model shares a_j, b_j over all features
    (Eq. 9; chromosome [a_0, a_1..a_d, b_1..b_d]).  Written as a complex
    polynomial in exp(i f), it must equal the per-feature model (recurrences)
    whose genes are tied across features."""
    rng = np.random.default_rng(4)
    N, d, NP = 4, 3, 7
    X = rng.uniform(-1, 1, (NP, N))
    shared = rng.uniform(-1, 1, 2 * d + 1)      # a_0, a_1..a_d, b_1..b_d
    ref = _fourier_as_polynomial(X, shared, d)[:, 0]
    tied = np.concatenate([[shared[0]]] + [shared[1:]] * N)
    out = game.outputs(X, tied, game.TRIG, d)[:, 0]
    np.testing.assert_allclose(out, ref, rtol=1e-13, atol=1e-13)


def test_shared_trig_model_matches_eq9_as_a_polynomial_in_exp_if():
    """The oracle's shared-gene outputs (sums computed once, then a product)
    against Eq. 9 evaluated as a complex polynomial in exp(i f) per feature;
    and the same model written as the per-feature model with tied genes."""
    rng = np.random.default_rng(8)
    N, d, NP, P = 5, 4, 9, 3
    X = rng.uniform(-3, 3, (NP, N))                   # raw radians, any range
    G = rng.uniform(-1, 1, (P, 2 * d + 1))
    ref = _fourier_as_polynomial(X, G, d)
    np.testing.assert_allclose(game.shared_trig_outputs(X, G, d), ref, rtol=1e-12, atol=1e-12)
    tied = np.concatenate([G[:, :1]] + [G[:, 1:]] * N, axis=1)
    np.testing.assert_allclose(game.outputs(X, tied, game.TRIG, d), ref, rtol=1e-12, atol=1e-12)


def test_shared_trig_sums_closed_forms():
    """sum_i cos(j f_i) over N equal features f is N cos(j f); at f = 0 the
    cos sums are N and the sin sums 0; with features f and -f the sin sums
    cancel (odd) and the cos sums double (even)."""
    d, N = 6, 7
    S = game.shared_trig_sums(np.zeros((1, N)), d)
    np.testing.assert_array_equal(S, np.concatenate([np.full((1, d), N), np.zeros((1, d))], 1))
    f = 0.37
    S = game.shared_trig_sums(np.full((1, N), f), d)
    j = np.arange(1, d + 1)
    np.testing.assert_allclose(S[0, :d], N * np.cos(j * f), rtol=1e-14)
    np.testing.assert_allclose(S[0, d:], N * np.sin(j * f), rtol=1e-14)
    S = game.shared_trig_sums(np.array([[f, -f, 1.1, -1.1]]), d)
    np.testing.assert_allclose(S[0, d:], 0.0, atol=1e-15)
    np.testing.assert_allclose(S[0, :d], 2 * np.cos(j * f) + 2 * np.cos(j * 1.1), rtol=1e-14)


def test_shared_trig_model_is_degree_one_power_model_on_the_sums():
    """The shared model equals the power expansion of degree 1 over the 2d
    per-pattern sums taken as features (the way the device evaluates it),
    with the same chromosome."""
    rng = np.random.default_rng(9)
    X = rng.uniform(-1, 1, (50, 11))
    d = 3
    G = rng.uniform(-1, 1, (4, 2 * d + 1))
    t = (rng.random(50) < 0.5).astype(float)
    Z = game.shared_trig_sums(X, d)
    np.testing.assert_allclose(game.outputs(Z, G, game.POWER, 1),
                               game.shared_trig_outputs(X, G, d), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(game.fitness(Z, t, G, game.POWER, 1, game.TMSE, 0.49),
                               game.shared_trig_fitness(X, t, G, d, game.TMSE, 0.49), rtol=1e-13)


def test_num_genes_matches_workload_counts():
    """29 genes for 7 features at degree 4, 161 for 20 at 8, 257 for 32 at 8."""
    assert game.num_genes(game.CHEBYSHEV, 7, 4) == 29
    assert game.num_genes(game.LEGENDRE, 20, 8) == 161
    assert game.num_genes(game.CHEBYSHEV, 32, 8) == 257
    assert game.num_genes(game.TRIG, 11, 8) == 177


# ------------------------------------------------------------ error functions
def _golden_rows(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "worked_example.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            t0, t1, o0, o1, fn, R, val = line.split()
            rows.append(((float(t0), float(t1)), (float(o0), float(o1)), fn, float(R), float(val)))
    return rows


def test_worked_example_from_the_paper(golden_dir):
    """MSE 0.24 / 0.13 and TMSE(R=0.5) 0 / 0.13 as printed (two decimals)."""
    rows = _golden_rows(golden_dir)
    assert len(rows) == 4
    for t, out, fn, R, printed in rows:
        kind = game.MSE if fn == "mse" else game.TMSE
        v = game.error_from_outputs(np.array(out)[:, None], np.array(t), kind, R)[0]
        assert abs(v - printed) < 0.005, (t, out, fn, v, printed)
    # the exact values behind the printed ones
    assert game.error_from_outputs(np.array([[0.49], [0.51]]), np.array([0.0, 1.0]))[0] == pytest.approx(0.2401, abs=1e-15)
    assert game.error_from_outputs(np.array([[0.0], [0.49]]), np.array([0.0, 1.0]))[0] == pytest.approx(0.13005, abs=1e-15)


def test_tmse_literal_reading_contradicts_worked_example():
    """Eq. 10 as printed (squared residual compared with R) gives 0, not 0.13,
    for the second solution of the worked example; the |r| > R reading gives
    the printed value."""
    out = np.array([[0.0], [0.49]])
    t = np.array([0.0, 1.0])
    assert game.error_from_outputs(out, t, game.TMSE, 0.5, literal_tmse=True)[0] == 0.0
    assert game.error_from_outputs(out, t, game.TMSE, 0.5)[0] == pytest.approx(0.13005)


def test_rmse_and_tmse_relations():
    rng = np.random.default_rng(5)
    out = rng.normal(size=(100, 6))
    t = rng.normal(size=100)
    mse = game.error_from_outputs(out, t, game.MSE)
    np.testing.assert_allclose(game.error_from_outputs(out, t, game.RMSE), np.sqrt(mse), rtol=1e-15)
    tm = game.error_from_outputs(out, t, game.TMSE, 0.3)
    assert np.all(tm <= mse + 1e-15)
    # a tube of width 0 drops only exact zeros
    np.testing.assert_allclose(game.error_from_outputs(out, t, game.TMSE, 0.0), mse, rtol=1e-15)


# ------------------------------------------------------------------- fitness
@pytest.mark.parametrize("basis", BASES)
def test_noise_free_teacher_has_zero_fitness(basis):
    """A target produced by a chromosome (evaluated with numpy's polynomial
    library) is fitted exactly by that chromosome."""
    rng = np.random.default_rng(6)
    N, d = 5, 4
    X = rng.uniform(-1, 1, (400, N))
    K = game.num_genes(basis, N, d)
    w = rng.uniform(-1, 1, K)
    t = datagen.teacher_values(X, basis, d, w)
    f = game.fitness(X, t, w[None, :], basis, d)
    assert f[0] < 1e-28


@pytest.mark.parametrize("basis", BASES)
def test_fitness_never_beats_least_squares(basis):
    """MSE is a quadratic in the genes; no chromosome goes below the
    least-squares optimum of the same linear model."""
    rng = np.random.default_rng(7)
    N, d = 3, 3
    X = rng.uniform(-1, 1, (300, N))
    t = rng.normal(size=300)
    K = game.num_genes(basis, N, d)
    _, mse_ls = game.least_squares_optimum(X, t, basis, d)
    W = rng.uniform(-1, 1, (200, K))
    assert np.all(game.fitness(X, t, W, basis, d) >= mse_ls - 1e-12)


def test_brute_force_grid_approaches_least_squares():
    """Tiny problem (N = 1, d = 2, 6 patterns): the exhaustive grid over genes
    {-1, -0.9, ..., 1}^3 never beats MSE_LS and gets close to it when the
    optimum lies inside the gene range."""
    rng = np.random.default_rng(8)
    X = rng.uniform(-1, 1, (6, 1))
    w_true = np.array([0.3, -0.5, 0.7])
    t = datagen.teacher_values(X, game.CHEBYSHEV, 2, w_true) + 0.01 * rng.normal(size=6)
    _, mse_ls = game.least_squares_optimum(X, t, game.CHEBYSHEV, 2)
    grid = np.round(np.arange(-10, 11) / 10.0, 10)
    W = np.array(np.meshgrid(grid, grid, grid, indexing="ij")).reshape(3, -1).T
    f = game.fitness(X, t, W, game.CHEBYSHEV, 2)
    assert f.min() >= mse_ls - 1e-15
    assert f.min() - mse_ls < 5e-3


@pytest.mark.parametrize("basis", BASES)
def test_quadratic_form_equals_direct_sum(basis):
    rng = np.random.default_rng(9)
    N, d = 4, 3
    X = rng.uniform(-1, 1, (250, N))
    t = rng.normal(size=250)
    W = rng.uniform(-1, 1, (16, game.num_genes(basis, N, d)))
    np.testing.assert_allclose(game.fitness(X, t, W, basis, d),
                               game.quadratic_form_mse(X, t, W, basis, d), rtol=1e-9)


@pytest.mark.parametrize("reps", [2, 5])
def test_row_replication_leaves_fitness_unchanged(reps):
    """Replicating every row (the paper's way of growing the data set) leaves
    every MSE unchanged."""
    rng = np.random.default_rng(10)
    X = rng.uniform(-1, 1, (123, 6))
    t = rng.normal(size=123)
    W = rng.uniform(-1, 1, (9, game.num_genes(game.LEGENDRE, 6, 5)))
    f1 = game.fitness(X, t, W, game.LEGENDRE, 5)
    fr = game.fitness(np.tile(X, (reps, 1)), np.tile(t, reps), W, game.LEGENDRE, 5)
    np.testing.assert_allclose(fr, f1, rtol=1e-12)


def test_classification_merit_counts():
    """Four patterns with one of each outcome: TP, TN, FP, FN."""
    out = np.array([0.9, 0.1, 0.7, 0.2])
    t = np.array([1.0, 0.0, 0.0, 1.0])
    m = game.classification_merit(out, t)
    assert m["accuracy"] == 0.5
    assert m["completeness"] == 0.5
    assert m["contamination"] == 0.5
    assert m["contamination_of_predicted"] == 0.5
