"""Seeded synthetic workloads.

The paper trains on 2,100 HST sources with 11 features and a 0/1 label and
scales up by replicating rows; that catalogue is not available, so these
generators stand in for it with inputs of the same structure: homogeneous
patterns of N features in [-1, 1] and one target each, either a noisy binary
label (a low signal-to-noise classification problem) or a noisy regression
value.

Teachers are random polynomials in the same per-feature basis the model
uses; their values come from numpy's own polynomial evaluators
(``numpy.polynomial.chebyshev.chebval`` and friends), so this module holds
none of the model's arithmetic and serves the oracle and the HIP path alike.

Workloads (all float32, row-major X [NP, N], t [NP]):
  small     2,000 x 7 uniform, Chebyshev d=4 binary teacher, 5 % label flips
  scale     200,000 x 20, mixture of three Gaussians clipped to [-1, 1],
            Legendre d=8 teacher + N(0, 0.05^2)
  precision 1,000,000 x 32 uniform, Chebyshev d=8 binary teacher, 5 % flips
  batched   256 runs with sizes drawn from seed 3
Validation sets have NP/4 rows drawn from seed + 1.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from numpy.polynomial import chebyshev, legendre, polynomial

CHEBYSHEV, LEGENDRE, POWER, TRIG = 0, 1, 2, 3


def _per_feature_values(x, basis: int, coeffs_1_to_d: np.ndarray) -> np.ndarray:
    """Library evaluation of sum_j c_j phi_j(x), j = 1..d, for one feature
    column (trigonometric: two coefficient rows, cos then sin)."""
    if basis == TRIG:
        d = coeffs_1_to_d.shape[-1]
        j = np.arange(1, d + 1, dtype=np.float64)
        ang = np.multiply.outer(x, j)
        return np.cos(ang) @ coeffs_1_to_d[0] + np.sin(ang) @ coeffs_1_to_d[1]
    c = np.concatenate([[0.0], coeffs_1_to_d[0]])
    ev = {CHEBYSHEV: chebyshev.chebval, LEGENDRE: legendre.legval,
          POWER: polynomial.polyval}[basis]
    return ev(x, c)


def teacher_values(X, basis: int, degree: int, genes: np.ndarray) -> np.ndarray:
    """float64 value of the teacher polynomial whose genes follow the
    library's canonical layout (bias, then per feature, block, degree)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[1]
    B = 2 if basis == TRIG else 1
    per = genes[1:].reshape(n, B, degree)
    out = np.full(X.shape[0], float(genes[0]))
    for i in range(n):
        out += _per_feature_values(X[:, i], basis, per[i])
    return out


@dataclasses.dataclass
class Problem:
    name: str
    basis: int
    degree: int
    X: np.ndarray
    t: np.ndarray
    X_val: np.ndarray
    t_val: np.ndarray
    teacher: np.ndarray
    population: int
    generations: int
    binary: bool

    @property
    def n_patterns(self) -> int:
        return self.X.shape[0]

    @property
    def n_features(self) -> int:
        return self.X.shape[1]

    @property
    def n_genes(self) -> int:
        return (2 if self.basis == TRIG else 1) * self.n_features * self.degree + 1


def _uniform_x(rng, n, nf):
    return rng.uniform(-1.0, 1.0, size=(n, nf))


def _mixture_x(rng, n, nf, means, sigmas):
    comp = rng.integers(0, len(means), size=n)
    x = means[comp] + rng.standard_normal((n, nf)) * sigmas[comp][:, None]
    return np.clip(x, -1.0, 1.0)


def binary_problem(name, n, nf, basis, degree, population, generations, seed=0, flip=0.05):
    """Binary label 1[teacher(x) > 0] with a fraction ``flip`` of labels
    flipped (the noisy 0/1 classification setting of the paper)."""
    rng = np.random.default_rng(seed)
    K = (2 if basis == TRIG else 1) * nf * degree + 1
    teacher = rng.uniform(-1.0, 1.0, size=K)
    sets = []
    for s, rows in ((seed, n), (seed + 1, max(1, n // 4))):
        r = np.random.default_rng(s) if s != seed else rng
        X = _uniform_x(r, rows, nf)
        y = (teacher_values(X, basis, degree, teacher) > 0).astype(np.float64)
        y = np.where(r.random(rows) < flip, 1.0 - y, y)
        sets.append((X.astype(np.float32), y.astype(np.float32)))
    (X, t), (Xv, tv) = sets
    return Problem(name, basis, degree, X, t, Xv, tv, teacher, population, generations, True)


def regression_problem(name, n, nf, basis, degree, population, generations, seed=0,
                       noise=0.05, mixture=0, with_validation=True):
    """Regression target teacher(x) + N(0, noise^2); X uniform in [-1, 1] or,
    with ``mixture`` > 0, an equal-weight mixture of that many isotropic
    Gaussians (means U[-0.5, 0.5], widths U[0.2, 0.5]) clipped to [-1, 1]."""
    rng = np.random.default_rng(seed)
    K = (2 if basis == TRIG else 1) * nf * degree + 1
    teacher = rng.uniform(-1.0, 1.0, size=K)
    if mixture:
        means = rng.uniform(-0.5, 0.5, size=(mixture, nf))
        sigmas = rng.uniform(0.2, 0.5, size=mixture)
    sets = []
    parts = ((seed, n), (seed + 1, max(1, n // 4))) if with_validation else ((seed, n),)
    for s, rows in parts:
        r = np.random.default_rng(s) if s != seed else rng
        X = _mixture_x(r, rows, nf, means, sigmas) if mixture else _uniform_x(r, rows, nf)
        y = teacher_values(X, basis, degree, teacher) + noise * r.standard_normal(rows)
        sets.append((X.astype(np.float32), y.astype(np.float32)))
    (X, t) = sets[0]
    (Xv, tv) = sets[1] if with_validation else (X[:0], t[:0])
    return Problem(name, basis, degree, X, t, Xv, tv, teacher, population, generations, False)


def small(seed=0):
    """2,000 x 7, Chebyshev d=4 (29 genes), population 50, 100 generations."""
    return binary_problem("small", 2000, 7, CHEBYSHEV, 4, 50, 100, seed)


def scale(seed=0, n=200_000):
    """200,000 x 20, Legendre d=8 (161 genes), population 2,048, 1,000 generations."""
    return regression_problem("scale", n, 20, LEGENDRE, 8, 2048, 1000, seed, mixture=3)


def precision(seed=0, n=1_000_000):
    """1,000,000 x 32, Chebyshev d=8 (257 genes), population 4,096."""
    return binary_problem("precision", n, 32, CHEBYSHEV, 8, 4096, 1000, seed)


def paper_shaped(seed=0):
    """The shape of the paper's knowledge base: 2,100 patterns x 11 features
    with a 0/1 label (here from a random degree-4 trigonometric teacher with
    5% flips), for the shared-gene polytrigo model with 23 chromosomes
    (2N + 1) and 4,000 generations.  Larger sets replicate its rows."""
    return binary_problem("paper-shaped", 2100, 11, TRIG, 4, 23, 4000, seed)


# Data sizes of the paper's scaling table and the rows that reproduce them
# by replicating the 2,100-row set (0.15 MB holds the 2,100 rows).
PAPER_SIZES_MB = (0.15, 16, 128, 512)


def paper_rows(size_mb: float) -> int:
    return int(round(2100 * size_mb / 0.15))


@dataclasses.dataclass
class RunShape:
    n_patterns: int
    n_features: int
    degree: int
    population: int
    basis: int


def batched_shapes(n_runs=256, seed=3):
    """Sizes of the independent runs of the batched workload: patterns
    log-uniform in [1e3, 2e5], features 4..64, degree 2..10, population
    32..1024, Chebyshev or power basis with equal probability."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_runs):
        n = int(round(math.exp(rng.uniform(math.log(1e3), math.log(2e5)))))
        nf = int(rng.integers(4, 65))
        d = int(rng.integers(2, 11))
        p = int(rng.integers(32, 1025))
        b = CHEBYSHEV if rng.random() < 0.5 else POWER
        out.append(RunShape(n, nf, d, p, b))
    return out


def batched_problem(shape: RunShape, run_index: int, base_seed=3, with_validation=True):
    """One run of the batched workload: X uniform, teacher + N(0, 0.05^2)."""
    return regression_problem(f"batched{run_index}", shape.n_patterns, shape.n_features,
                              shape.basis, shape.degree, shape.population, 100,
                              seed=base_seed * 100_003 + run_index,
                              with_validation=with_validation)


def random_genes(P, K, seed, low=-1.0, high=1.0):
    """Random chromosomes (float32) for fitness-only tests."""
    return np.random.default_rng(seed).uniform(low, high, size=(P, K)).astype(np.float32)
