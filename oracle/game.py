"""GAME fitness in float64: expansion, pattern output, error functions.

Test infrastructure (see ``oracle/__init__.py``).  Every function restates a
passage of the paper; none is tuned for speed.

Notation (Sec. 2): NP patterns, N features per pattern, degree d, B basis
blocks per feature (B = 2 for the trigonometric expansion of Eq. 8, else 1).

Gene layout (per-feature genes, one bias):
    gene 0                      -> a_0, the bias of Eq. 2
    gene 1 + i*B*d + b*d + j-1  -> feature i (0-based), block b, degree j=1..d
For the trigonometric basis block 0 carries cos(j x) and block 1 sin(j x),
which is the order [a_1..a_d, b_1..b_d] of the chromosome described after
Eq. 9, applied per feature.  The paper's own model shares a_j, b_j across
features (Eq. 2, Eq. 9); that model is the special case in which the genes
of all features are tied (checked in the tests).
"""
from __future__ import annotations

import numpy as np

CHEBYSHEV, LEGENDRE, POWER, TRIG = 0, 1, 2, 3
BASIS_NAMES = {"chebyshev": CHEBYSHEV, "legendre": LEGENDRE, "power": POWER, "trig": TRIG}

MSE, RMSE, TMSE = 0, 1, 2


def basis_id(basis) -> int:
    if isinstance(basis, str):
        return BASIS_NAMES[basis]
    return int(basis)


def blocks(basis) -> int:
    """B of Eq. 6/7: two coefficient groups (cos, sin) for Eq. 8, else one."""
    return 2 if basis_id(basis) == TRIG else 1


def num_genes(basis, n_features: int, degree: int) -> int:
    """Genes per chromosome: one bias plus B*d genes for each feature."""
    return blocks(basis) * n_features * degree + 1


def basis_table(x, basis, degree: int) -> np.ndarray:
    """phi_{b,j}(x) for b < B, j = 1..d, in float64; shape x.shape + (B, d).

    Eq. 1 writes G(f) = a_0 + sum_j a_j g^j(f), where g^j is the j-th member
    of the chosen function sequence (Eq. 8 makes it cos(jx) and sin(jx)).
      Chebyshev T_j: T_0 = 1, T_1 = x, T_{j+1} = 2x T_j - T_{j-1}
      Legendre  P_j: P_0 = 1, P_1 = x, (j+1) P_{j+1} = (2j+1) x P_j - j P_{j-1}
      power:         x^j
      trig (Eq. 8):  cos(j x) and sin(j x)
    """
    b = basis_id(basis)
    x = np.asarray(x, dtype=np.float64)
    out = np.empty(x.shape + (blocks(b), degree), dtype=np.float64)
    if b == TRIG:
        for j in range(1, degree + 1):
            out[..., 0, j - 1] = np.cos(j * x)
            out[..., 1, j - 1] = np.sin(j * x)
        return out
    prev = np.ones_like(x)  # member 0
    cur = x.copy()          # member 1
    for j in range(1, degree + 1):
        out[..., 0, j - 1] = cur
        if b == CHEBYSHEV:
            nxt = 2.0 * x * cur - prev
        elif b == LEGENDRE:
            nxt = ((2 * j + 1) * x * cur - j * prev) / (j + 1)
        elif b == POWER:
            nxt = x * cur
        else:
            raise ValueError(f"unknown basis {basis}")
        prev, cur = cur, nxt
    return out


def expand(X, basis, degree: int) -> np.ndarray:
    """Expanded design matrix Phi [NP, B*N*d] in the canonical gene order
    (column c = i*B*d + b*d + j-1 multiplies gene 1 + c)."""
    X = np.asarray(X, dtype=np.float64)
    tab = basis_table(X, basis, degree)          # [NP, N, B, d]
    return tab.reshape(X.shape[0], -1)


def outputs(X, genes, basis, degree: int) -> np.ndarray:
    """Out(pat_k) of Eq. 2 for every pattern k and chromosome p: [NP, P].

    Out = a_0 + sum_i sum_b sum_j gene(i,b,j) * phi_{b,j}(f_i)."""
    genes = np.atleast_2d(np.asarray(genes, dtype=np.float64))
    phi = expand(X, basis, degree)
    if phi.shape[1] + 1 != genes.shape[1]:
        raise ValueError("gene count does not match B*N*d+1")
    return genes[:, 0][None, :] + phi @ genes[:, 1:].T


def pattern_errors(out, t, error_fn=MSE, R: float = 0.0, literal_tmse: bool = False):
    """E_k per pattern (Eq. 3), or its thresholded form (Eq. 10).

    TMSE: the paper's worked example (R = 0.5 gives 0 for outputs 0.49/0.51
    and 0.13 for 0/0.49 on targets 0/1) holds only when a residual counts if
    |t - Out| > R, so that is the default reading; ``literal_tmse`` compares
    the squared residual with R as Eq. 10 is printed."""
    out = np.asarray(out, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    r = t.reshape((-1,) + (1,) * (out.ndim - 1)) - out
    e = r * r
    if error_fn == TMSE:
        keep = (e > R) if literal_tmse else (np.abs(r) > R)
        e = np.where(keep, e, 0.0)
    return e


def error_from_outputs(out, t, error_fn=MSE, R: float = 0.0, literal_tmse: bool = False):
    """MSE (Eq. 4), RMSE (Eq. 5) or TMSE (Eq. 10 averaged like Eq. 4) over
    the NP patterns along axis 0."""
    e = pattern_errors(out, t, error_fn, R, literal_tmse)
    m = e.sum(axis=0) / e.shape[0]
    return np.sqrt(m) if error_fn == RMSE else m


def fitness(X, t, genes, basis, degree: int, error_fn=MSE, R: float = 0.0,
            literal_tmse: bool = False) -> np.ndarray:
    """Fitness of each chromosome over the whole set: [P] float64."""
    return error_from_outputs(outputs(X, genes, basis, degree), t, error_fn, R, literal_tmse)


def least_squares_optimum(X, t, basis, degree: int):
    """The best chromosome of the model, ignoring the [-1, 1] gene range:
    Out is linear in the genes (Eq. 2), so min_w MSE is a linear least-squares
    problem on the design matrix [1, Phi].  Returns (w*, MSE_LS)."""
    phi = expand(X, basis, degree)
    A = np.concatenate([np.ones((phi.shape[0], 1)), phi], axis=1)
    t = np.asarray(t, dtype=np.float64)
    w, *_ = np.linalg.lstsq(A, t, rcond=None)
    r = t - A @ w
    return w, float(r @ r) / A.shape[0]


def quadratic_form_mse(X, t, genes, basis, degree: int) -> np.ndarray:
    """MSE(w) = (w^T G w - 2 b^T w + c) / NP with G = A^T A, b = A^T t,
    c = t^T t and A = [1, Phi]: the same quantity as Eq. 4, expanded."""
    phi = expand(X, basis, degree)
    A = np.concatenate([np.ones((phi.shape[0], 1)), phi], axis=1)
    t = np.asarray(t, dtype=np.float64)
    G = A.T @ A
    bv = A.T @ t
    c = t @ t
    W = np.atleast_2d(np.asarray(genes, dtype=np.float64))
    return (np.einsum("pk,kl,pl->p", W, G, W) - 2.0 * W @ bv + c) / A.shape[0]


def classification_merit(out, t, threshold: float = 0.5):
    """Accuracy, completeness and contamination (Sec. 5, figures of merit).

    A pattern is predicted as class 1 when Out >= threshold.  Accuracy is the
    fraction classified correctly; completeness the fraction of class-1
    patterns predicted as 1; contamination the fraction of class-0 patterns
    predicted as 1, as the paper defines it.  The other common convention,
    the fraction of predicted-1 patterns that are class 0, is returned too."""
    out = np.asarray(out, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    pred = out >= threshold
    pos = t > 0.5
    tp = float(np.sum(pred & pos))
    tn = float(np.sum(~pred & ~pos))
    fp = float(np.sum(pred & ~pos))
    fn = float(np.sum(~pred & pos))
    n = tp + tn + fp + fn
    return {
        "accuracy": (tp + tn) / n if n else float("nan"),
        "completeness": tp / (tp + fn) if tp + fn else float("nan"),
        "contamination": fp / (fp + tn) if fp + tn else float("nan"),
        "contamination_of_predicted": fp / (tp + fp) if tp + fp else float("nan"),
    }


# ------------------------------------------------ the paper's shared-gene model
def shared_trig_sums(X, degree: int) -> np.ndarray:
    """Per-pattern sums of Eq. 9 that do not depend on the genes, computed
    once per data set (Sec. 4.1 keeps the cos/sin sums out of the training
    loop): column j-1 is sum_i cos(j f_i), column d+j-1 is sum_i sin(j f_i),
    j = 1..d; shape [NP, 2d], float64."""
    X = np.asarray(X, dtype=np.float64)
    j = np.arange(1, degree + 1, dtype=np.float64)
    ang = X[:, :, None] * j[None, None, :]                  # [NP, N, d]
    return np.concatenate([np.cos(ang).sum(axis=1), np.sin(ang).sum(axis=1)], axis=1)


def shared_trig_outputs(X, genes, degree: int) -> np.ndarray:
    """Out of Eq. 9 with the genes shared by all features, chromosome
    [a_0, a_1..a_d, b_1..b_d] (2d+1 genes, Eq. 7): [NP, P]."""
    genes = np.atleast_2d(np.asarray(genes, dtype=np.float64))
    if genes.shape[1] != 2 * degree + 1:
        raise ValueError("the shared model has 2d+1 genes")
    S = shared_trig_sums(X, degree)
    return genes[:, 0][None, :] + S @ genes[:, 1:].T


def shared_trig_fitness(X, t, genes, degree: int, error_fn=MSE, R: float = 0.0,
                        literal_tmse: bool = False) -> np.ndarray:
    """Fitness of each shared-gene chromosome over the whole set: [P]."""
    return error_from_outputs(shared_trig_outputs(X, genes, degree), t, error_fn, R, literal_tmse)
