"""The "run" use case (model outputs of given chromosomes) and the
classification counts behind the figures of merit, against the float64
oracle.

Tolerance of an output, derived from the float32 arithmetic: each basis
value phi_j (|phi| <= 1 for features in [-1, 1] and for cos/sin) carries at
most about (j^2 + 2) units of 2^-24 from its recurrence, and the fused
multiply-add chain over the K genes adds at most K + 1 units relative to the
running sum, whose magnitude stays below sum |w|.  So
|Out_gpu - Out_oracle| <= 2 * 2^-24 * (K + 1 + d^2 + 2) * sum_c |w_c|.
A class decision is compared only where the oracle's output is farther
than that from the threshold; closer patterns may go either way.
"""
import numpy as np
import pytest

from oracle import game as og
from paper_1304_0597_amd import datagen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gg():
    from paper_1304_0597_amd import game
    game.lib()
    return game


def bound(genes, K, d):
    return 2.0 * 2.0 ** -24 * (K + 1 + d * d + 2) * np.abs(genes.astype(np.float64)).sum(axis=1)


def make(gg, basis, d, NP, N, P=8, seed=0, binary=True):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, (NP, N)).astype(np.float32)
    t = (rng.random(NP) < 0.5).astype(np.float32) if binary else rng.normal(0, 1, NP).astype(np.float32)
    c = gg.config(basis=basis, degree=d, population=P, tournament_k=min(3, P),
                  elitism=min(2, P - 1), seed=seed)
    g = gg.Game(c, torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda())
    return X, t, g


@pytest.mark.parametrize("basis", [0, 1, 2, 3])
@pytest.mark.parametrize("d,NP,N,n", [(1, 1, 1, 1), (4, 1000, 7, 3), (8, 3001, 20, 5),
                                      (16, 515, 3, 2)])
def test_predict_matches_oracle(gg, basis, d, NP, N, n):
    X, t, g = make(gg, basis, d, NP, N, P=max(n, 2))
    K = g.n_genes
    genes = np.random.default_rng(d + NP).uniform(-1, 1, (n, K)).astype(np.float32)
    out = g.predict(torch.from_numpy(genes).cuda()).cpu().numpy()
    ref = og.outputs(X, genes, basis, d).T                     # [n, NP]
    tol = bound(genes, K, d)[:, None]
    assert out.shape == (n, NP)
    assert np.all(np.abs(out - ref) <= tol)
    # another data set of the same feature count
    X2 = np.random.default_rng(9).uniform(-1, 1, (77, N)).astype(np.float32)
    out2 = g.predict(torch.from_numpy(genes).cuda(), torch.from_numpy(X2).cuda()).cpu().numpy()
    assert np.all(np.abs(out2 - og.outputs(X2, genes, basis, d).T) <= tol)
    g.close()


def _counts_from(out, t, thr):
    pred = out >= thr
    pos = t > 0.5
    return np.stack([(pred & pos).sum(1), (pred & ~pos).sum(1), (~pred & ~pos).sum(1),
                     (~pred & pos).sum(1)], axis=1)


@pytest.mark.parametrize("basis,d,thr", [(0, 4, 0.5), (1, 6, 0.5), (2, 3, 0.0), (3, 2, 0.25)])
def test_classify_counts(gg, basis, d, thr):
    NP, N, n = 4099, 9, 4
    X, t, g = make(gg, basis, d, NP, N, P=n, seed=basis)
    K = g.n_genes
    genes = np.random.default_rng(basis).uniform(-0.2, 0.2, (n, K)).astype(np.float32)
    genes[:, 0] = 0.5
    gd = torch.from_numpy(genes).cuda()
    counts = g.classify(gd, threshold=thr).cpu().numpy()
    assert np.all(counts.sum(1) == NP)
    # the same decisions as the stored float32 outputs
    out = g.predict(gd).cpu().numpy()
    assert np.array_equal(counts, _counts_from(out, t, thr))
    # the oracle's decisions wherever they are unambiguous
    ref = og.outputs(X, genes, basis, d).T
    sure = np.abs(ref - thr) > bound(genes, K, d)[:, None]
    pos = t > 0.5
    for r in range(n):
        s = sure[r]
        lo = _counts_from(ref[r:r + 1, s], t[s], thr)[0]
        amb_pos, amb_neg = int((~s & pos).sum()), int((~s & ~pos).sum())
        tp, fp, tn, fn = counts[r]
        assert lo[0] <= tp <= lo[0] + amb_pos and lo[3] <= fn <= lo[3] + amb_pos
        assert lo[1] <= fp <= lo[1] + amb_neg and lo[2] <= tn <= lo[2] + amb_neg
    g.close()


def test_merit_of_a_trained_run(gg):
    """The small binary workload trained for 30 generations; the best
    chromosome's figures of merit on its validation set against the oracle's
    classification_merit of the oracle outputs."""
    prob = datagen.small()
    c = gg.config(basis=prob.basis, degree=prob.degree, population=prob.population, seed=0,
                  max_generations=30, target=0.0)
    g = gg.Game(c, torch.from_numpy(prob.X).cuda(), torch.from_numpy(prob.t).cuda())
    g.init_population()
    _, best, _ = g.run()
    Xv, tv = torch.from_numpy(prob.X_val).cuda(), torch.from_numpy(prob.t_val).cuda()
    counts = g.classify(torch.from_numpy(best).cuda().view(1, -1), Xv, tv).cpu().numpy()[0]
    m = gg.game_merit(counts)
    ref = og.classification_merit(og.outputs(prob.X_val, best[None, :], prob.basis,
                                             prob.degree)[:, 0], prob.t_val)
    n = len(prob.t_val)
    for k in ("accuracy", "completeness", "contamination", "contamination_of_predicted"):
        # at most a couple of borderline decisions may differ
        assert abs(m[k] - ref[k]) <= 3.0 / max(1, min(n, counts.sum())) + 1e-12 or (
            np.isnan(m[k]) and np.isnan(ref[k])), k
    g.close()


def test_predict_rejects_bad_arguments(gg):
    X, t, g = make(gg, 0, 2, 10, 2, P=2)
    genes = torch.zeros((1, g.n_genes), device="cuda")
    with pytest.raises(gg.GameError):
        gg.game_predict(g.h, None, genes, 0, torch.empty((1, 10), device="cuda"))
    with pytest.raises(gg.GameError):
        gg.game_classify(g.h, torch.from_numpy(X).cuda(), None, genes, 1, 0.5,
                         torch.empty((1, 4), dtype=torch.int64, device="cuda"))
    g.close()
