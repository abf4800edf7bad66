"""BF16 fitness form and the float64 re-score against the float64 oracle.

BF16 tolerance, derived from the arithmetic (not fitted).  For pattern k let
S_k = sum_c |phi_kc w_c| (float64, from the oracle's expansion).  Each
product of two round-to-nearest-even bfloat16 values has relative error at
most 2^-8 + 2^-18; the float32 recurrence that produces phi adds at most
d^2 2^-24 <= 2^-16 relative; float32 accumulation of K terms adds at most
K 2^-24 of S_k; the epilogue's float32 bias add and subtraction add at most
2^-23 (|Out_k| + |t_k|).  So |dOut_k| <= delta_k with
    delta_k = (2^-8 + 2^-16 + K 2^-24) S_k + 2^-23 (|Out_k| + |t_k|),
and by Cauchy-Schwarz the error of the mean of squared residuals is at most
    2 sqrt(MSE) sqrt(mean delta^2) + mean delta^2,
plus 2^-18 MSE for the float32 sums of 32 squares per tile.
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


def bf16_bound(X, t, W, basis, d):
    phi = og.expand(X, basis, d)
    W64 = np.asarray(W, np.float64)
    S = np.abs(phi) @ np.abs(W64[:, 1:]).T                    # [NP, P]
    out = W64[:, 0][None, :] + phi @ W64[:, 1:].T
    K = W.shape[1]
    delta = (2.0 ** -8 + 2.0 ** -16 + K * 2.0 ** -24) * S \
        + 2.0 ** -23 * (np.abs(out) + np.abs(np.asarray(t, np.float64))[:, None])
    mse = og.error_from_outputs(out, t)
    md2 = np.mean(delta ** 2, axis=0)
    return mse, 2 * np.sqrt(mse) * np.sqrt(md2) + md2 + 2.0 ** -18 * mse


def make_game(gg, X, t, basis, d, P, precision=1, **kw):
    c = gg.config(basis=basis, degree=d, population=max(P, 2), tournament_k=min(3, max(P, 2)),
                  elitism=1, precision=precision, **kw)
    return gg.Game(c, torch.from_numpy(np.ascontiguousarray(X)).cuda(),
                   torch.from_numpy(np.ascontiguousarray(t)).cuda())


def problem(NP, N, d, P, basis, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, (NP, N)).astype(np.float32)
    t = rng.normal(0, 1, NP).astype(np.float32)
    W = rng.uniform(-1, 1, (P, og.num_genes(basis, N, d))).astype(np.float32)
    return X, t, W


# Feature counts that are multiples of 4 take the LDS-copy path for features
# and targets (several tiles per workgroup in the 70,000-row case, so both
# buffers alternate; ragged last tiles); the others load into registers.
SHAPES = [(1, 1, 1, 1), (300, 3, 8, 130), (1000, 7, 4, 50), (777, 9, 3, 129), (513, 5, 16, 64),
          (2049, 33, 8, 200), (600, 20, 5, 257), (256, 64, 2, 128), (1000, 8, 4, 50),
          (3001, 12, 7, 130), (515, 4, 16, 64), (4099, 32, 8, 129), (70000, 16, 3, 40),
          (300001, 4, 2, 10)]


@pytest.mark.parametrize("basis", [0, 1, 2, 3])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_bf16_within_derived_bound(gg, basis, shape):
    NP, N, d, P = shape
    X, t, W = problem(NP, N, d, P, basis, seed=sum(shape) + basis)
    g = make_game(gg, X, t, basis, d, P)
    f32, f64 = g.fitness(torch.from_numpy(W).cuda(), with64=True)
    f64 = f64.cpu().numpy()
    ref, bound = bf16_bound(X, t, W, basis, d)
    err = np.abs(f64 - ref)
    assert np.all(err <= bound), (np.max(err / bound), np.max(err / ref))
    g.close()


@pytest.mark.parametrize("basis", [0, 1, 2, 3])
@pytest.mark.parametrize("d", [1, 2, 3, 5, 6, 7, 9, 11, 15, 16])
def test_bf16_every_group_shape(gg, basis, d):
    """Degrees that are not divisors of 8 pack several sub-features into a
    lane's 8 values (G = 8 / gcd(d, 8) per group)."""
    X, t, W = problem(400, 5, d, 33, basis, seed=40 + d)
    g = make_game(gg, X, t, basis, d, 33)
    f64 = g.fitness(torch.from_numpy(W).cuda(), with64=True)[1].cpu().numpy()
    ref, bound = bf16_bound(X, t, W, basis, d)
    assert np.all(np.abs(f64 - ref) <= bound)
    g.close()


@pytest.mark.parametrize("basis", [0, 1, 2, 3])
def test_rescore64_matches_oracle(gg, basis):
    X, t, W = problem(3000, 6, 7, 40, basis, seed=50 + basis)
    g = make_game(gg, X, t, basis, 7, 40)
    r = g.rescore64(torch.from_numpy(W).cuda()).cpu().numpy()
    ref = og.fitness(X, t, W, basis, 7)
    np.testing.assert_allclose(r, ref, rtol=1e-11)
    Xv, tv, _ = problem(777, 6, 7, 1, basis, seed=60 + basis)
    rv = g.rescore64(torch.from_numpy(W[:5]).cuda(), torch.from_numpy(Xv).cuda(),
                     torch.from_numpy(tv).cuda()).cpu().numpy()
    np.testing.assert_allclose(rv, og.fitness(Xv, tv, W[:5], basis, 7), rtol=1e-11)
    g.close()


def test_rescore64_tmse(gg):
    X, t, W = problem(2000, 4, 3, 20, 0, seed=70)
    t = (t > 0).astype(np.float32)
    W *= 0.2
    g = make_game(gg, X, t, 0, 3, 20, error_fn=2, tmse_R=0.49)
    r = g.rescore64(torch.from_numpy(W).cuda()).cpu().numpy()
    ref = og.fitness(X, t, W, 0, 3, og.TMSE, 0.49)
    np.testing.assert_allclose(r, ref, rtol=1e-11)
    g.close()


def test_bf16_deterministic(gg):
    X, t, W = problem(5000, 12, 8, 300, 0, seed=80)
    g = make_game(gg, X, t, 0, 8, 300)
    Wd = torch.from_numpy(W).cuda()
    a = g.fitness(Wd, with64=True)[1].cpu().numpy()
    b = g.fitness(Wd, with64=True)[1].cpu().numpy()
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    g.close()


def test_bf16_run_reports_float64_elite(gg):
    """A BF16 run: the genetic step is driven by BF16 fitness, the reported
    elite error is its float64 re-score."""
    prob = datagen.small()
    g = make_game(gg, prob.X, prob.t, prob.basis, prob.degree, prob.population, seed=5,
                  max_generations=25, target=0.0)
    g.init_population()
    gens, best, err = g.run()
    assert gens == 25
    ref = og.fitness(prob.X, prob.t, best[None, :], prob.basis, prob.degree)[0]
    assert abs(err - ref) <= 1e-11 * ref
    pop, fit = g.population()
    st = g.state()
    bf = float(fit.cpu().numpy()[st["best_index"]])
    _, bound = bf16_bound(prob.X, prob.t, best[None, :], prob.basis, prob.degree)
    assert abs(bf - ref) <= bound[0] + 1e-7 * ref
    g.close()


def test_precision_workload_sampled(gg):
    """1,000,000 x 32, Chebyshev d=8 (257 genes), 4,096 chromosomes in one
    launch; the float64 re-score (checked against the oracle on a few) gives
    the per-result error of the BF16 values."""
    prob = datagen.precision()
    P = prob.population
    W = datagen.random_genes(P, prob.n_genes, 13)
    g = make_game(gg, prob.X, prob.t, prob.basis, prob.degree, P)
    Wd = torch.from_numpy(W).cuda()
    f64 = g.fitness(Wd, with64=True)[1].cpu().numpy()
    idx = np.array([0, 1, 777, 2048, P - 1])
    r64 = g.rescore64(Wd[idx].contiguous()).cpu().numpy()
    ref, bound = bf16_bound(prob.X, prob.t, W[idx], prob.basis, prob.degree)
    np.testing.assert_allclose(r64, ref, rtol=1e-10)
    assert np.all(np.abs(f64[idx] - ref) <= bound), np.abs(f64[idx] - ref) / bound
    g.close()
