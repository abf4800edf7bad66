"""Parity of the HIP fitness kernels with the float64 oracle.

Tolerance (float32 path): |f_gpu - f_ref| <= 1e-5 * f_ref + 1e-7 * mean(t^2),
a relative bound with an absolute floor for fitness values near zero.
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


def within(f_gpu, f_ref, t, rel=1e-5, floor=1e-7):
    bound = rel * np.abs(f_ref) + floor * float(np.mean(np.asarray(t, np.float64) ** 2))
    return np.abs(np.asarray(f_gpu, np.float64) - f_ref) <= bound


def gpu_fitness(gg, basis, d, X, t, W, error_fn=0, R=0.49):
    P = max(2, W.shape[0])
    cfg = gg.config(basis=basis, degree=d, population=P, tournament_k=min(3, P), elitism=1,
                    error_fn=error_fn, tmse_R=R)
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    td = torch.from_numpy(np.ascontiguousarray(t)).cuda()
    Wd = torch.from_numpy(np.ascontiguousarray(W)).cuda()
    g = gg.Game(cfg, Xd, td)
    f, f64 = g.fitness(Wd, with64=True)
    torch.cuda.synchronize()
    out = f.cpu().numpy(), f64.cpu().numpy()
    g.close()
    return out


def problem(NP, N, d, P, basis, seed, binary=False, edge=False):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1, 1, (NP, N)).astype(np.float32)
    if edge:
        X[::3] = np.sign(X[::3]) * np.float32(1.0)
    t = (rng.random(NP) < 0.5).astype(np.float32) if binary else \
        rng.normal(0, 2, NP).astype(np.float32)
    K = og.num_genes(basis, N, d)
    W = rng.uniform(-1, 1, (P, K)).astype(np.float32)
    return X, t, W


SHAPES = [
    # NP, N, d, P: tails of the 256-row tile and the 64-chromosome tile,
    # odd feature counts, K-chunking (more than 128 K-steps per lane half)
    (1, 1, 1, 1), (7, 3, 2, 5), (255, 4, 3, 63), (256, 5, 4, 64), (257, 7, 4, 65),
    (2000, 7, 4, 50), (3001, 20, 8, 130), (777, 9, 5, 129), (600, 1, 16, 3),
    (513, 64, 2, 100), (300, 33, 10, 70), (1100, 300, 1, 66),
    # few chromosomes over many patterns: hundreds of pattern splits
    (300001, 4, 2, 10),
    # 128-chromosome tiles over splits of 4 pattern tiles and a last split
    # of 3 (the two wave groups of a workgroup walk unequal tile counts),
    # with the genes in one chunk and in chunks (180 K-steps per lane half)
    (100000, 5, 3, 200), (100000, 40, 9, 150),
    # K-chunks through the two gene buffers over several tiles per split,
    # odd sub-feature count (zeroed half pair in the last chunk)
    (8000, 33, 10, 1100),
]


@pytest.mark.parametrize("basis", [0, 1, 2, 3])
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_fitness_matches_oracle(gg, basis, shape):
    NP, N, d, P = shape
    if basis == 3 and N * 2 * d + 1 > 4097:
        pytest.skip("too many genes")
    X, t, W = problem(NP, N, d, P, basis, seed=NP + N + d + P + basis)
    f32, f64 = gpu_fitness(gg, basis, d, X, t, W)
    ref = og.fitness(X, t, W, basis, d)
    ok = within(f64, ref, t)
    assert ok.all(), (np.max(np.abs(f64 - ref) / ref), f64[~ok][:4], ref[~ok][:4])
    assert np.array_equal(f32, f64.astype(np.float32))


@pytest.mark.parametrize("basis", [0, 1, 2, 3])
@pytest.mark.parametrize("d", list(range(1, 17)))
def test_every_degree(gg, basis, d):
    N = 3
    X, t, W = problem(300, N, d, 17, basis, seed=100 + d, edge=True)
    _, f64 = gpu_fitness(gg, basis, d, X, t, W)
    ref = og.fitness(X, t, W, basis, d)
    assert within(f64, ref, t).all(), np.max(np.abs(f64 - ref) / ref)


def test_noise_free_teacher_is_near_zero(gg):
    """Targets produced by a chromosome: the GPU error of that chromosome is
    zero up to float32 rounding of the outputs."""
    rng = np.random.default_rng(5)
    X = rng.uniform(-1, 1, (5000, 7)).astype(np.float32)
    w = rng.uniform(-1, 1, 29).astype(np.float32)
    t = datagen.teacher_values(X, 0, 4, w.astype(np.float64)).astype(np.float32)
    W = np.stack([w, rng.uniform(-1, 1, 29).astype(np.float32)])
    _, f64 = gpu_fitness(gg, 0, 4, X, t, W)
    assert f64[0] < 1e-10
    assert f64[1] > 1e-2


@pytest.mark.parametrize("error_fn", [1, 2, 3])
def test_error_functions(gg, error_fn):
    R = 0.49
    X, t, W = problem(1500, 6, 3, 40, 0, seed=7, binary=True)
    W *= 0.2
    _, f64 = gpu_fitness(gg, 0, 3, X, t, W, error_fn=error_fn, R=R)
    out = og.outputs(X, W, 0, 3)
    kind = {1: og.RMSE, 2: og.TMSE, 3: og.TMSE}[error_fn]
    ref = og.error_from_outputs(out, t, kind, R, literal_tmse=(error_fn == 3))
    if error_fn == 1:
        assert within(f64, ref, t).all()
        return
    # A residual within float32 rounding of the threshold may fall on either
    # side; allow its whole contribution for each such pattern.
    r = t.astype(np.float64)[:, None] - out
    q = np.abs(r) if error_fn == 2 else r * r
    near = np.abs(q - R) <= 1e-5 * np.maximum(1.0, np.abs(q))
    budget = (near * (r * r)).sum(axis=0) / X.shape[0]
    floor = 1e-7 * float(np.mean(t.astype(np.float64) ** 2))
    assert np.all(np.abs(f64 - ref) <= 1e-5 * ref + floor + budget)
    # thresholding only drops terms: never above the plain MSE (same tolerance)
    mse = og.fitness(X, t, W, 0, 3)
    assert np.all(f64 <= mse + 1e-5 * mse + floor)


def test_nan_input_gives_infinite_error(gg):
    X, t, W = problem(500, 4, 3, 10, 0, seed=8)
    X[123, 2] = np.nan
    f32, f64 = gpu_fitness(gg, 0, 3, X, t, W)
    assert np.all(np.isinf(f32)) and np.all(np.isinf(f64))


@pytest.mark.parametrize("P", [10, 200], ids=["64-chromosome-tiles", "128-chromosome-tiles"])
def test_non_finite_genes_give_infinite_error(gg, P):
    """Rows past the data take a zero A operand; a chromosome with a NaN or
    infinite gene must still end at +inf (its valid rows are non-finite),
    and its neighbours must keep their oracle values, over a ragged last
    pattern tile (777 rows)."""
    X, t, W = problem(777, 5, 3, P, 0, seed=11)
    bad = [1, P // 2, P - 1]
    W[bad[0], 4] = np.nan
    W[bad[1], 7] = -np.inf
    W[bad[2], 0] = np.inf           # the bias gene
    f32, f64 = gpu_fitness(gg, 0, 3, X, t, W)
    assert np.all(np.isposinf(f32[bad])) and np.all(np.isposinf(f64[bad]))
    good = np.setdiff1d(np.arange(P), bad)
    ref = og.fitness(X, t, W[good], 0, 3)
    assert within(f64[good], ref, t).all()


def test_deterministic_bitwise(gg):
    X, t, W = problem(4000, 11, 6, 200, 1, seed=9)
    a = gpu_fitness(gg, 1, 6, X, t, W)[1]
    b = gpu_fitness(gg, 1, 6, X, t, W)[1]
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_row_replication_invariance(gg):
    """Replicating the data set (the paper's scale-up) changes the error only
    by float rounding."""
    X, t, W = problem(700, 5, 4, 30, 0, seed=10)
    _, f1 = gpu_fitness(gg, 0, 4, X, t, W)
    _, f4 = gpu_fitness(gg, 0, 4, np.tile(X, (4, 1)), np.tile(t, 4), W)
    np.testing.assert_allclose(f4, f1, rtol=2e-6)


def test_evaluate_on_validation_set(gg):
    prob = datagen.small()
    Xd = torch.from_numpy(prob.X).cuda()
    td = torch.from_numpy(prob.t).cuda()
    cfg = gg.config(basis=prob.basis, degree=prob.degree, population=prob.population)
    g = gg.Game(cfg, Xd, td)
    W = datagen.random_genes(prob.population, prob.n_genes, 3)
    err = g.evaluate(torch.from_numpy(prob.X_val).cuda(), torch.from_numpy(prob.t_val).cuda(),
                     torch.from_numpy(W).cuda()).cpu().numpy()
    ref = og.fitness(prob.X_val, prob.t_val, W, prob.basis, prob.degree)
    assert within(err, ref, prob.t_val).all()
    g.close()


def test_small_workload_all_chromosomes(gg):
    prob = datagen.small()
    W = datagen.random_genes(prob.population, prob.n_genes, 11)
    _, f64 = gpu_fitness(gg, prob.basis, prob.degree, prob.X, prob.t, W)
    ref = og.fitness(prob.X, prob.t, W, prob.basis, prob.degree)
    assert within(f64, ref, prob.t).all()


def test_scale_workload_sampled(gg):
    """200,000 x 20, Legendre d=8, 2,048 chromosomes in the launch the
    benchmark times; the oracle scores a sample of 48 chromosomes."""
    prob = datagen.scale()
    W = datagen.random_genes(prob.population, prob.n_genes, 12)
    f32, f64 = gpu_fitness(gg, prob.basis, prob.degree, prob.X, prob.t, W)
    idx = np.random.default_rng(0).choice(prob.population, 48, replace=False)
    idx = np.concatenate([idx, [0, prob.population - 1]])
    ref = og.fitness(prob.X, prob.t, W[idx], prob.basis, prob.degree)
    assert within(f64[idx], ref, prob.t).all(), np.max(np.abs(f64[idx] - ref) / ref)


def test_precision_shape_fp32_sampled(gg):
    """1,000,000 x 32, Chebyshev d=8 (257 genes), 4,096 chromosomes in one
    float32 launch (the shape of the plain float32 reference run of the
    time-to-target comparison): 32 chromosomes, among them the first and last
    of the first and last 64-chromosome tiles, against the float64 oracle."""
    prob = datagen.precision()
    P = prob.population
    W = datagen.random_genes(P, prob.n_genes, 14)
    f32, f64 = gpu_fitness(gg, prob.basis, prob.degree, prob.X, prob.t, W)
    rng = np.random.default_rng(1)
    edges = [0, 63, P - 64, P - 1]
    rest = rng.choice(np.setdiff1d(np.arange(P), edges), 28, replace=False)
    idx = np.sort(np.concatenate([edges, rest]))
    ref = og.fitness(prob.X, prob.t, W[idx], prob.basis, prob.degree)
    ok = within(f64[idx], ref, prob.t)
    assert ok.all(), np.max(np.abs(f64[idx] - ref) / ref)
    assert np.array_equal(f32, f64.astype(np.float32))


@pytest.mark.parametrize("shape", [(3001, 20, 4, 130), (300, 33, 10, 70), (8000, 33, 10, 1100)],
                         ids=lambda s: "x".join(map(str, s)))
def test_trig_table_gives_the_kernels_own_bits(gg, shape):
    """A float32 trig run seeds the recurrence from the (cos x, sin x) table
    computed once at game_create; the same chromosomes evaluated on a copy
    of the patterns (another address, so no table) seed it with sincosf in
    every tile.  The float64 errors are bit-identical, and the batched form
    (sincosf in its kernel) gives them too."""
    NP, N, d, P = shape
    X, t, W = problem(NP, N, d, P, 3, seed=NP + N)
    cfg = gg.config(basis=3, degree=d, population=P, tournament_k=3, elitism=1)
    Xd, td = torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()
    g = gg.Game(cfg, Xd, td)
    Wd = torch.from_numpy(W).cuda()
    _, f_table = g.fitness(Wd, with64=True)
    f_copy = g.evaluate(Xd.clone(), td, Wd)
    torch.cuda.synchronize()
    a, b = f_table.cpu().numpy(), f_copy.cpu().numpy()
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    assert within(a, og.fitness(X, t, W, 3, d), t).all()
    g.close()
    batch = gg.Batch([(Xd, td)], [cfg])
    gg.game_batch_tune(batch.h, 2, 64)
    batch.init()
    pop, _ = batch.population(0)
    g2 = gg.Game(cfg, Xd, td)
    _, f_pop = g2.fitness(pop.contiguous(), with64=True)
    batch.evaluate()
    _, f_batch = batch.population(0)
    torch.cuda.synchronize()
    assert np.array_equal(f_batch.cpu().numpy().view(np.uint32),
                          f_pop.cpu().numpy().astype(np.float32).view(np.uint32))
    g2.close()
    batch.close()
