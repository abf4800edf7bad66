"""Batched form: many independent runs in one persistent fitness launch per
generation.  Each run must follow its own trajectory: generation 0 equal to
the oracle's, every later generation equal to the oracle's genetic step
driven by the device fitness, fitness within the float32 tolerance of the
float64 oracle, and the same trajectory as the run alone."""
import numpy as np
import pytest

from oracle import ga as oga
from oracle import game as og
from paper_1304_0597_amd import datagen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gg():
    from paper_1304_0597_amd import game
    game.lib()
    return game


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)


# NP, N, d, P, basis: uneven sizes, ragged tiles, every basis, K-chunking
RUNS = [(1000, 7, 4, 50, 0), (3001, 20, 8, 130, 1), (257, 5, 3, 33, 2), (700, 4, 6, 64, 3),
        (5000, 33, 10, 96, 0), (1500, 64, 2, 200, 2)]


def make_runs(gg, runs=RUNS, max_gen=6, seed0=11):
    problems, cfgs, host = [], [], []
    for i, (NP, N, d, P, basis) in enumerate(runs):
        rng = np.random.default_rng(seed0 + i)
        X = rng.uniform(-1, 1, (NP, N)).astype(np.float32)
        t = rng.normal(0, 1, NP).astype(np.float32)
        problems.append((torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()))
        cfgs.append(gg.config(basis=basis, degree=d, population=P, seed=100 + i,
                              tournament_k=3, elitism=2, elite_mode=i % 2,
                              p_mutation=0.05 + 0.05 * (i % 3), max_generations=max_gen,
                              target=0.0, selection=i % 3))
        host.append((X, t))
    return problems, cfgs, host


def oracle_cfg(c):
    return oga.GAConfig(population=c.population, tournament_k=c.tournament_k, elitism=c.elitism,
                        elite_mode=c.elite_mode, p_crossover=c.p_crossover,
                        p_mutation=c.p_mutation, sigma_mutation=c.sigma_mutation, seed=c.seed,
                        init_mode=c.init_mode, selection=c.selection)


def test_batch_generations_follow_oracle(gg):
    problems, cfgs, host = make_runs(gg)
    b = gg.Batch(problems, cfgs)
    b.init()
    for r, c in enumerate(cfgs):
        pop0, _ = b.population(r)
        ref = oga.init_population(c.population, b.n_genes[r], c.seed, c.init_mode)
        assert np.array_equal(bits(pop0.cpu().numpy()), bits(ref)), r
    for gen in range(3):
        before = [b.population(r)[0].cpu().numpy() for r in range(b.n_runs)]
        b.step()
        for r, c in enumerate(cfgs):
            after, fit = b.population(r)
            after, fit = after.cpu().numpy(), fit.cpu().numpy()
            X, t = host[r]
            ref_f = og.fitness(X, t, before[r], c.basis, c.degree)
            assert np.all(np.abs(fit - ref_f) <= 1e-5 * ref_f + 1e-7 * np.mean(t.astype(np.float64) ** 2)), r
            ref_next = oga.ga_next(before[r], fit, gen + 1, oracle_cfg(c))
            assert np.array_equal(bits(after), bits(ref_next)), (gen, r)
    b.close()


def test_batch_run_equals_single_runs(gg):
    problems, cfgs, _ = make_runs(gg, max_gen=7)
    b = gg.Batch(problems, cfgs)
    b.init()
    gens, best = b.run()
    assert np.all(gens == 7)
    for r, c in enumerate(cfgs):
        g = gg.Game(c, *problems[r])
        g.init_population()
        n, _, err = g.run()
        assert n == 7
        pb, fb = b.population(r)
        ps, fs = g.population()
        assert np.array_equal(bits(pb.cpu().numpy()), bits(ps.cpu().numpy())), r
        assert abs(best[r] - err) <= 1e-12 * err, r
        g.close()
    b.close()


def test_autotune_leaves_populations_and_picks_a_candidate(gg):
    problems, cfgs, _ = make_runs(gg)
    b = gg.Batch(problems, cfgs)
    b.init()
    b.step()
    before = [bits(b.population(r)[0].cpu().numpy()) for r in range(b.n_runs)]
    res = b.autotune(reps=2)
    assert res["tiles_per_item"] in gg.AUTOTUNE_TILES and res["grid"] in gg.AUTOTUNE_GRIDS
    assert len(res["times_ms"]) == len(gg.AUTOTUNE_TILES) * len(gg.AUTOTUNE_GRIDS)
    assert all(v > 0 for v in res["times_ms"].values())
    assert abs(res["ms"] - min(res["times_ms"].values())) < 1e-6
    after = [bits(b.population(r)[0].cpu().numpy()) for r in range(b.n_runs)]
    assert all(np.array_equal(x, y) for x, y in zip(before, after))
    n_items, tiles, grid = b.items()
    assert tiles == res["tiles_per_item"] and grid == res["grid"] and n_items > 0
    # the tuned decomposition continues the same trajectory as the default
    b.step()
    b2 = gg.Batch(problems, cfgs)
    b2.init()
    b2.step()
    b2.step()
    for r in range(b.n_runs):
        assert np.array_equal(bits(b.population(r)[0].cpu().numpy()),
                              bits(b2.population(r)[0].cpu().numpy()))
    b.close()
    b2.close()


# Edges of the two-tile waves: a run under one pattern tile, exactly two
# full tiles, three tiles (a wave's second tile missing in the last step),
# degree 1, a population over many chromosome tiles, chunked genes, and the
# smallest runs (one pattern and one feature; three patterns, trig).
EDGE_RUNS = [(100, 3, 5, 40, 0), (512, 6, 1, 64, 2), (768, 9, 4, 1000, 1), (60, 40, 9, 70, 3),
             (1900, 48, 10, 65, 1), (1, 1, 1, 4, 0), (3, 2, 2, 5, 3)]


@pytest.mark.parametrize("tiles,grid", [(None, None), (1, 256), (3, 512)],
                         ids=["default", "1-tile-items", "3-tile-items"])
def test_batch_edges_equal_single_runs(gg, tiles, grid):
    problems, cfgs, _ = make_runs(gg, runs=EDGE_RUNS, max_gen=4, seed0=31)
    b = gg.Batch(problems, cfgs)
    if tiles is not None:
        b.tune(tiles, grid)
    b.init()
    gens, best = b.run()
    assert np.all(gens == 4)
    for r, c in enumerate(cfgs):
        g = gg.Game(c, *problems[r])
        g.init_population()
        n, _, err = g.run()
        assert n == 4
        pb, fb = b.population(r)
        ps, fs = g.population()
        assert np.array_equal(bits(pb.cpu().numpy()), bits(ps.cpu().numpy())), r
        assert np.array_equal(bits(fb.cpu().numpy()), bits(fs.cpu().numpy())), r
        assert best[r] == err, r
        g.close()
    b.close()


@pytest.mark.parametrize("tiles,grid", [(1, 64), (32, 1024), (3, 7)])
def test_any_decomposition_gives_the_same_trajectory(gg, tiles, grid):
    problems, cfgs, _ = make_runs(gg, runs=RUNS[:4], max_gen=3)
    b1 = gg.Batch(problems, cfgs)
    b1.tune(tiles, grid)
    b1.init()
    g1, e1 = b1.run()
    b2 = gg.Batch(problems, cfgs)
    b2.init()
    g2, e2 = b2.run()
    assert np.array_equal(g1, g2)
    np.testing.assert_allclose(e1, e2, rtol=1e-12)
    for r in range(b1.n_runs):
        assert np.array_equal(bits(b1.population(r)[0].cpu().numpy()),
                              bits(b2.population(r)[0].cpu().numpy()))
    b1.close()
    b2.close()


def test_per_run_decomposition_and_bucketed_autotuner(gg):
    """Per-run items sizes (game_batch_tune_runs) and the bucketed autotuner
    keep every run on the trajectory of the default decomposition, bit for
    bit; the autotuner's choice is set and reported back."""
    from paper_1304_0597_amd import batch_tuning
    problems, cfgs, _ = make_runs(gg)
    ref = gg.Batch(problems, cfgs)
    ref.init()
    for _ in range(3):
        ref.step()
    b = gg.Batch(problems, cfgs)
    tiles = [1, 3, 8, 2, 16, 5]
    b.tune_runs(tiles, 300)
    got, grid = b.tuning()
    assert list(got) == tiles and grid == 300 and b.items()[1] == 0
    b.init()
    b.step()
    buckets = [batch_tuning.bucket_of(k) for k in b.n_genes]
    res = b.autotune_buckets(buckets, batch_tuning.N_BUCKETS, reps=1)
    got, grid = b.tuning()
    assert list(got) == [res["tiles_per_bucket"][k] for k in buckets]
    assert grid == res["grid"] and res["ms"] > 0
    assert all(t in gg.AUTOTUNE_TILES for t in res["tiles_per_bucket"])
    b.step()
    b.step()
    for r in range(b.n_runs):
        assert np.array_equal(bits(b.population(r)[0].cpu().numpy()),
                              bits(ref.population(r)[0].cpu().numpy()))
    with pytest.raises(ValueError):
        b.tune_runs(tiles[:-1], 300)
    with pytest.raises(gg.GameError):
        b.tune_runs([0] * len(tiles), 300)
    b.close()
    ref.close()


def test_batched_workload_sample(gg):
    """The first 12 runs of the 256-run batched workload recipe at full size;
    fitness of two runs checked against the oracle on sampled chromosomes."""
    shapes = datagen.batched_shapes()[:12]
    problems, cfgs, host = [], [], []
    for i, sh in enumerate(shapes):
        prob = datagen.batched_problem(sh, i, with_validation=False)
        problems.append((torch.from_numpy(prob.X).cuda(), torch.from_numpy(prob.t).cuda()))
        cfgs.append(gg.config(basis=sh.basis, degree=sh.degree, population=sh.population,
                              seed=i, max_generations=100, target=0.0))
        host.append(prob)
    b = gg.Batch(problems, cfgs)
    b.autotune(reps=1)
    b.init()
    before = [b.population(r)[0].cpu().numpy() for r in (0, 5)]
    b.step()
    for k, r in enumerate((0, 5)):
        _, fit = b.population(r)
        fit = fit.cpu().numpy()
        idx = np.array([0, 1, cfgs[r].population - 1])
        p = host[r]
        ref = og.fitness(p.X, p.t, before[k][idx], p.basis, p.degree)
        assert np.all(np.abs(fit[idx] - ref) <= 1e-5 * ref + 1e-7 * np.mean(p.t.astype(np.float64) ** 2))
    b.close()


def test_batch_error_functions_follow_single_runs(gg):
    """Runs with RMSE, TMSE (|r| > R) and the literal TMSE (r^2 > R) in one
    batch: each follows its single-run trajectory bit for bit."""
    runs = [(900, 6, 3, 40, 0), (1300, 9, 5, 70, 2), (700, 4, 8, 33, 1)]
    problems, cfgs = [], []
    for i, (NP, N, d, P, basis) in enumerate(runs):
        rng = np.random.default_rng(40 + i)
        X = rng.uniform(-1, 1, (NP, N)).astype(np.float32)
        t = (rng.random(NP) < 0.5).astype(np.float32)
        problems.append((torch.from_numpy(X).cuda(), torch.from_numpy(t).cuda()))
        cfgs.append(gg.config(basis=basis, degree=d, population=P, seed=7 + i, elitism=2,
                              error_fn=i + 1, tmse_R=0.49, max_generations=5, target=0.0))
    b = gg.Batch(problems, cfgs)
    b.init()
    gens, best = b.run()
    assert np.all(gens == 5)
    for r, c in enumerate(cfgs):
        g = gg.Game(c, *problems[r])
        g.init_population()
        n, _, err = g.run()
        assert n == 5
        pb, fb = b.population(r)
        ps, fs = g.population()
        assert np.array_equal(bits(pb.cpu().numpy()), bits(ps.cpu().numpy())), r
        assert abs(best[r] - err) <= 1e-12 * max(err, 1e-30), r
        g.close()
    b.close()


def test_batch_evaluate_is_the_steps_evaluation(gg):
    """game_batch_evaluate gives each run exactly the fitness the next
    generation's evaluation gives (same work list, same sums), and leaves
    the queues ready for that generation."""
    problems, cfgs, host = make_runs(gg)
    b = gg.Batch(problems, cfgs)
    b.init()
    b.step()
    b.evaluate()
    ev = [b.population(r)[1].cpu().numpy().copy() for r in range(b.n_runs)]
    pops = [b.population(r)[0].cpu().numpy().copy() for r in range(b.n_runs)]
    b.step()
    for r, c in enumerate(cfgs):
        fit = b.population(r)[1].cpu().numpy()
        assert np.array_equal(ev[r].view(np.uint32), fit.view(np.uint32)), r
        X, t = host[r]
        ref = og.fitness(X, t, pops[r], c.basis, c.degree)
        assert np.all(np.abs(ev[r] - ref) <= 1e-5 * ref + 1e-7 * np.mean(t.astype(np.float64) ** 2))
    b.close()
