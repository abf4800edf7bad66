"""Pins of the oracle's random-number generator and genetic operators."""
import os

import numpy as np
import pytest
from scipy import stats

from oracle import game
from oracle import ga
from oracle.philox import block, mulhilo64, philox4x64_10
from paper_1304_0597_amd import datagen


# ---------------------------------------------------------------- Philox
def test_philox_known_answers(golden_dir):
    with open(os.path.join(golden_dir, "philox4x64_10_kat.txt")) as fh:
        rows = [l.split() for l in fh if l.strip() and not l.startswith("#")]
    assert len(rows) >= 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = philox4x64_10(np.array(v[0:4], dtype=np.uint64), np.array(v[4:6], dtype=np.uint64))
        assert [int(x) for x in out] == v[6:10]


def test_philox_matches_numpy_bit_generator():
    """numpy.random.Philox advances its counter before producing a block, so
    its first four outputs are the block of counter + 1."""
    rng = np.random.default_rng(11)
    for _ in range(20):
        ctr = [int(x) for x in rng.integers(0, 2 ** 63, 4, dtype=np.int64)]
        key = [int(x) for x in rng.integers(0, 2 ** 63, 2, dtype=np.int64)]
        bg = np.random.Philox(counter=ctr, key=key)
        ref = bg.random_raw(8)
        c1 = list(ctr)
        c1[0] += 1
        c2 = list(ctr)
        c2[0] += 2
        mine = np.concatenate([philox4x64_10(np.array(c1, np.uint64), np.array(key, np.uint64)),
                               philox4x64_10(np.array(c2, np.uint64), np.array(key, np.uint64))])
        assert [int(x) for x in mine] == [int(x) for x in ref]


def test_mulhilo_against_python_integers():
    rng = np.random.default_rng(12)
    a = rng.integers(0, 2 ** 63, 1000, dtype=np.int64).astype(np.uint64) * np.uint64(2) + np.uint64(1)
    b = rng.integers(0, 2 ** 63, 1000, dtype=np.int64).astype(np.uint64) * np.uint64(2)
    hi, lo = mulhilo64(a, b)
    for x, y, h, l in zip(a, b, hi, lo):
        p = int(x) * int(y)
        assert int(h) == p >> 64 and int(l) == p & (2 ** 64 - 1)


# ------------------------------------------------------------- draw helpers
def test_gauss12_is_exact_and_unit_variance():
    b = block(5, 2, 1, np.arange(20000, dtype=np.uint64), 0)
    z = ga.gauss12(b)
    scaled = z.astype(np.float64) * 65536.0
    assert np.all(scaled == np.round(scaled))           # exact in float32
    assert np.all(np.abs(z) <= 6.0)
    assert abs(z.mean()) < 0.03 and abs(z.var() - 1.0) < 0.03
    assert stats.kstest(z, "norm").pvalue > 1e-4


def test_coin_and_index_draws():
    assert ga.coin_threshold(1.0) == 2 ** 32
    assert ga.coin_threshold(0.0) == 0
    w = ga.words(block(1, 1, 1, np.arange(5000, dtype=np.uint64), 0)).ravel()
    assert np.all(w < np.uint64(ga.coin_threshold(1.0)))
    frac = np.mean(w < np.uint64(ga.coin_threshold(0.3)))
    assert abs(frac - 0.3) < 0.01
    idx = ga.index_draw(w, 7).astype(np.int64)
    assert idx.min() == 0 and idx.max() == 6
    assert stats.chisquare(np.bincount(idx, minlength=7)).pvalue > 1e-4


@pytest.mark.parametrize("mode", [ga.INIT_NORMAL, ga.INIT_UNIFORM, ga.INIT_UNIT])
def test_init_modes(mode):
    pop = ga.init_population(200, 50, seed=3, mode=mode)
    assert pop.dtype == np.float32 and pop.shape == (200, 50)
    if mode == ga.INIT_NORMAL:
        assert pop.min() >= -1 and pop.max() <= 1
        assert abs(pop.mean()) < 0.02 and abs(pop.std() - 1 / 3) < 0.02
    elif mode == ga.INIT_UNIFORM:
        assert pop.min() >= -1 and pop.max() < 1
        assert np.all(pop.astype(np.float64) * 2 ** 23 == np.round(pop.astype(np.float64) * 2 ** 23))
        assert abs(pop.var() - 1 / 3) < 0.02
    else:
        assert pop.min() >= 0 and pop.max() < 1 and abs(pop.mean() - 0.5) < 0.02
    # deterministic and keyed by the seed
    assert np.array_equal(pop, ga.init_population(200, 50, seed=3, mode=mode))
    assert not np.array_equal(pop, ga.init_population(200, 50, seed=4, mode=mode))


# ------------------------------------------------------------------ ranking
def test_rank_order_nan_last_and_ties_by_index():
    f = np.array([0.5, np.nan, 0.1, 0.5, -0.0, 0.0, np.inf, 0.1], dtype=np.float32)
    order = ga.rank_order(f)
    key = [(np.inf if np.isnan(v) else float(v) + 0.0, i) for i, v in enumerate(f)]
    assert list(order) == [i for _, i in sorted(key)]


# ---------------------------------------------------------------- operators
def _pop_fit(P=40, K=13, seed=0):
    rng = np.random.default_rng(seed)
    pop = rng.uniform(-1, 1, (P, K)).astype(np.float32)
    fit = rng.uniform(0, 2, P).astype(np.float32)
    return pop, fit


@pytest.mark.parametrize("mode", [0, 1])
def test_elitism(mode):
    pop, fit = _pop_fit()
    cfg = ga.GAConfig(population=40, elitism=3, elite_mode=mode, seed=1)
    nxt = ga.ga_next(pop, fit, 1, cfg)
    order = np.argsort(fit, kind="stable")
    for e in range(3):
        src = order[0] if mode == 0 else order[e]
        assert np.array_equal(nxt[e], pop[src])


def test_no_crossover_no_mutation_copies_tournament_winners():
    """p_c = p_m = 0: every child is a copy of a population row, and with a
    tournament as large as the population almost every copy is the best."""
    pop, fit = _pop_fit()
    cfg = ga.GAConfig(population=40, tournament_k=40, elitism=2, p_crossover=0.0,
                      p_mutation=0.0, seed=2)
    nxt = ga.ga_next(pop, fit, 1, cfg)
    rows = {pop[i].tobytes(): i for i in range(40)}
    src = [rows[r.tobytes()] for r in nxt[2:]]
    best = int(np.argmin(fit))
    assert np.mean(np.array(src) == best) > 0.5


def test_crossover_children_are_complementary_one_cut():
    pop, fit = _pop_fit(P=41, K=17)
    cfg = ga.GAConfig(population=41, tournament_k=3, elitism=1, p_crossover=1.0,
                      p_mutation=0.0, seed=3)
    nxt = ga.ga_next(pop, fit, 5, cfg)
    p1, p2, cross, cut = ga.select_pairs(fit, 41, 17, 5, cfg)
    assert np.all(cross) and cut.min() >= 1 and cut.max() <= 16
    for q in range(p1.size):
        a = nxt[1 + 2 * q]
        assert np.array_equal(a[:cut[q]], pop[p1[q]][:cut[q]])
        assert np.array_equal(a[cut[q]:], pop[p2[q]][cut[q]:])
        if 2 + 2 * q < 41:
            b = nxt[2 + 2 * q]
            assert np.array_equal(np.sort(np.stack([a, b]), 0),
                                  np.sort(np.stack([pop[p1[q]], pop[p2[q]]]), 0))


def test_cut_points_uniform():
    fit = np.zeros(2000, np.float32)
    cfg = ga.GAConfig(population=2000, elitism=0, p_crossover=1.0, seed=4)
    _, _, _, cut = ga.select_pairs(fit, 2000, 9, 1, cfg)
    counts = np.bincount(cut, minlength=9)[1:]
    assert counts.size == 8 and stats.chisquare(counts).pvalue > 1e-4


def test_k1_tournament_draws_parents_uniformly():
    fit = np.random.default_rng(0).uniform(size=16).astype(np.float32)
    cfg = ga.GAConfig(population=16, tournament_k=1, elitism=0, seed=5)
    cnt = np.zeros(16)
    for g in range(1, 40):
        p1, p2, _, _ = ga.select_pairs(fit, 16, 5, g, cfg)
        cnt += np.bincount(np.concatenate([p1, p2]), minlength=16)
    assert stats.chisquare(cnt).pvalue > 1e-4


def test_mutation_rate_range_and_zero_sigma():
    pop = np.zeros((500, 40), np.float32) + np.float32(0.95)
    fit = np.zeros(500, np.float32)
    cfg = ga.GAConfig(population=500, elitism=0, p_crossover=0.0, p_mutation=0.2,
                      sigma_mutation=0.5, seed=6)
    nxt = ga.ga_next(pop, fit, 1, cfg)
    changed = nxt != pop
    assert abs(changed.mean() - 0.2) < 0.01
    assert nxt.min() >= -1 and nxt.max() <= 1
    assert np.any(nxt == 1.0)                       # the clamp is reached
    cfg0 = ga.GAConfig(population=500, elitism=0, p_crossover=0.0, p_mutation=1.0,
                       sigma_mutation=0.0, seed=6)
    assert np.array_equal(ga.ga_next(pop, fit, 1, cfg0), pop)


def test_odd_offspring_count_drops_last_child():
    pop, fit = _pop_fit(P=10)
    cfg = ga.GAConfig(population=10, elitism=3, seed=7)
    nxt = ga.ga_next(pop, fit, 1, cfg)
    assert nxt.shape == (10, pop.shape[1])


def test_nan_fitness_is_never_elite():
    pop, fit = _pop_fit()
    fit[:] = np.nan
    fit[17] = 3.0
    cfg = ga.GAConfig(population=40, elitism=2, seed=8)
    nxt = ga.ga_next(pop, fit, 1, cfg)
    assert np.array_equal(nxt[0], pop[17]) and np.array_equal(nxt[1], pop[17])


def test_run_best_fitness_non_increasing_and_stop_rules():
    prob = datagen.small()
    X, t = prob.X[:500], prob.t[:500]
    cfg = ga.GAConfig(population=30, seed=0)
    res = ga.run(X, t, prob.basis, prob.degree, cfg, max_generations=15, target=0.0)
    h = np.array(res["history"])
    assert res["generations"] == 15 and h.size == 16
    assert np.all(np.diff(h) <= 1e-7 * h[:-1])       # elitism keeps the best
    assert h[-1] < h[0]
    # the error threshold stops at generation 0 when it is already met
    res0 = ga.run(X, t, prob.basis, prob.degree, cfg, max_generations=15, target=1e9)
    assert res0["generations"] == 0
    assert np.all(np.abs(res["population"]) <= 1)


# ------------------------------------------------------- ranking / roulette
def test_ranking_probabilities_are_linear():
    """Rank r of P is drawn with probability (P - r) / (P (P + 1) / 2)."""
    P = 8
    fit = np.random.default_rng(0).permutation(P).astype(np.float32)   # rank of i = fit[i]
    u = ga.words(block(1, 1, 1, np.arange(40000, dtype=np.uint64), 0)).ravel()
    picks = ga.ranking_pick(fit, u)
    ranks = fit[picks].astype(np.int64)
    counts = np.bincount(ranks, minlength=P)
    expected = (P - np.arange(P)) / (P * (P + 1) / 2) * u.size
    assert stats.chisquare(counts, expected).pvalue > 1e-4


def test_ranking_exact_boundaries():
    """The integer cumulative weights put draw t = 0 on rank 0 and the
    largest draw on rank P - 1."""
    fit = np.array([0.3, 0.1, 0.2], np.float32)       # order: 1, 2, 0
    assert ga.ranking_pick(fit, np.array([0], np.uint64))[0] == 1
    assert ga.ranking_pick(fit, np.array([2 ** 32 - 1], np.uint64))[0] == 0
    # W = 6: ranks own [0,3), [3,5), [5,6); t = (u * 6) >> 32
    u_for = lambda t: np.array([int(np.ceil(t * 2 ** 32 / 6))], np.uint64)
    assert ga.ranking_pick(fit, u_for(3))[0] == 2 and ga.ranking_pick(fit, u_for(5))[0] == 0


def test_roulette_probabilities_follow_inverse_error():
    fit = np.array([1.0, 0.5, 0.25, np.inf, np.nan], np.float32)
    cum = ga.roulette_cumulative(fit)
    assert cum[-1] == cum[2]                           # inf and NaN weigh 0
    u = ga.words(block(2, 1, 1, np.arange(40000, dtype=np.uint64), 0)).ravel()
    picks = ga.roulette_pick(cum, u)
    counts = np.bincount(picks, minlength=5)
    assert counts[3] == 0 and counts[4] == 0
    w = 1.0 / (np.array([1.0, 0.5, 0.25]) + 1e-12)
    assert stats.chisquare(counts[:3], w / w.sum() * u.size).pvalue > 1e-4


def test_roulette_all_infinite_falls_back_to_uniform():
    fit = np.full(6, np.inf, np.float32)
    cum = ga.roulette_cumulative(fit)
    u = ga.words(block(3, 1, 1, np.arange(6000, dtype=np.uint64), 0)).ravel()
    picks = ga.roulette_pick(cum, u)
    assert picks.min() == 0 and picks.max() == 5
    assert stats.chisquare(np.bincount(picks, minlength=6)).pvalue > 1e-4


@pytest.mark.parametrize("sel", [ga.SELECT_RANKING, ga.SELECT_ROULETTE])
def test_selection_modes_run_and_keep_the_elite(sel):
    prob = datagen.small()
    X, t = prob.X[:400], prob.t[:400]
    cfg = ga.GAConfig(population=30, seed=0, selection=sel)
    res = ga.run(X, t, prob.basis, prob.degree, cfg, max_generations=12, target=0.0)
    h = np.array(res["history"])
    assert np.all(np.diff(h) <= 1e-7 * h[:-1]) and h[-1] < h[0]
