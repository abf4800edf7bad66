"""The paper's own shared-gene polytrigo model (Eq. 9): the per-pattern
cos/sin sums computed once on the device, and the training loop run as the
degree-1 power model over those sums, against the float64 oracle.

Tolerances.  The sums are evaluated in float64 and rounded to float32 once,
so each is within half an ulp of the exact value: 2^-24 |Z| plus float64
noise (N d 1e-15).  The fitness then carries the float32 rounding of Z into
Out: per pattern |dOut_k| <= delta_k = 2^-24 sum_c |g_c Z_kc|, so a squared
residual moves by at most 2 |r_k| delta_k + delta_k^2, and its mean over the
patterns is added to the float32 fitness tolerance (1e-5 relative plus the
absolute floor).  A TMSE residual within delta_k plus float32 rounding of R
may fall on either side, and its whole contribution is allowed.
"""
import numpy as np
import pytest

from oracle import ga as oga
from oracle import game as og

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gg():
    from paper_1304_0597_amd import game
    game.lib()
    return game


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)


@pytest.mark.parametrize("d", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("NP,N", [(1, 1), (257, 11), (2100, 11), (1000, 3)])
def test_trig_sums_match_oracle(gg, d, NP, N):
    X = np.random.default_rng(NP + N + d).uniform(-3, 3, (NP, N)).astype(np.float32)
    Z = gg.game_trig_sums(torch.from_numpy(X).cuda(), d)
    torch.cuda.synchronize()
    Z = Z.cpu().numpy()
    ref = og.shared_trig_sums(X, d)
    assert Z.shape == (NP, 2 * d)
    assert np.all(np.abs(Z - ref) <= 2.0 ** -24 * np.abs(ref) + N * d * 1e-15)


def test_trig_sums_rejects_bad_degree(gg):
    X = torch.zeros((4, 2), device="cuda")
    for d in (0, 17):
        with pytest.raises(gg.GameError):
            gg.game_trig_sums(X, d, torch.empty((4, 34), device="cuda"))


def _shared_game(gg, X, t, d, P=23, error_fn=2, R=0.49, seed=0, max_gen=4000):
    Xd = torch.from_numpy(X).cuda()
    Z = gg.game_trig_sums(Xd, d)
    c = gg.config(basis=2, degree=1, population=P, tournament_k=4, elitism=2, p_crossover=0.9,
                  p_mutation=0.2, sigma_mutation=0.1, error_fn=error_fn, tmse_R=R, seed=seed,
                  max_generations=max_gen, target=0.0)
    return gg.Game(c, Z, torch.from_numpy(t).cuda()), Z


def _fit_bound(X, t, G, d, error_fn, R):
    """Oracle fitness of the shared-gene chromosomes G and the part of the
    tolerance that the float32 rounding of the sums adds (see the module
    docstring)."""
    ref = og.shared_trig_fitness(X, t, G, d, error_fn, R)
    G64 = np.atleast_2d(np.asarray(G, np.float64))
    Z = og.shared_trig_sums(X, d)
    delta = 2.0 ** -24 * (np.abs(Z) @ np.abs(G64[:, 1:]).T)            # [NP, P]
    r = t.astype(np.float64)[:, None] - og.shared_trig_outputs(X, G64, d)
    budget = (2 * np.abs(r) * delta + delta * delta).mean(axis=0)
    if error_fn == 2:
        near = np.abs(np.abs(r) - R) <= delta + 1e-5 * np.maximum(1.0, np.abs(r))
        budget = budget + (near * r * r).sum(axis=0) / X.shape[0]
    return ref, budget


@pytest.mark.parametrize("d", [1, 2, 4, 8])
@pytest.mark.parametrize("error_fn", [0, 2])
def test_shared_fitness_matches_oracle(gg, d, error_fn):
    rng = np.random.default_rng(d)
    X = rng.uniform(-1, 1, (2100, 11)).astype(np.float32)
    t = (rng.random(2100) < 0.5).astype(np.float32)
    g, Z = _shared_game(gg, X, t, d, error_fn=error_fn)
    assert g.n_genes == 2 * d + 1
    G = rng.uniform(-1, 1, (23, 2 * d + 1)).astype(np.float32) * 0.1
    f32, f64 = g.fitness(torch.from_numpy(G).cuda(), with64=True)
    ref, budget = _fit_bound(X, t, G, d, error_fn, 0.49)
    floor = 1e-7 * float(np.mean(t.astype(np.float64) ** 2))
    assert np.all(np.abs(f64.cpu().numpy() - ref) <= 1e-5 * ref + floor + budget)
    g.close()


def test_paper_shaped_run_follows_oracle(gg):
    """2,100 x 11, polytrigo d = 4 shared genes (9 per chromosome), 23
    chromosomes (2N + 1), tournament 4, crossover 0.9, mutation 0.2,
    elitism 2, TMSE R = 0.49: each generation is the oracle's genetic step
    of the device fitness, and that fitness is the oracle's."""
    rng = np.random.default_rng(11)
    X = rng.uniform(-1, 1, (2100, 11)).astype(np.float32)
    t = (rng.random(2100) < 0.5).astype(np.float32)
    d = 4
    g, Z = _shared_game(gg, X, t, d)
    c = g.cfg
    ocfg = oga.GAConfig(population=23, tournament_k=4, elitism=2, elite_mode=c.elite_mode,
                        p_crossover=0.9, p_mutation=0.2, sigma_mutation=0.1, seed=0,
                        init_mode=c.init_mode)
    g.init_population()
    for gen in range(10):
        pop, _ = g.population()
        g.step()
        nxt, fit = g.population()
        pop, nxt, fit = pop.cpu().numpy(), nxt.cpu().numpy(), fit.cpu().numpy()
        ref, budget = _fit_bound(X, t, pop, d, 2, 0.49)
        floor = 1e-7 * float(np.mean(t.astype(np.float64) ** 2))
        assert np.all(np.abs(fit - ref) <= 1e-5 * ref + floor + budget), gen
        assert np.array_equal(bits(nxt), bits(oga.ga_next(pop, fit, gen + 1, ocfg))), gen
    # the whole 4,000-generation training as one graph-captured run
    gens, best, err = g.run()
    assert gens == 4000
    ref, budget = _fit_bound(X, t, best[None, :], d, 2, 0.49)
    assert abs(err - ref[0]) <= 1e-5 * ref[0] + 1e-7 * float(np.mean(t.astype(np.float64) ** 2)) \
        + budget[0], (err, ref[0], budget[0])
    g.close()
