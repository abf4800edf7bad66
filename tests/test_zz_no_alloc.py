"""game_ga_next_static, the genetic step whose scratch is a fixed array inside
the library (for callers that cannot allocate), gives bit for bit what
game_ga_next gives with a caller workspace, and what the oracle gives, on two
calls in a row with the second on a smaller population.  The first call is
the library's first use of its fixed scratch on the device."""
import numpy as np
import pytest

from oracle import ga as oga

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def gg():
    from paper_1304_0597_amd import game
    game.lib()
    return game


def bits(a):
    return np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)


def oracle_cfg(c):
    return oga.GAConfig(population=c.population, tournament_k=c.tournament_k, elitism=c.elitism,
                        elite_mode=c.elite_mode, p_crossover=c.p_crossover,
                        p_mutation=c.p_mutation, sigma_mutation=c.sigma_mutation, seed=c.seed,
                        init_mode=c.init_mode, selection=c.selection)


def _inputs(P, K, seed):
    rng = np.random.default_rng(seed)
    pop = rng.uniform(-1, 1, (P, K)).astype(np.float32)
    fit = rng.uniform(0, 1, P).astype(np.float32)
    fit[rng.choice(P, max(1, P // 10), replace=False)] = fit[0]          # ties
    fit[rng.choice(P, max(1, P // 20), replace=False)] = np.nan          # NaN
    return pop, fit


# (P, K, generation): the second call is smaller than the first, so stale
# rank order and roulette sums of the first call would show in it.
CALLS = [(8192, 33, 5), (4096, 257, 3), (50, 29, 1)]


@pytest.mark.parametrize("selection", [0, 1, 2], ids=["tournament", "ranking", "roulette"])
def test_static_scratch_matches_workspace_path(gg, selection):
    for i, (P, K, gen) in enumerate(CALLS):
        pop, fit = _inputs(P, K, 1000 * selection + i)
        c = gg.config(population=P, tournament_k=3, elitism=2, p_crossover=0.9,
                      p_mutation=0.2, sigma_mutation=0.1, seed=4242 + i, selection=selection)
        pop_d, fit_d = torch.from_numpy(pop).cuda(), torch.from_numpy(fit).cuda()
        out_static = torch.full((P, K), np.nan, dtype=torch.float32, device="cuda")
        gg.game_ga_next_static(c, K, pop_d, fit_d, gen, out_static)
        ws = torch.empty(gg.game_ga_workspace_size(c), dtype=torch.uint8, device="cuda")
        out_ws = torch.full((P, K), np.nan, dtype=torch.float32, device="cuda")
        gg.game_ga_next(c, K, pop_d, fit_d, gen, out_ws, ws)
        torch.cuda.synchronize()
        got = out_static.cpu().numpy()
        assert np.array_equal(bits(got), bits(out_ws.cpu().numpy())), (P, K)
        ref = oga.ga_next(pop, fit, gen, oracle_cfg(c))
        assert np.array_equal(bits(got), bits(ref)), (P, K)


def test_static_scratch_rejects_oversized_population(gg):
    P, K = 8193, 2
    c = gg.config(population=8192)
    c.population = P
    pop = torch.zeros((P, K), dtype=torch.float32, device="cuda")
    fit = torch.zeros(P, dtype=torch.float32, device="cuda")
    out = torch.empty((P, K), dtype=torch.float32, device="cuda")
    with pytest.raises(gg.GameError) as e:
        gg.game_ga_next_static(c, K, pop, fit, 1, out)
    assert e.value.code == gg.GAME_EINVAL
    assert "8192" in str(e.value)
