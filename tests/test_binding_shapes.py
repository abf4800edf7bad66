"""The Python binding checks every tensor's shape against the sizes of its
handle before anything reaches the library, so a mismatched tensor raises
ValueError rather than letting a kernel read or write past an allocation
(host logic, no GPU needed: the handles below are registered sizes only and
the library is never called with them)."""
import pytest

from paper_1304_0597_amd import game

torch = pytest.importorskip("torch")

FAKE, FAKE_BATCH, FAKE_SUR = 0x7E57_0001, 0x7E57_0002, 0x7E57_0003


@pytest.fixture(autouse=True)
def fake_handles():
    game._handles[FAKE] = {"n_patterns": 100, "n_features": 7, "n_genes": 29, "population": 50}
    game._handles[FAKE_BATCH] = {"runs": [{"population": 40, "n_genes": 13}]}
    game._handles[FAKE_SUR] = {"n_genes": 29, "max_batch": 64, "minibatch": 32, "n_params": 999}
    yield
    for h in (FAKE, FAKE_BATCH, FAKE_SUR):
        game._handles.pop(h, None)


def f32(*shape):
    return torch.zeros(shape, dtype=torch.float32)


def shape_error(fn, *args):
    with pytest.raises(ValueError) as ei:
        fn(*args)
    msg = str(ei.value)
    assert "expected shape" in msg or "rows" in msg or "elements" in msg or "run " in msg, msg


def test_create_checks_targets_against_patterns():
    cfg = game.config()
    shape_error(game.game_create, cfg, f32(100, 7), f32(99), f32(1))
    shape_error(game.game_create, cfg, f32(100, 7), f32(100, 1), f32(1))
    shape_error(game.game_create, cfg, f32(100), f32(100), f32(1))


def test_fitness_checks_genes_and_outputs():
    shape_error(game.game_fitness, FAKE, f32(50, 28), 50, f32(50))          # K
    shape_error(game.game_fitness, FAKE, f32(49, 29), 50, f32(50))          # rows < n
    shape_error(game.game_fitness, FAKE, f32(50, 29), 50, f32(49))          # outputs
    shape_error(game.game_fitness, FAKE, f32(50, 29), 50, f32(50),
                torch.zeros(10, dtype=torch.float64))
    with pytest.raises(ValueError, match="GPU tensor"):                    # shapes fine
        game.game_fitness(FAKE, f32(50, 29), 50, f32(50))


def test_other_data_sets_need_the_handles_feature_count():
    shape_error(game.game_evaluate, FAKE, f32(30, 6), f32(30), f32(5, 29), 5,
                torch.zeros(5, dtype=torch.float64))
    shape_error(game.game_evaluate, FAKE, f32(30, 7), f32(31), f32(5, 29), 5,
                torch.zeros(5, dtype=torch.float64))
    shape_error(game.game_rescore64, FAKE, f32(30, 8), f32(30), f32(5, 29), 5,
                torch.zeros(5, dtype=torch.float64))
    shape_error(game.game_classify, FAKE, f32(30, 7), f32(30), f32(5, 29), 5, 0.5,
                torch.zeros((5, 3), dtype=torch.int64))


def test_predict_output_is_chromosomes_by_patterns():
    shape_error(game.game_predict, FAKE, None, f32(2, 29), 2, f32(2, 99))    # own set: 100
    shape_error(game.game_predict, FAKE, None, f32(2, 29), 2, f32(1, 100))   # rows < n
    shape_error(game.game_predict, FAKE, f32(30, 7), f32(2, 29), 2, f32(2, 100))
    shape_error(game.game_predict, FAKE, f32(30, 5), f32(2, 29), 2, f32(2, 30))


def test_population_copies_need_the_full_population():
    shape_error(game.game_set_population, FAKE, f32(49, 29), 0)
    shape_error(game.game_set_population, FAKE, f32(50 * 29), 0)
    shape_error(game.game_get_population, FAKE, f32(50, 29), f32(49))
    with pytest.raises(ValueError, match="n_genes"):
        game.game_run(FAKE, 28)


def test_stateless_calls_check_against_the_configuration():
    cfg = game.config(population=50)
    shape_error(game.game_ga_next, cfg, 29, f32(50, 29), f32(49), 1, f32(50, 29), f32(1))
    shape_error(game.game_ga_next, cfg, 29, f32(50, 29), f32(50), 1, f32(50, 30), f32(1))
    shape_error(game.game_init_genes, cfg, 29, f32(51, 29))
    shape_error(game.game_rank, f32(10), 11, torch.zeros(11, dtype=torch.int32))
    shape_error(game.game_trig_sums, f32(10, 3), 4, f32(10, 7))


def test_batch_and_surrogate_calls():
    shape_error(game.game_batch_get_population, FAKE_BATCH, 0, f32(40, 12))
    shape_error(game.game_batch_get_population, FAKE_BATCH, 1, f32(40, 13))
    with pytest.raises(ValueError, match="n_runs"):
        game.game_batch_run(FAKE_BATCH, 2)
    shape_error(game._descs, [(f32(10, 3), f32(9))], [game.config()])
    shape_error(game.game_surrogate_predict, FAKE_SUR, f32(8, 28), 8, f32(8))
    shape_error(game.game_surrogate_predict, FAKE_SUR, f32(8, 29), 8, f32(7))
    shape_error(game.game_surrogate_gradients, FAKE_SUR, f32(8, 29), f32(8), 8, f32(998))
    shape_error(game.game_surrogate_set_params, FAKE_SUR, f32(10))
    shape_error(game.game_surrogate_train_step, FAKE_SUR, f32(8, 29), f32(7), 8)


def test_unknown_handles_are_rejected():
    with pytest.raises(ValueError, match="unknown handle"):
        game.game_fitness(0x7E57_00FF, f32(50, 29), 50, f32(50))
