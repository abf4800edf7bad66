"""The C-ABI library loads, exports every function include/game.h declares,
lays out game_config as C does, and validates configurations (host logic,
no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1304_0597_amd import game

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "game.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(game_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_abi():
    names = declared_functions()
    for n in ["game_create", "game_fitness", "game_step", "game_run", "game_destroy",
              "game_ga_next", "game_rank", "game_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    L = game.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert set(declared_functions()) <= set(game._SIGS), "binding lacks a signature"


def test_config_struct_layout_matches_c(tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "game.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu\", sizeof(game_config),"
        " offsetof(game_config, p_crossover), offsetof(game_config, seed),"
        " offsetof(game_config, max_generations), offsetof(game_config, target),"
        " offsetof(game_config, selection));return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    g = game.game_config
    assert got == [ctypes.sizeof(g), g.p_crossover.offset, g.seed.offset,
                   g.max_generations.offset, g.target.offset, g.selection.offset]


def test_defaults_and_gene_counts():
    c = game.config()
    assert (c.basis, c.degree, c.population, c.tournament_k, c.elitism) == (0, 4, 50, 3, 2)
    assert abs(c.p_crossover - 0.9) < 1e-7 and abs(c.target - 1e-3) < 1e-15
    assert game.game_num_genes(c, 7) == 29
    assert game.game_num_genes(game.config(basis=game.GAME_LEGENDRE, degree=8), 20) == 161
    assert game.game_num_genes(game.config(basis=game.GAME_TRIG, degree=8), 11) == 177


@pytest.mark.parametrize("field,value", [
    ("basis", 4), ("degree", 0), ("degree", 17), ("population", 1), ("population", 8193),
    ("tournament_k", 0), ("tournament_k", 51), ("elitism", 50), ("elite_mode", 2),
    ("init_mode", 3), ("error_fn", 4), ("p_crossover", 1.5), ("p_mutation", -0.1),
    ("sigma_mutation", -1.0), ("max_generations", -1), ("selection", 3), ("selection", -1),
])
def test_invalid_configs_are_rejected(field, value):
    c = game.config()
    setattr(c, field, value)
    with pytest.raises(game.GameError) as ei:
        game.game_num_genes(c, 7)
    assert ei.value.code == game.GAME_EINVAL
    assert game.game_last_error()
    assert game.lib().game_workspace_size(ctypes.byref(c), 100, 7) == 0


def _documented_range(field):
    """The 'lo..hi' range the header's comment gives for a game_config field."""
    src = open(HEADER).read()
    m = re.search(r"int32_t\s+" + field + r";\s*/\*\s*(\S+)\.\.(\S+)", src)
    assert m, field
    return m.group(1), m.group(2)


def test_documented_ranges_are_the_enforced_ones():
    """tournament_k, elitism and population: the header's range is what the
    library accepts, at both ends."""
    assert _documented_range("tournament_k") == ("1", "population")
    for P in (2, 50, 8192):
        game.game_num_genes(game.config(population=P, tournament_k=P, elitism=1), 3)
        game.game_num_genes(game.config(population=P, tournament_k=1, elitism=1), 3)
        for k in (0, P + 1):
            with pytest.raises(game.GameError):
                game.game_num_genes(game.config(population=P, tournament_k=k, elitism=1), 3)
    assert _documented_range("elitism") == ("0", "population-1")
    game.game_num_genes(game.config(population=50, elitism=49), 3)
    game.game_num_genes(game.config(population=50, elitism=0), 3)
    with pytest.raises(game.GameError):
        game.game_num_genes(game.config(population=50, elitism=50), 3)
    assert re.search(r"int32_t\s+population;\s*/\*\s*P, 2\.\.8192", open(HEADER).read())
    game.game_num_genes(game.config(population=8192, tournament_k=3), 3)
    with pytest.raises(game.GameError):
        game.game_num_genes(game.config(population=8193, tournament_k=3), 3)


def test_tmse_threshold_range():
    c = game.config(error_fn=game.GAME_TMSE, tmse_R=0.0)
    with pytest.raises(game.GameError):
        game.game_num_genes(c, 3)
    c.tmse_R = 0.49
    assert game.game_num_genes(c, 3) == 13


def test_too_many_genes():
    c = game.config(degree=16)
    assert game.game_num_genes(c, 256) == 4097
    with pytest.raises(game.GameError):
        game.game_num_genes(c, 257)


def test_workspace_size_grows_with_population():
    a = game.game_workspace_size(game.config(population=64), 1000, 8)
    b = game.game_workspace_size(game.config(population=2048), 1000, 8)
    assert b > a > 0 and a % 256 == 0 and b % 256 == 0


def test_null_arguments_fail_without_gpu():
    L = game.lib()
    assert L.game_destroy(None) == game.GAME_EINVAL
    h = ctypes.c_void_p()
    c = game.config()
    rc = L.game_create(ctypes.byref(c), None, None, 10, 7, None, 0, None, ctypes.byref(h))
    assert rc == game.GAME_EINVAL and h.value is None
    assert L.game_config_default(None) == game.GAME_EINVAL


def test_run_desc_layout_matches_c(tmp_path):
    prog = tmp_path / "desc.c"
    prog.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "game.h"\n'
        "int main(void){printf(\"%zu %zu %zu\", sizeof(game_run_desc),"
        " offsetof(game_run_desc, n_patterns), offsetof(game_run_desc, cfg));return 0;}\n")
    exe = tmp_path / "desc"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)],
                   check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    d = game.game_run_desc
    assert got == [ctypes.sizeof(d), d.n_patterns.offset, d.cfg.offset]


def test_batch_rejects_invalid_runs_without_gpu():
    descs = (game.game_run_desc * 2)()
    for i in range(2):
        descs[i].n_patterns = 1000
        descs[i].n_features = 5
        descs[i].cfg = game.config()
    assert game.lib().game_batch_workspace_size(descs, 2) > 0
    descs[1].cfg.precision = game.GAME_BF16
    assert game.lib().game_batch_workspace_size(descs, 2) == 0
    assert "run 1" in game.game_last_error()
    descs[1].cfg.precision = game.GAME_FP32
    descs[1].cfg.degree = 0
    assert game.lib().game_batch_workspace_size(descs, 2) == 0
    assert game.lib().game_batch_workspace_size(descs, 0) == 0


@pytest.mark.parametrize("counts", [(10, 2, 30, 5), (0, 0, 5, 0), (3, 0, 0, 0), (0, 4, 0, 6),
                                    (0, 0, 0, 0)])
def test_merit_follows_the_oracle_definitions(counts):
    """game_merit (host arithmetic on the four counts) against the oracle's
    figures of merit of outputs and labels built to give those counts."""
    import numpy as np
    from oracle import game as og
    tp, fp, tn, fn = counts
    out = np.array([1.0] * tp + [1.0] * fp + [0.0] * tn + [0.0] * fn)
    t = np.array([1.0] * tp + [0.0] * fp + [0.0] * tn + [1.0] * fn)
    got = game.game_merit(counts)
    if sum(counts) == 0:
        assert all(np.isnan(v) for v in got.values())
        return
    ref = og.classification_merit(out, t)
    for k, v in ref.items():
        assert (np.isnan(v) and np.isnan(got[k])) or got[k] == pytest.approx(v, rel=1e-15), k


def test_predict_null_handle_fails_without_gpu():
    L = game.lib()
    assert L.game_predict(None, None, 0, None, 1, None) == game.GAME_EINVAL
    assert L.game_classify(None, None, None, 0, None, 1, ctypes.c_float(0.5), None) == game.GAME_EINVAL
    assert L.game_merit(None, None) == game.GAME_EINVAL


def test_autotune_candidate_count_matches_header():
    src = open(HEADER).read()
    n = int(re.search(r"#define\s+GAME_AUTOTUNE_CANDIDATES\s+(\d+)", src).group(1))
    assert n == len(game.AUTOTUNE_TILES) * len(game.AUTOTUNE_GRIDS)


def test_batch_shape_buckets():
    """Runs are bucketed by their expansion terms K - 1 (bounds 32, 64, 128,
    256, then open); the table maps each run to its bucket's value."""
    from paper_1304_0597_amd import batch_tuning as bt
    assert [bt.bucket_of(k) for k in (2, 33, 34, 65, 66, 129, 130, 257, 258, 4097)] == \
        [0, 0, 1, 1, 2, 2, 3, 3, 4, 4]
    table = {"tiles_per_bucket": [1, 2, 4, 8, 16]}
    assert bt.tiles_for(table, [9, 60, 100, 200, 641]) == [1, 2, 4, 8, 16]
    assert bt.N_BUCKETS == len(table["tiles_per_bucket"])
