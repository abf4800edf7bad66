"""Work decomposition of the batched form by shape bucket, and its committed
table.

    python -m paper_1304_0597_amd.batch_tuning      (needs the GPU)

runs the library's bucketed autotuner (game_batch_autotune_buckets) on the
batched workload (256 runs drawn from seed 3) and writes batch_tuning.json
beside this file.  Runs are bucketed by their number of expansion terms
K - 1 = B*N*d, which sets how much gene staging and epilogue work an item
carries per MFMA: a run's patterns are cut into items of the table's
tiles_per_item for its bucket (game_batch_tune_runs).  bench.py applies the
table instead of tuning while it measures.
"""
from __future__ import annotations

import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE_PATH = os.path.join(HERE, "batch_tuning.json")
BUCKET_BOUNDS = (32, 64, 128, 256)   # upper bounds of K - 1 per bucket; the last is open
N_BUCKETS = len(BUCKET_BOUNDS) + 1
WORKLOAD = "batched: 256 runs from seed 3"


def bucket_of(n_genes: int) -> int:
    """Bucket of a run with n_genes = K genes (K - 1 expansion terms)."""
    terms = n_genes - 1
    for i, bound in enumerate(BUCKET_BOUNDS):
        if terms <= bound:
            return i
    return len(BUCKET_BOUNDS)


def load(path: str = TABLE_PATH):
    """The committed table, or None if there is none."""
    try:
        with open(path) as f:
            return json.load(f)
    except OSError:
        return None


def tiles_for(table: dict, n_genes_of_runs) -> list:
    """tiles_per_item of every run under `table`."""
    return [table["tiles_per_bucket"][bucket_of(k)] for k in n_genes_of_runs]


def batched_workload(device="cuda:0"):
    """(problems, cfgs, shapes) of the batched workload on the GPU."""
    import torch

    from . import datagen
    from . import game as gg
    shapes = datagen.batched_shapes()
    problems, cfgs = [], []
    for i, sh in enumerate(shapes):
        prob = datagen.batched_problem(sh, i, with_validation=False)
        problems.append((torch.from_numpy(prob.X).to(device), torch.from_numpy(prob.t).to(device)))
        cfgs.append(gg.config(basis=sh.basis, degree=sh.degree, population=sh.population,
                              seed=i, max_generations=1 << 30, target=-1.0))
    return problems, cfgs, shapes


def main() -> None:
    from . import game as gg
    gg.lib()
    problems, cfgs, _ = batched_workload()
    batch = gg.Batch(problems, cfgs)
    batch.init()
    uniform = batch.autotune(reps=3)
    buckets = [bucket_of(k) for k in batch.n_genes]
    tuned = batch.autotune_buckets(buckets, N_BUCKETS, reps=3)
    batch.close()
    table = {"workload": WORKLOAD,
             "bucket_upper_bounds_of_terms": list(BUCKET_BOUNDS),
             "runs_per_bucket": [buckets.count(i) for i in range(N_BUCKETS)],
             "tiles_per_bucket": tuned["tiles_per_bucket"],
             "grid": tuned["grid"],
             "tuned_ms": round(tuned["ms"], 3),
             "uniform_best": {"tiles_per_item": uniform["tiles_per_item"],
                              "grid": uniform["grid"], "ms": round(uniform["ms"], 3)}}
    with open(TABLE_PATH, "w") as f:
        json.dump(table, f, indent=1)
        f.write("\n")
    print(json.dumps(table), flush=True)


if __name__ == "__main__":
    main()
