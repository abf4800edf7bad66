"""ctypes binding of libgame's C ABI (include/game.h).

Same names as the C functions; arguments are torch tensors on the GPU (device
memory and streams come from PyTorch) and are passed as raw pointers.  Every
step of the computation runs in the HIP library: this module only marshals
arguments, and it raises if ``libgame.so`` has not been built.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_float, c_int32, c_int64, c_size_t, c_uint64, c_void_p

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgame.so")

GAME_OK, GAME_EINVAL, GAME_EWORKSPACE, GAME_EHIP, GAME_ESTATE = 0, -1, -2, -3, -4
GAME_CHEBYSHEV, GAME_LEGENDRE, GAME_POWER, GAME_TRIG = 0, 1, 2, 3
GAME_MSE, GAME_RMSE, GAME_TMSE, GAME_TMSE_SQUARED = 0, 1, 2, 3
GAME_FP32, GAME_BF16 = 0, 1
GAME_INIT_NORMAL, GAME_INIT_UNIFORM, GAME_INIT_UNIT = 0, 1, 2
GAME_TOURNAMENT, GAME_RANKING, GAME_ROULETTE = 0, 1, 2


class game_config(ctypes.Structure):
    _fields_ = [
        ("basis", c_int32), ("degree", c_int32), ("population", c_int32),
        ("tournament_k", c_int32), ("elitism", c_int32), ("elite_mode", c_int32),
        ("init_mode", c_int32), ("error_fn", c_int32), ("precision", c_int32),
        ("p_crossover", c_float), ("p_mutation", c_float), ("sigma_mutation", c_float),
        ("tmse_R", c_float), ("seed", c_uint64), ("max_generations", c_int32),
        ("target", c_double), ("selection", c_int32),
    ]


class game_surrogate_config(ctypes.Structure):
    _fields_ = [("hidden", c_int32), ("fp32_operands", c_int32), ("archive", c_int32),
                ("minibatch", c_int32), ("train_steps", c_int32), ("lr", c_float),
                ("oversample", c_int32), ("audit", c_int32), ("rho_min", c_float),
                ("min_archive", c_int32), ("seed", c_uint64)]


class game_run_desc(ctypes.Structure):
    _fields_ = [("X_dev", c_void_p), ("t_dev", c_void_p), ("n_patterns", c_int64),
                ("n_features", c_int32), ("reserved", c_int32), ("cfg", game_config)]


class GameError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libgame error {code}: {msg}")
        self.code = code


_lib = None
_SIGS = {
    "game_config_default": (c_int32, [POINTER(game_config)]),
    "game_num_genes": (c_int32, [POINTER(game_config), c_int32]),
    "game_workspace_size": (c_size_t, [POINTER(game_config), c_int64, c_int32]),
    "game_create": (c_int32, [POINTER(game_config), c_void_p, c_void_p, c_int64, c_int32,
                              c_void_p, c_size_t, c_void_p, POINTER(c_void_p)]),
    "game_destroy": (c_int32, [c_void_p]),
    "game_fitness": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p]),
    "game_evaluate": (c_int32, [c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_int32,
                                c_void_p]),
    "game_rescore64": (c_int32, [c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_int32,
                                 c_void_p]),
    "game_predict": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p, c_int32, c_void_p]),
    "game_classify": (c_int32, [c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_int32, c_float,
                                c_void_p]),
    "game_merit": (c_int32, [c_void_p, c_void_p]),
    "game_trig_sums": (c_int32, [c_void_p, c_int64, c_int32, c_int32, c_void_p, c_void_p]),
    "game_init_population": (c_int32, [c_void_p]),
    "game_step": (c_int32, [c_void_p]),
    "game_run": (c_int32, [c_void_p, c_int32, c_double, POINTER(c_int32), c_void_p,
                           POINTER(c_double)]),
    "game_get_population": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "game_set_population": (c_int32, [c_void_p, c_void_p, c_int32]),
    "game_get_state": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32),
                                 POINTER(c_double)]),
    "game_rank": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "game_ga_workspace_size": (c_size_t, [POINTER(game_config)]),
    "game_ga_next": (c_int32, [POINTER(game_config), c_int32, c_void_p, c_void_p, c_int32,
                               c_void_p, c_void_p, c_size_t, c_void_p]),
    "game_ga_next_static": (c_int32, [POINTER(game_config), c_int32, c_void_p, c_void_p, c_int32,
                                      c_void_p, c_void_p]),
    "game_init_genes": (c_int32, [POINTER(game_config), c_int32, c_void_p, c_void_p]),
    "game_last_error": (ctypes.c_char_p, []),
    "game_surrogate_config_default": (c_int32, [POINTER(game_surrogate_config)]),
    "game_surrogate_workspace_size": (c_size_t, [POINTER(game_surrogate_config), c_int32,
                                                 c_int32]),
    "game_surrogate_create": (c_int32, [POINTER(game_surrogate_config), c_int32, c_int32,
                                        c_void_p, c_size_t, c_void_p, POINTER(c_void_p)]),
    "game_surrogate_destroy": (c_int32, [c_void_p]),
    "game_surrogate_num_params": (c_int64, [c_void_p]),
    "game_surrogate_get_params": (c_int32, [c_void_p, c_void_p]),
    "game_surrogate_get_input_stats": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "game_surrogate_set_params": (c_int32, [c_void_p, c_void_p]),
    "game_surrogate_predict": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p]),
    "game_surrogate_gradients": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_void_p,
                                           c_void_p]),
    "game_surrogate_train_step": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32]),
    "game_attach_surrogate": (c_int32, [c_void_p, c_void_p]),
    "game_surrogate_stats": (c_int32, [c_void_p, POINTER(c_float), POINTER(c_int32),
                                       POINTER(c_int32), POINTER(c_int32), POINTER(c_int32)]),
    "game_batch_workspace_size": (c_size_t, [POINTER(game_run_desc), c_int32]),
    "game_batch_create": (c_int32, [POINTER(game_run_desc), c_int32, c_void_p, c_size_t, c_void_p,
                                    POINTER(c_void_p)]),
    "game_batch_destroy": (c_int32, [c_void_p]),
    "game_batch_tune": (c_int32, [c_void_p, c_int32, c_int32]),
    "game_batch_tune_runs": (c_int32, [c_void_p, c_void_p, c_int32]),
    "game_batch_get_tuning": (c_int32, [c_void_p, c_void_p, POINTER(c_int32)]),
    "game_batch_autotune_buckets": (c_int32, [c_void_p, c_int32, c_void_p, c_int32, c_void_p,
                                              POINTER(c_int32), POINTER(c_float)]),
    "game_batch_autotune": (c_int32, [c_void_p, c_int32, POINTER(c_int32), POINTER(c_int32),
                                      POINTER(c_float), c_void_p]),
    "game_batch_init": (c_int32, [c_void_p]),
    "game_batch_step": (c_int32, [c_void_p]),
    "game_batch_evaluate": (c_int32, [c_void_p]),
    "game_batch_run": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "game_batch_get_population": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "game_batch_num_items": (c_int32, [c_void_p, POINTER(c_int32), POINTER(c_int32),
                                       POINTER(c_int32)]),
}


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1304_0597_amd.build`")
        # torch first: libgame then binds to the HIP runtime torch has loaded
        # (two HIP runtimes in one process do not share devices or streams).
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def game_last_error() -> str:
    return lib().game_last_error().decode()


def _check(rc: int) -> int:
    if rc < 0:
        raise GameError(rc, game_last_error())
    return rc


def _ptr(t, dtype=None) -> int:
    """Device pointer of a contiguous CUDA/HIP tensor (None -> NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a GPU tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected dtype {dtype}, got {t.dtype}")
    return t.data_ptr()


# Sizes of every live handle, recorded by the create calls: the shape checks
# below compare each tensor with them before anything reaches the library,
# so a mismatched tensor raises ValueError instead of a kernel reading or
# writing past an allocation.
_handles: dict = {}


def _dims(h) -> dict:
    try:
        return _handles[h]
    except KeyError:
        raise ValueError("unknown handle (not created here, or already destroyed)") from None


def _shape(t, shape, name) -> None:
    """t (if not None) has exactly `shape`; None entries match any size."""
    if t is None:
        return
    got = tuple(t.shape)
    if len(got) != len(shape) or any(e is not None and g != e for g, e in zip(got, shape)):
        want = "x".join("*" if e is None else str(e) for e in shape)
        raise ValueError(f"{name}: expected shape [{want}], got {list(got)}")


def _rows(t, n, cols, name) -> None:
    """t is [rows x cols] with at least n rows (n chromosomes read or written)."""
    _shape(t, (None, cols), name)
    if t.shape[0] < n:
        raise ValueError(f"{name}: {t.shape[0]} rows, the call uses {n}")


def _numel(t, n, name) -> None:
    """t (if not None) has at least n elements."""
    if t is not None and t.numel() < n:
        raise ValueError(f"{name}: {t.numel()} elements, the call uses {n}")


def _data(X, t, n_features, name="X") -> None:
    """A data set: X [NP x N] with the expected N, t [NP] (if given)."""
    _shape(X, (None, n_features), name)
    if t is not None:
        _shape(t, (X.shape[0],), "t")


def _stream(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def config(**kw) -> game_config:
    """A game_config with the library defaults, overridden by ``kw``."""
    c = game_config()
    _check(lib().game_config_default(ctypes.byref(c)))
    for k, v in kw.items():
        if not hasattr(c, k):
            raise AttributeError(k)
        setattr(c, k, v)
    return c


def game_config_default() -> game_config:
    return config()


def game_num_genes(cfg: game_config, n_features: int) -> int:
    return _check(lib().game_num_genes(ctypes.byref(cfg), n_features))


def game_workspace_size(cfg: game_config, n_patterns: int, n_features: int) -> int:
    n = lib().game_workspace_size(ctypes.byref(cfg), n_patterns, n_features)
    if n == 0:
        raise GameError(GAME_EINVAL, game_last_error())
    return n


def game_create(cfg, X, t, workspace, stream=None) -> int:
    import torch
    _shape(X, (None, None), "X")
    _shape(t, (X.shape[0],), "t")
    K = game_num_genes(cfg, X.shape[1])
    h = c_void_p()
    _check(lib().game_create(ctypes.byref(cfg), _ptr(X, torch.float32), _ptr(t, torch.float32),
                             X.shape[0], X.shape[1], _ptr(workspace),
                             workspace.numel() * workspace.element_size(), _stream(stream),
                             ctypes.byref(h)))
    _handles[h.value] = {"n_patterns": X.shape[0], "n_features": X.shape[1], "n_genes": K,
                         "population": cfg.population}
    return h.value


def game_destroy(h) -> None:
    _check(lib().game_destroy(h))
    _handles.pop(h, None)


def game_fitness(h, genes, n, fitness, fitness64=None) -> None:
    import torch
    _rows(genes, n, _dims(h)["n_genes"], "genes")
    _numel(fitness, n, "fitness")
    _numel(fitness64, n, "fitness64")
    _check(lib().game_fitness(h, _ptr(genes, torch.float32), n, _ptr(fitness, torch.float32),
                              _ptr(fitness64, torch.float64)))


def game_evaluate(h, X, t, genes, n, err64) -> None:
    import torch
    d = _dims(h)
    _data(X, t, d["n_features"])
    _rows(genes, n, d["n_genes"], "genes")
    _numel(err64, n, "err64")
    _check(lib().game_evaluate(h, _ptr(X, torch.float32), _ptr(t, torch.float32), X.shape[0],
                               _ptr(genes, torch.float32), n, _ptr(err64, torch.float64)))


def game_rescore64(h, X, t, genes, n, err64) -> None:
    """X, t None -> the handle's own data set."""
    import torch
    d = _dims(h)
    _data(X, t, d["n_features"])
    _rows(genes, n, d["n_genes"], "genes")
    _numel(err64, n, "err64")
    n_patterns = X.shape[0] if X is not None else 0
    _check(lib().game_rescore64(h, _ptr(X, torch.float32), _ptr(t, torch.float32), n_patterns,
                                _ptr(genes, torch.float32), n, _ptr(err64, torch.float64)))


def game_predict(h, X, genes, n, out) -> None:
    """X None -> the handle's own data set."""
    import torch
    d = _dims(h)
    _data(X, None, d["n_features"])
    n_patterns = X.shape[0] if X is not None else d["n_patterns"]
    _rows(genes, n, d["n_genes"], "genes")
    _rows(out, n, n_patterns, "out")
    n_patterns = X.shape[0] if X is not None else 0
    _check(lib().game_predict(h, _ptr(X, torch.float32), n_patterns, _ptr(genes, torch.float32),
                              n, _ptr(out, torch.float32)))


def game_classify(h, X, t, genes, n, threshold, counts) -> None:
    """X, t None -> the handle's own data set."""
    import torch
    d = _dims(h)
    _data(X, t, d["n_features"])
    _rows(genes, n, d["n_genes"], "genes")
    _rows(counts, n, 4, "counts")
    n_patterns = X.shape[0] if X is not None else 0
    _check(lib().game_classify(h, _ptr(X, torch.float32), _ptr(t, torch.float32), n_patterns,
                               _ptr(genes, torch.float32), n, threshold,
                               _ptr(counts, torch.int64)))


def game_trig_sums(X, degree: int, Z=None, stream=None):
    """Per-pattern cos/sin sums of the shared-gene model: Z [NP x 2*degree]."""
    import torch
    _shape(X, (None, None), "X")
    if Z is None:
        Z = torch.empty((X.shape[0], 2 * degree), dtype=torch.float32, device=X.device)
    if 1 <= degree <= 16:      # other degrees are the library's to reject
        _shape(Z, (X.shape[0], 2 * degree), "Z")
    _check(lib().game_trig_sums(_ptr(X, torch.float32), X.shape[0], X.shape[1], degree,
                                _ptr(Z, torch.float32), _stream(stream)))
    return Z


def game_merit(counts) -> dict:
    """counts: four integers (TP, FP, TN, FN)."""
    c = (ctypes.c_int64 * 4)(*[int(v) for v in counts])
    m = (c_double * 4)()
    _check(lib().game_merit(c, m))
    return {"accuracy": m[0], "completeness": m[1], "contamination": m[2],
            "contamination_of_predicted": m[3]}


def game_init_population(h) -> None:
    _check(lib().game_init_population(h))


def game_step(h) -> None:
    _check(lib().game_step(h))


def game_run(h, n_genes: int, max_generations: int = -1, target: float = -1.0):
    """Returns (generations_done, best_genes [K] float32 numpy, best_error)."""
    if n_genes != _dims(h)["n_genes"]:
        raise ValueError(f"n_genes {n_genes}, the handle has {_dims(h)['n_genes']}")
    gens = c_int32()
    best = np.zeros(n_genes, dtype=np.float32)
    err = c_double()
    _check(lib().game_run(h, max_generations, target, ctypes.byref(gens),
                          best.ctypes.data_as(c_void_p), ctypes.byref(err)))
    return gens.value, best, err.value


def game_get_population(h, genes, fitness=None) -> None:
    import torch
    d = _dims(h)
    _shape(genes, (d["population"], d["n_genes"]), "genes")
    _shape(fitness, (d["population"],), "fitness")
    _check(lib().game_get_population(h, _ptr(genes, torch.float32), _ptr(fitness, torch.float32)))


def game_set_population(h, genes, generation: int) -> None:
    import torch
    d = _dims(h)
    _shape(genes, (d["population"], d["n_genes"]), "genes")
    _check(lib().game_set_population(h, _ptr(genes, torch.float32), generation))


def game_get_state(h) -> dict:
    g, s, b, e = c_int32(), c_int32(), c_int32(), c_double()
    _check(lib().game_get_state(h, ctypes.byref(g), ctypes.byref(s), ctypes.byref(b),
                                ctypes.byref(e)))
    return {"generation": g.value, "stopped": s.value, "best_index": b.value,
            "best_error": e.value}


def game_rank(fitness, n, order, stream=None) -> None:
    import torch
    _numel(fitness, n, "fitness")
    _numel(order, n, "order")
    _check(lib().game_rank(_ptr(fitness, torch.float32), n, _ptr(order, torch.int32),
                           _stream(stream)))


def game_ga_workspace_size(cfg) -> int:
    n = lib().game_ga_workspace_size(ctypes.byref(cfg))
    if n == 0:
        raise GameError(GAME_EINVAL, game_last_error())
    return n


def game_ga_next(cfg, n_genes, pop, fitness, generation, out, workspace, stream=None) -> None:
    import torch
    _shape(pop, (cfg.population, n_genes), "pop")
    _shape(fitness, (cfg.population,), "fitness")
    _shape(out, (cfg.population, n_genes), "out")
    _check(lib().game_ga_next(ctypes.byref(cfg), n_genes, _ptr(pop, torch.float32),
                              _ptr(fitness, torch.float32), generation, _ptr(out, torch.float32),
                              _ptr(workspace), workspace.numel() * workspace.element_size(),
                              _stream(stream)))


def game_ga_next_static(cfg, n_genes, pop, fitness, generation, out, stream=None) -> None:
    import torch
    _shape(pop, (cfg.population, n_genes), "pop")
    _shape(fitness, (cfg.population,), "fitness")
    _shape(out, (cfg.population, n_genes), "out")
    _check(lib().game_ga_next_static(ctypes.byref(cfg), n_genes, _ptr(pop, torch.float32),
                                     _ptr(fitness, torch.float32), generation,
                                     _ptr(out, torch.float32), _stream(stream)))


def game_init_genes(cfg, n_genes, out, stream=None) -> None:
    import torch
    _shape(out, (cfg.population, n_genes), "out")
    _check(lib().game_init_genes(ctypes.byref(cfg), n_genes, _ptr(out, torch.float32),
                                 _stream(stream)))


class Game:
    """A handle plus the torch-allocated workspace it carves, and references
    to the data set so it stays alive."""

    def __init__(self, cfg: game_config, X, t, stream=None):
        import torch
        self.cfg = cfg
        self.X, self.t = X, t
        self.n_genes = game_num_genes(cfg, X.shape[1])
        nbytes = game_workspace_size(cfg, X.shape[0], X.shape[1])
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=X.device)
        self.h = game_create(cfg, X, t, self.workspace, stream)

    def close(self):
        if self.h:
            game_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def fitness(self, genes, with64=False):
        import torch
        n = genes.shape[0]
        f = torch.empty(n, dtype=torch.float32, device=genes.device)
        f64 = torch.empty(n, dtype=torch.float64, device=genes.device) if with64 else None
        game_fitness(self.h, genes, n, f, f64)
        return (f, f64) if with64 else f

    def evaluate(self, X, t, genes):
        import torch
        out = torch.empty(genes.shape[0], dtype=torch.float64, device=genes.device)
        game_evaluate(self.h, X, t, genes, genes.shape[0], out)
        return out

    def rescore64(self, genes, X=None, t=None):
        import torch
        out = torch.empty(genes.shape[0], dtype=torch.float64, device=genes.device)
        game_rescore64(self.h, X, t, genes, genes.shape[0], out)
        return out

    def predict(self, genes, X=None):
        import torch
        n_patterns = X.shape[0] if X is not None else self.X.shape[0]
        out = torch.empty((genes.shape[0], n_patterns), dtype=torch.float32, device=genes.device)
        game_predict(self.h, X, genes, genes.shape[0], out)
        return out

    def classify(self, genes, X=None, t=None, threshold=0.5):
        """Counts [n x 4] (TP, FP, TN, FN) on the device."""
        import torch
        counts = torch.empty((genes.shape[0], 4), dtype=torch.int64, device=genes.device)
        game_classify(self.h, X, t, genes, genes.shape[0], threshold, counts)
        return counts

    def init_population(self):
        game_init_population(self.h)

    def step(self):
        game_step(self.h)

    def run(self, max_generations=-1, target=-1.0):
        return game_run(self.h, self.n_genes, max_generations, target)

    def population(self):
        import torch
        g = torch.empty((self.cfg.population, self.n_genes), dtype=torch.float32,
                        device=self.X.device)
        f = torch.empty(self.cfg.population, dtype=torch.float32, device=self.X.device)
        game_get_population(self.h, g, f)
        return g, f

    def set_population(self, genes, generation):
        game_set_population(self.h, genes, generation)

    def state(self):
        return game_get_state(self.h)


# ------------------------------------------------------------------ batches
AUTOTUNE_TILES = (1, 2, 4, 8, 16, 32, 64, 128)
AUTOTUNE_GRIDS = (256, 512, 1024)


def _descs(problems, cfgs):
    import torch
    arr = (game_run_desc * len(problems))()
    for i, ((X, t), c) in enumerate(zip(problems, cfgs)):
        _data(X, t, None, f"run {i}: X")
        arr[i].X_dev = _ptr(X, torch.float32)
        arr[i].t_dev = _ptr(t, torch.float32)
        arr[i].n_patterns = X.shape[0]
        arr[i].n_features = X.shape[1]
        arr[i].reserved = 0
        arr[i].cfg = c
    return arr


def game_batch_workspace_size(descs, n_runs) -> int:
    n = lib().game_batch_workspace_size(descs, n_runs)
    if n == 0:
        raise GameError(GAME_EINVAL, game_last_error())
    return n


def game_batch_create(descs, n_runs, workspace, stream=None) -> int:
    if n_runs > len(descs):
        raise ValueError(f"{len(descs)} run descriptors, the call uses {n_runs}")
    runs = [{"population": descs[i].cfg.population,
             "n_genes": game_num_genes(descs[i].cfg, descs[i].n_features)} for i in range(n_runs)]
    h = c_void_p()
    _check(lib().game_batch_create(descs, n_runs, _ptr(workspace),
                                   workspace.numel() * workspace.element_size(), _stream(stream),
                                   ctypes.byref(h)))
    _handles[h.value] = {"runs": runs, "n_runs": n_runs}
    return h.value


def game_batch_destroy(b) -> None:
    _check(lib().game_batch_destroy(b))
    _handles.pop(b, None)


def game_batch_tune(b, tiles_per_item, grid) -> None:
    _check(lib().game_batch_tune(b, tiles_per_item, grid))


def game_batch_tune_runs(b, tiles_per_item, grid) -> None:
    t = np.ascontiguousarray(tiles_per_item, dtype=np.int32)
    if t.ndim != 1 or t.size != _dims(b)["n_runs"]:
        raise ValueError(f"tiles_per_item: expected {_dims(b)['n_runs']} values, got {t.size}")
    _check(lib().game_batch_tune_runs(b, t.ctypes.data_as(c_void_p), grid))


def game_batch_get_tuning(b) -> tuple:
    t = np.zeros(_dims(b)["n_runs"], dtype=np.int32)
    g = c_int32()
    _check(lib().game_batch_get_tuning(b, t.ctypes.data_as(c_void_p), ctypes.byref(g)))
    return t, g.value


def game_batch_autotune_buckets(b, bucket_of_run, n_buckets, reps=3) -> dict:
    k = np.ascontiguousarray(bucket_of_run, dtype=np.int32)
    if k.ndim != 1 or k.size != _dims(b)["n_runs"]:
        raise ValueError(f"bucket_of_run: expected {_dims(b)['n_runs']} values, got {k.size}")
    out = np.zeros(n_buckets, dtype=np.int32)
    g, ms = c_int32(), c_float()
    _check(lib().game_batch_autotune_buckets(b, reps, k.ctypes.data_as(c_void_p), n_buckets,
                                             out.ctypes.data_as(c_void_p), ctypes.byref(g),
                                             ctypes.byref(ms)))
    return {"tiles_per_bucket": [int(v) for v in out], "grid": g.value, "ms": ms.value}


def game_batch_autotune(b, reps=3) -> dict:
    t, g, ms = c_int32(), c_int32(), c_float()
    times = np.zeros(len(AUTOTUNE_TILES) * len(AUTOTUNE_GRIDS), dtype=np.float32)
    _check(lib().game_batch_autotune(b, reps, ctypes.byref(t), ctypes.byref(g), ctypes.byref(ms),
                                     times.ctypes.data_as(c_void_p)))
    table = {f"{tt}x{gg}": float(times[i * len(AUTOTUNE_GRIDS) + j])
             for i, tt in enumerate(AUTOTUNE_TILES) for j, gg in enumerate(AUTOTUNE_GRIDS)}
    return {"tiles_per_item": t.value, "grid": g.value, "ms": ms.value, "times_ms": table}


def game_batch_init(b) -> None:
    _check(lib().game_batch_init(b))


def game_batch_step(b) -> None:
    _check(lib().game_batch_step(b))


def game_batch_evaluate(b) -> None:
    _check(lib().game_batch_evaluate(b))


def game_batch_run(b, n_runs):
    if n_runs != len(_dims(b)["runs"]):
        raise ValueError(f"n_runs {n_runs}, the batch has {len(_dims(b)['runs'])}")
    gens = np.zeros(n_runs, dtype=np.int32)
    best = np.zeros(n_runs, dtype=np.float64)
    _check(lib().game_batch_run(b, gens.ctypes.data_as(c_void_p), best.ctypes.data_as(c_void_p)))
    return gens, best


def game_batch_get_population(b, run, genes, fitness=None) -> None:
    import torch
    runs = _dims(b)["runs"]
    if not 0 <= run < len(runs):
        raise ValueError(f"run {run} not in 0..{len(runs) - 1}")
    _shape(genes, (runs[run]["population"], runs[run]["n_genes"]), "genes")
    _shape(fitness, (runs[run]["population"],), "fitness")
    _check(lib().game_batch_get_population(b, run, _ptr(genes, torch.float32),
                                           _ptr(fitness, torch.float32)))


def game_batch_num_items(b):
    n, t, g = c_int32(), c_int32(), c_int32()
    _check(lib().game_batch_num_items(b, ctypes.byref(n), ctypes.byref(t), ctypes.byref(g)))
    return n.value, t.value, g.value


class Batch:
    """Many runs advanced together: problems is a list of (X, t) GPU tensors,
    cfgs the matching game_config list."""

    def __init__(self, problems, cfgs, stream=None):
        import torch
        self.problems = problems
        self.cfgs = cfgs
        self.n_runs = len(problems)
        self.descs = _descs(problems, cfgs)
        self.n_genes = [game_num_genes(c, X.shape[1]) for (X, _), c in zip(problems, cfgs)]
        nbytes = game_batch_workspace_size(self.descs, self.n_runs)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=problems[0][0].device)
        self.h = game_batch_create(self.descs, self.n_runs, self.workspace, stream)

    def close(self):
        if self.h:
            game_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tune(self, tiles_per_item, grid):
        game_batch_tune(self.h, tiles_per_item, grid)

    def autotune(self, reps=3):
        return game_batch_autotune(self.h, reps)

    def tune_runs(self, tiles_per_item, grid):
        game_batch_tune_runs(self.h, tiles_per_item, grid)

    def tuning(self):
        return game_batch_get_tuning(self.h)

    def autotune_buckets(self, bucket_of_run, n_buckets, reps=3):
        return game_batch_autotune_buckets(self.h, bucket_of_run, n_buckets, reps)

    def init(self):
        game_batch_init(self.h)

    def step(self):
        game_batch_step(self.h)

    def evaluate(self):
        game_batch_evaluate(self.h)

    def run(self):
        return game_batch_run(self.h, self.n_runs)

    def population(self, run):
        import torch
        dev = self.problems[run][0].device
        g = torch.empty((self.cfgs[run].population, self.n_genes[run]), dtype=torch.float32,
                        device=dev)
        f = torch.empty(self.cfgs[run].population, dtype=torch.float32, device=dev)
        game_batch_get_population(self.h, run, g, f)
        return g, f

    def items(self):
        return game_batch_num_items(self.h)


# ---------------------------------------------------------------- surrogate
def surrogate_config(**kw) -> game_surrogate_config:
    c = game_surrogate_config()
    _check(lib().game_surrogate_config_default(ctypes.byref(c)))
    for k, v in kw.items():
        if not hasattr(c, k):
            raise AttributeError(k)
        setattr(c, k, v)
    return c


def game_surrogate_config_default() -> game_surrogate_config:
    return surrogate_config()


def game_surrogate_workspace_size(cfg, n_genes, max_batch) -> int:
    n = lib().game_surrogate_workspace_size(ctypes.byref(cfg), n_genes, max_batch)
    if n == 0:
        raise GameError(GAME_EINVAL, game_last_error())
    return n


def game_surrogate_create(cfg, n_genes, max_batch, workspace, stream=None) -> int:
    h = c_void_p()
    _check(lib().game_surrogate_create(ctypes.byref(cfg), n_genes, max_batch, _ptr(workspace),
                                       workspace.numel() * workspace.element_size(),
                                       _stream(stream), ctypes.byref(h)))
    _handles[h.value] = {"n_genes": n_genes, "max_batch": max_batch,
                         "minibatch": cfg.minibatch,
                         "n_params": lib().game_surrogate_num_params(h.value)}
    return h.value


def game_surrogate_destroy(s) -> None:
    _check(lib().game_surrogate_destroy(s))
    _handles.pop(s, None)


def game_surrogate_num_params(s) -> int:
    return _check(lib().game_surrogate_num_params(s))


def game_surrogate_get_params(s, params) -> None:
    import torch
    _numel(params, _dims(s)["n_params"], "params")
    _check(lib().game_surrogate_get_params(s, _ptr(params, torch.float32)))


def game_surrogate_get_input_stats(s, mean, inv_std) -> None:
    import torch
    n = _dims(s)["n_genes"]
    _numel(mean, n, "mean")
    _numel(inv_std, n, "inv_std")
    _check(lib().game_surrogate_get_input_stats(s, _ptr(mean, torch.float32),
                                                _ptr(inv_std, torch.float32)))


def game_surrogate_set_params(s, params) -> None:
    import torch
    _numel(params, _dims(s)["n_params"], "params")
    _check(lib().game_surrogate_set_params(s, _ptr(params, torch.float32)))


def game_surrogate_predict(s, genes, n, y) -> None:
    import torch
    _rows(genes, n, _dims(s)["n_genes"], "genes")
    _numel(y, n, "y")
    _check(lib().game_surrogate_predict(s, _ptr(genes, torch.float32), n, _ptr(y, torch.float32)))


def game_surrogate_gradients(s, genes, target, n, grads, y=None) -> None:
    import torch
    d = _dims(s)
    _rows(genes, n, d["n_genes"], "genes")
    _numel(target, n, "target")
    _numel(grads, d["n_params"], "grads")
    _numel(y, n, "y")
    _check(lib().game_surrogate_gradients(s, _ptr(genes, torch.float32),
                                          _ptr(target, torch.float32), n,
                                          _ptr(grads, torch.float32), _ptr(y, torch.float32)))


def game_surrogate_train_step(s, genes, target, n) -> None:
    import torch
    _rows(genes, n, _dims(s)["n_genes"], "genes")
    _numel(target, n, "target")
    _check(lib().game_surrogate_train_step(s, _ptr(genes, torch.float32),
                                           _ptr(target, torch.float32), n))


def game_attach_surrogate(h, s) -> None:
    _check(lib().game_attach_surrogate(h, s))


def game_surrogate_stats(s) -> dict:
    rho, last, total, cnt, steps = c_float(), c_int32(), c_int32(), c_int32(), c_int32()
    _check(lib().game_surrogate_stats(s, ctypes.byref(rho), ctypes.byref(last),
                                      ctypes.byref(total), ctypes.byref(cnt), ctypes.byref(steps)))
    return {"rho": rho.value, "screened_last": last.value, "screened_total": total.value,
            "archive_count": cnt.value, "adam_steps": steps.value}


class Surrogate:
    """The network plus its torch-allocated workspace."""

    def __init__(self, cfg: game_surrogate_config, n_genes: int, max_batch: int, device="cuda",
                 stream=None):
        import torch
        self.cfg = cfg
        self.n_genes = n_genes
        self.max_batch = max_batch
        nbytes = game_surrogate_workspace_size(cfg, n_genes, max_batch)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.h = game_surrogate_create(cfg, n_genes, max_batch, self.workspace, stream)
        self.n_params = game_surrogate_num_params(self.h)

    def close(self):
        if self.h:
            game_surrogate_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        import torch
        p = torch.empty(self.n_params, dtype=torch.float32, device=self.workspace.device)
        game_surrogate_get_params(self.h, p)
        return p

    def set_params(self, p):
        game_surrogate_set_params(self.h, p)

    def input_stats(self):
        """(mean, inv_std) of the network's input standardisation."""
        import torch
        n = self.n_genes
        mu = torch.empty(n, dtype=torch.float32, device=self.workspace.device)
        inv = torch.empty(n, dtype=torch.float32, device=self.workspace.device)
        game_surrogate_get_input_stats(self.h, mu, inv)
        return mu, inv

    def predict(self, genes):
        import torch
        y = torch.empty(genes.shape[0], dtype=torch.float32, device=genes.device)
        game_surrogate_predict(self.h, genes, genes.shape[0], y)
        return y

    def gradients(self, genes, target):
        import torch
        g = torch.empty(self.n_params, dtype=torch.float32, device=genes.device)
        y = torch.empty(genes.shape[0], dtype=torch.float32, device=genes.device)
        game_surrogate_gradients(self.h, genes, target, genes.shape[0], g, y)
        return g, y

    def train_step(self, genes, target):
        game_surrogate_train_step(self.h, genes, target, genes.shape[0])

    def stats(self):
        return game_surrogate_stats(self.h)
