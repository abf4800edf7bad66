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


class game_config(ctypes.Structure):
    _fields_ = [
        ("basis", c_int32), ("degree", c_int32), ("population", c_int32),
        ("tournament_k", c_int32), ("elitism", c_int32), ("elite_mode", c_int32),
        ("init_mode", c_int32), ("error_fn", c_int32), ("precision", c_int32),
        ("p_crossover", c_float), ("p_mutation", c_float), ("sigma_mutation", c_float),
        ("tmse_R", c_float), ("seed", c_uint64), ("max_generations", c_int32),
        ("target", c_double),
    ]


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
    "game_init_genes": (c_int32, [POINTER(game_config), c_int32, c_void_p, c_void_p]),
    "game_last_error": (ctypes.c_char_p, []),
}


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1304_0597_amd.build`")
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
    h = c_void_p()
    _check(lib().game_create(ctypes.byref(cfg), _ptr(X, torch.float32), _ptr(t, torch.float32),
                             X.shape[0], X.shape[1], _ptr(workspace),
                             workspace.numel() * workspace.element_size(), _stream(stream),
                             ctypes.byref(h)))
    return h.value


def game_destroy(h) -> None:
    _check(lib().game_destroy(h))


def game_fitness(h, genes, n, fitness, fitness64=None) -> None:
    import torch
    _check(lib().game_fitness(h, _ptr(genes, torch.float32), n, _ptr(fitness, torch.float32),
                              _ptr(fitness64, torch.float64)))


def game_evaluate(h, X, t, genes, n, err64) -> None:
    import torch
    _check(lib().game_evaluate(h, _ptr(X, torch.float32), _ptr(t, torch.float32), X.shape[0],
                               _ptr(genes, torch.float32), n, _ptr(err64, torch.float64)))


def game_init_population(h) -> None:
    _check(lib().game_init_population(h))


def game_step(h) -> None:
    _check(lib().game_step(h))


def game_run(h, n_genes: int, max_generations: int = -1, target: float = -1.0):
    """Returns (generations_done, best_genes [K] float32 numpy, best_error)."""
    gens = c_int32()
    best = np.zeros(n_genes, dtype=np.float32)
    err = c_double()
    _check(lib().game_run(h, max_generations, target, ctypes.byref(gens),
                          best.ctypes.data_as(c_void_p), ctypes.byref(err)))
    return gens.value, best, err.value


def game_get_population(h, genes, fitness=None) -> None:
    import torch
    _check(lib().game_get_population(h, _ptr(genes, torch.float32), _ptr(fitness, torch.float32)))


def game_set_population(h, genes, generation: int) -> None:
    import torch
    _check(lib().game_set_population(h, _ptr(genes, torch.float32), generation))


def game_get_state(h) -> dict:
    g, s, b, e = c_int32(), c_int32(), c_int32(), c_double()
    _check(lib().game_get_state(h, ctypes.byref(g), ctypes.byref(s), ctypes.byref(b),
                                ctypes.byref(e)))
    return {"generation": g.value, "stopped": s.value, "best_index": b.value,
            "best_error": e.value}


def game_rank(fitness, n, order, stream=None) -> None:
    import torch
    _check(lib().game_rank(_ptr(fitness, torch.float32), n, _ptr(order, torch.int32),
                           _stream(stream)))


def game_ga_workspace_size(cfg) -> int:
    n = lib().game_ga_workspace_size(ctypes.byref(cfg))
    if n == 0:
        raise GameError(GAME_EINVAL, game_last_error())
    return n


def game_ga_next(cfg, n_genes, pop, fitness, generation, out, workspace, stream=None) -> None:
    import torch
    _check(lib().game_ga_next(ctypes.byref(cfg), n_genes, _ptr(pop, torch.float32),
                              _ptr(fitness, torch.float32), generation, _ptr(out, torch.float32),
                              _ptr(workspace), workspace.numel() * workspace.element_size(),
                              _stream(stream)))


def game_init_genes(cfg, n_genes, out, stream=None) -> None:
    import torch
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
