"""GAME's genetic loop: initialisation, ranking, elitism, selection, crossover,
mutation and the training iteration.

Test infrastructure (see ``oracle/__init__.py``).

The paper fixes the loop (Sec. 4.1: generate the population, compute the
fitness and sort, test the stop criteria, evolve with the genetic operators,
repeat) and the operator *rates* (Sec. 5: crossover 0.9, mutation 0.2,
tournament of 4, elitism 2, error threshold 0.001), but not the operators'
exact form nor the random-number scheme.  This module fixes them as follows,
and the HIP library implements the same reading:

* parents are chosen by tournament (the default), by linear ranking or by
  roulette wheel (the two criteria named in Sec. 2), defined below;
* every draw comes from Philox4x64-10 with key (seed, stream) and counter
  (generation, unit, block, 0); stream 0 = initialisation (unit = chromosome,
  block = gene), 1 = selection and crossover (unit = child pair), 2 = mutation
  (unit = child slot, block = gene);
* a block's 32-bit words are lo(o0), hi(o0), lo(o1), ..., hi(o3);
* an index in [0, n) is (u32 * n) >> 32; a coin with probability p fires when
  u32 < floor(p * 2^32) (p = 1 always fires);
* a unit Gaussian is the Irwin-Hall sum of the twelve 16-bit fields S of
  words o1..o3: z = (S - 393210) * 2^-16, exactly representable in float32;
* genes are float32; every float step (sigma*z, g + sigma*z, the clamp to
  [-1, 1]) is one IEEE round-to-nearest-even operation.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import game
from .philox import block

STREAM_INIT, STREAM_SELECT, STREAM_MUTATE = 0, 1, 2
INIT_NORMAL, INIT_UNIFORM, INIT_UNIT = 0, 1, 2
SELECT_TOURNAMENT, SELECT_RANKING, SELECT_ROULETTE = 0, 1, 2

_M32 = np.uint64(0xFFFFFFFF)


@dataclasses.dataclass
class GAConfig:
    population: int
    tournament_k: int = 3
    elitism: int = 2
    elite_mode: int = 0          # 0: E copies of the winner; 1: the E best
    p_crossover: float = 0.9
    p_mutation: float = 0.05
    sigma_mutation: float = 0.1
    seed: int = 0
    init_mode: int = INIT_NORMAL
    selection: int = SELECT_TOURNAMENT


def words(blocks_u64: np.ndarray) -> np.ndarray:
    """[..., 4] uint64 Philox outputs -> [..., 8] uint32-valued words."""
    lo = blocks_u64 & _M32
    hi = blocks_u64 >> np.uint64(32)
    return np.stack([lo, hi], axis=-1).reshape(blocks_u64.shape[:-1] + (8,))


def coin_threshold(p: float) -> int:
    """floor(p * 2^32) with p taken as float32, then widened exactly."""
    return int(np.floor(float(np.float32(p)) * 4294967296.0))


def index_draw(u32, n: int):
    return (np.asarray(u32, dtype=np.uint64) * np.uint64(n)) >> np.uint64(32)


def gauss12(blocks_u64: np.ndarray) -> np.ndarray:
    """Irwin-Hall(12) unit Gaussian from output words o1, o2, o3 (float32)."""
    s = np.zeros(blocks_u64.shape[:-1], dtype=np.int64)
    for w in (1, 2, 3):
        v = blocks_u64[..., w]
        for f in range(4):
            s += ((v >> np.uint64(16 * f)) & np.uint64(0xFFFF)).astype(np.int64)
    return ((s - 393210).astype(np.float64) * 2.0 ** -16).astype(np.float32)


def clamp_unit(v: np.ndarray) -> np.ndarray:
    """Clamp to [-1, 1]; NaN passes through unchanged."""
    v = np.asarray(v, dtype=np.float32)
    one = np.float32(1.0)
    return np.where(v < -one, -one, np.where(v > one, one, v)).astype(np.float32)


def init_population(P: int, K: int, seed: int, mode: int = INIT_NORMAL) -> np.ndarray:
    """Generation-0 genes (the three random modes listed in Sec. 2):
    normal in [-1, 1] (sigma 1/3, clamped), uniform in [-1, 1), uniform in
    [0, 1)."""
    ch = np.arange(P, dtype=np.uint64)[:, None]
    gn = np.arange(K, dtype=np.uint64)[None, :]
    b = block(seed, STREAM_INIT, 0, ch, gn)               # [P, K, 4]
    lo = (b[..., 0] & _M32) >> np.uint64(8)                 # 24 bits
    if mode == INIT_NORMAL:
        return clamp_unit(np.float32(1.0 / 3.0) * gauss12(b))
    if mode == INIT_UNIFORM:
        return ((lo.astype(np.int64) - (1 << 23)).astype(np.float64) * 2.0 ** -23).astype(np.float32)
    if mode == INIT_UNIT:
        return (lo.astype(np.float64) * 2.0 ** -24).astype(np.float32)
    raise ValueError(f"unknown init mode {mode}")


def canonical_fitness(fit) -> np.ndarray:
    """float32 ranking keys: NaN counts as +inf and -0 as +0."""
    f = np.asarray(fit, dtype=np.float32).copy()
    f[np.isnan(f)] = np.inf
    f[f == 0] = np.float32(0.0)
    return f


def rank_order(fit) -> np.ndarray:
    """Chromosome indices sorted by (fitness ascending, index ascending)."""
    f = canonical_fitness(fit)
    return np.lexsort((np.arange(f.size), f)).astype(np.int64)


def _tournament(f: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """Winner of each row of candidate indices: lowest (fitness, index)."""
    best = idx[:, 0].copy()
    for c in range(1, idx.shape[1]):
        cand = idx[:, c]
        better = (f[cand] < f[best]) | ((f[cand] == f[best]) & (cand < best))
        best = np.where(better, cand, best)
    return best


def ranking_pick(fit, u32) -> np.ndarray:
    """Linear ranking with selection pressure 2 (one of the two selection
    criteria named in Sec. 2): rank r (0 = best) has weight P - r.  The
    draw t = (u32 * P(P+1)/2) >> 32 picks the rank whose cumulative weight
    interval contains t."""
    f = canonical_fitness(fit)
    P = f.size
    order = rank_order(f)
    W = P * (P + 1) // 2
    t = (np.asarray(u32, dtype=np.uint64) * np.uint64(W)) >> np.uint64(32)
    r = np.arange(P, dtype=np.int64)
    cum_end = (r + 1) * P - (r + 1) * r // 2            # weight of ranks 0..r
    ranks = np.searchsorted(cum_end, t.astype(np.int64), side="right")
    return order[ranks]


def roulette_cumulative(fit) -> np.ndarray:
    """Roulette wheel (the other criterion of Sec. 2): weight 1/(MSE + 1e-12)
    in float64 (an infinite or NaN error weighs 0), summed left to right."""
    f = canonical_fitness(fit).astype(np.float64)
    w = 1.0 / (f + 1e-12)
    return np.cumsum(w)


def roulette_pick(cum, u32) -> np.ndarray:
    """First index whose cumulative weight exceeds (u32 2^-32) * total; a
    wheel of zero total falls back to the uniform index draw."""
    total = cum[-1]
    u = np.asarray(u32, dtype=np.uint64)
    if not total > 0:
        return index_draw(u, cum.size).astype(np.int64)
    target = (u.astype(np.float64) * 2.0 ** -32) * total
    return np.minimum(np.searchsorted(cum, target, side="right"), cum.size - 1).astype(np.int64)


def select_pairs(fit, P: int, K: int, generation: int, cfg: GAConfig):
    """Parent selection and crossover decisions for every child pair.

    Returns (parent1, parent2, crossover, cut), each of length
    ceil((P - E) / 2).  Pair q reads stream-1 words in order: the draws for
    parent 1 and parent 2 (k words each for a tournament of size k, one word
    each for ranking and roulette), the crossover coin, then the cut point
    1 + (u32 * (K - 1)) >> 32, a cut in [1, K-1]."""
    E = cfg.elitism
    k = cfg.tournament_k if cfg.selection == SELECT_TOURNAMENT else 1
    n_pairs = (P - E + 1) // 2
    f = canonical_fitness(fit)
    n_words = 2 * k + 2
    n_blocks = (n_words + 7) // 8
    q = np.arange(n_pairs, dtype=np.uint64)[:, None]
    bl = np.arange(n_blocks, dtype=np.uint64)[None, :]
    w = words(block(cfg.seed, STREAM_SELECT, generation, q, bl)).reshape(n_pairs, -1)
    if cfg.selection == SELECT_TOURNAMENT:
        p1 = _tournament(f, index_draw(w[:, 0:k], P).astype(np.int64))
        p2 = _tournament(f, index_draw(w[:, k:2 * k], P).astype(np.int64))
    elif cfg.selection == SELECT_RANKING:
        p1 = ranking_pick(f, w[:, 0])
        p2 = ranking_pick(f, w[:, 1])
    elif cfg.selection == SELECT_ROULETTE:
        cum = roulette_cumulative(f)
        p1 = roulette_pick(cum, w[:, 0])
        p2 = roulette_pick(cum, w[:, 1])
    else:
        raise ValueError(f"unknown selection {cfg.selection}")
    cross = w[:, 2 * k] < np.uint64(coin_threshold(cfg.p_crossover))
    cut = (1 + index_draw(w[:, 2 * k + 1], K - 1)).astype(np.int64)
    return p1, p2, cross, cut


def mutate(children: np.ndarray, slots: np.ndarray, generation: int, cfg: GAConfig) -> np.ndarray:
    """Per-gene Gaussian mutation of the children in ``slots``: with
    probability p_m a gene becomes clamp(g + sigma * z, -1, 1)."""
    K = children.shape[1]
    b = block(cfg.seed, STREAM_MUTATE, generation,
              np.asarray(slots, dtype=np.uint64)[:, None],
              np.arange(K, dtype=np.uint64)[None, :])          # [n, K, 4]
    fire = (b[..., 0] & _M32) < np.uint64(coin_threshold(cfg.p_mutation))
    step = np.float32(cfg.sigma_mutation) * gauss12(b)           # float32 RNE
    moved = clamp_unit(children + step)                          # float32 RNE
    return np.where(fire, moved, children).astype(np.float32)


def ga_next(pop, fit, generation: int, cfg: GAConfig) -> np.ndarray:
    """The population of generation ``generation`` built from ``pop`` (the
    previous generation) and its float32 fitness ``fit``.

    Slots 0..E-1: elitism, kept unchanged and unmutated (E copies of the
    winner, or the E best with elite_mode 1).  Slots E+2q and E+2q+1: the
    two children of pair q (the second is dropped when P - E is odd)."""
    pop = np.asarray(pop, dtype=np.float32)
    P, K = pop.shape
    E = cfg.elitism
    out = np.empty_like(pop)
    order = rank_order(fit)
    if E:
        src = np.full(E, order[0]) if cfg.elite_mode == 0 else order[:E]
        out[:E] = pop[src]
    p1, p2, cross, cut = select_pairs(fit, P, K, generation, cfg)
    g = np.arange(K)[None, :]
    swap = cross[:, None] & (g >= cut[:, None])
    a = np.where(swap, pop[p2], pop[p1])
    b = np.where(swap, pop[p1], pop[p2])
    kids = np.empty((2 * p1.size, K), dtype=np.float32)
    kids[0::2], kids[1::2] = a, b
    kids = kids[:P - E]
    slots = np.arange(E, P)
    out[E:] = mutate(kids, slots, generation, cfg)
    return out


def run(X, t, basis, degree: int, cfg: GAConfig, max_generations: int,
        target: float = 1e-3, error_fn=game.MSE, R: float = 0.0, pop0=None):
    """The training use case: evaluate, rank, test the stop criteria (error
    threshold or maximum number of iterations), evolve, repeat.

    The stop test runs after every evaluation, generation 0 included;
    ``generations`` counts the evolution steps applied."""
    K = game.num_genes(basis, np.asarray(X).shape[1], degree)
    pop = init_population(cfg.population, K, cfg.seed, cfg.init_mode) if pop0 is None \
        else np.asarray(pop0, dtype=np.float32)
    history = []
    g = 0
    while True:
        f64 = game.fitness(X, t, pop, basis, degree, error_fn, R)
        f32 = f64.astype(np.float32)
        best = int(rank_order(f32)[0])
        history.append(float(f64[best]))
        if f64[best] <= target or g >= max_generations:
            break
        g += 1
        pop = ga_next(pop, f32, g, cfg)
    return {"population": pop, "fitness": f64, "best": best, "best_genes": pop[best].copy(),
            "best_fitness": float(f64[best]), "generations": g, "history": history}
