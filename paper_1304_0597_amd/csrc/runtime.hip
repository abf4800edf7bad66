// Host runtime of libgame: configuration checks, workspace carving, kernel
// launches on the caller's stream, and the graph-captured training loop.
// The library allocates no device memory: every buffer comes from the
// caller's workspace.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>

#include "../../include/game.h"
#include "common.h"

using namespace game;

namespace {

thread_local std::string g_error;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(GAME_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define GAME_HIP(call)                               \
  do {                                               \
    hipError_t e_ = (call);                          \
    if (e_ != hipSuccess) return hip_fail(e_, #call); \
  } while (0)

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int blocks_of(int basis) { return basis == GAME_TRIG ? 2 : 1; }

int64_t genes_of(const game_config* c, int32_t n_features) {
  return (int64_t)blocks_of(c->basis) * n_features * c->degree + 1;
}

int check_config(const game_config* c, int32_t n_features) {
  if (!c) return fail(GAME_EINVAL, "config is NULL");
  if (c->basis < 0 || c->basis > 3) return fail(GAME_EINVAL, "basis %d not in 0..3", c->basis);
  if (c->degree < 1 || c->degree > kMaxDegree)
    return fail(GAME_EINVAL, "degree %d not in 1..%d", c->degree, kMaxDegree);
  if (c->population < 2 || c->population > kMaxPopulation)
    return fail(GAME_EINVAL, "population %d not in 2..%d", c->population, kMaxPopulation);
  if (c->tournament_k < 1 || c->tournament_k > c->population || c->tournament_k > 64)
    return fail(GAME_EINVAL, "tournament_k %d not in 1..min(population, 64)", c->tournament_k);
  if (c->elitism < 0 || c->elitism >= c->population)
    return fail(GAME_EINVAL, "elitism %d not in 0..population-1", c->elitism);
  if (c->elite_mode != 0 && c->elite_mode != 1)
    return fail(GAME_EINVAL, "elite_mode %d not 0 or 1", c->elite_mode);
  if (c->init_mode < 0 || c->init_mode > 2)
    return fail(GAME_EINVAL, "init_mode %d not in 0..2", c->init_mode);
  if (c->error_fn < 0 || c->error_fn > 3)
    return fail(GAME_EINVAL, "error_fn %d not in 0..3", c->error_fn);
  if (c->precision != GAME_FP32)
    return fail(GAME_EINVAL, "precision %d is not available in this build", c->precision);
  if (!(c->p_crossover >= 0.f && c->p_crossover <= 1.f))
    return fail(GAME_EINVAL, "p_crossover not in [0, 1]");
  if (!(c->p_mutation >= 0.f && c->p_mutation <= 1.f))
    return fail(GAME_EINVAL, "p_mutation not in [0, 1]");
  if (!(c->sigma_mutation >= 0.f) || isinf(c->sigma_mutation))
    return fail(GAME_EINVAL, "sigma_mutation must be finite and >= 0");
  if ((c->error_fn == GAME_TMSE || c->error_fn == GAME_TMSE_SQUARED) &&
      !(c->tmse_R > 0.f && c->tmse_R < 1.f))
    return fail(GAME_EINVAL, "tmse_R must lie in (0, 1)");
  if (c->max_generations < 0) return fail(GAME_EINVAL, "max_generations < 0");
  if (n_features < 1) return fail(GAME_EINVAL, "n_features %d < 1", n_features);
  if (genes_of(c, n_features) > kMaxGenes)
    return fail(GAME_EINVAL, "B*N*d+1 = %lld genes exceeds %d", (long long)genes_of(c, n_features),
                kMaxGenes);
  return GAME_OK;
}

struct Layout {
  size_t state, pop0, pop1, fit32, fit64, order, partial, total;
};

Layout layout(const game_config* c, int32_t n_features) {
  const size_t P = (size_t)c->population;
  const size_t K = (size_t)genes_of(c, n_features);
  const size_t Ppad = (P + kTileCols - 1) / kTileCols * kTileCols;
  Layout L{};
  size_t off = 0;
  L.state = off; off += align_up(sizeof(RunState));
  L.pop0 = off; off += align_up(P * K * sizeof(float));
  L.pop1 = off; off += align_up(P * K * sizeof(float));
  L.fit32 = off; off += align_up(P * sizeof(float));
  L.fit64 = off; off += align_up(P * sizeof(double));
  L.order = off; off += align_up(P * sizeof(int32_t));
  L.partial = off; off += align_up(Ppad * kMaxSplits * sizeof(double));
  L.total = off;
  return L;
}

uint64_t coin_threshold(float p) { return (uint64_t)floor((double)p * 4294967296.0); }

}  // namespace

struct game_ctx {
  game_config cfg;
  const float* X;
  const float* t;
  int64_t NP;
  int32_t N;
  int32_t K;
  hipStream_t stream;
  hipStream_t capture_stream;
  RunState* state;
  float* pop[2];
  float* fit32;
  double* fit64;
  int32_t* order;
  double* partial;
  bool initialized;
  hipGraphExec_t graph;
  int graph_steps;
};

namespace {

FitArgs fit_args(const game_ctx* h, const float* X, const float* t, int64_t NP, const float* genes,
                 int32_t n) {
  FitArgs a{};
  a.X = X;
  a.t = t;
  a.NP = NP;
  a.N = h->N;
  a.K = h->K;
  a.genes = genes;
  a.n_chrom = n;
  a.partial = h->partial;
  a.error_fn = h->cfg.error_fn;
  a.R = h->cfg.tmse_R;
  plan_fitness(a, h->cfg.degree, h->cfg.basis);
  return a;
}

GAArgs ga_args(const game_config* c, int32_t K) {
  GAArgs g{};
  g.P = c->population;
  g.K = K;
  g.k = c->tournament_k;
  g.E = c->elitism;
  g.elite_mode = c->elite_mode;
  g.thr_cross = coin_threshold(c->p_crossover);
  g.thr_mut = coin_threshold(c->p_mutation);
  g.sigma = c->sigma_mutation;
  g.seed = c->seed;
  return g;
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

// One generation of the loop on stream s: evaluate pop[gen & 1], finish and
// rank, stop test, then build pop[(gen + 1) & 1].
int enqueue_step(game_ctx* h, hipStream_t s) {
  FitArgs fa = fit_args(h, h->X, h->t, h->NP, h->pop[0], h->cfg.population);
  fa.genes_alt = h->pop[1];
  fa.gen_sel = &h->state->gen;
  fa.stop = &h->state->stop;
  fa.stop_seen = &h->state->stop_seen;
  GAME_HIP(launch_fitness_f32(fa, h->cfg.basis, h->cfg.degree, s));
  RankArgs ra{};
  ra.partial = h->partial;
  ra.n_splits = fa.n_splits;
  ra.ld_partial = fa.ld_partial;
  ra.NP = h->NP;
  ra.P = h->cfg.population;
  ra.error_fn = h->cfg.error_fn;
  ra.fit32 = h->fit32;
  ra.fit64 = h->fit64;
  ra.order = h->order;
  ra.state = h->state;
  GAME_HIP(launch_finish_rank(ra, s));
  GAArgs ga = ga_args(&h->cfg, h->K);
  ga.pop_a = h->pop[0];
  ga.pop_b = h->pop[1];
  ga.out_a = h->pop[0];
  ga.out_b = h->pop[1];
  ga.fitness = h->fit32;
  ga.order = h->order;
  ga.gen_ptr = &h->state->gen;
  ga.stop = &h->state->stop;
  GAME_HIP(launch_ga_next(ga, s));
  return GAME_OK;
}

__global__ void copy_current_kernel(const RunState* st, const float* pop0, const float* pop1,
                                    int64_t n, float* out) {
  const float* src = (st->gen & 1) ? pop1 : pop0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = src[i];
}

}  // namespace

extern "C" {

int game_config_default(game_config* c) {
  if (!c) return fail(GAME_EINVAL, "config is NULL");
  memset(c, 0, sizeof *c);
  c->basis = GAME_CHEBYSHEV;
  c->degree = 4;
  c->population = 50;
  c->tournament_k = 3;
  c->elitism = 2;
  c->elite_mode = 0;
  c->init_mode = GAME_INIT_NORMAL;
  c->error_fn = GAME_MSE;
  c->precision = GAME_FP32;
  c->p_crossover = 0.9f;
  c->p_mutation = 0.05f;
  c->sigma_mutation = 0.1f;
  c->tmse_R = 0.49f;
  c->seed = 0;
  c->max_generations = 100;
  c->target = 1e-3;
  return GAME_OK;
}

int game_num_genes(const game_config* c, int32_t n_features) {
  const int rc = check_config(c, n_features);
  if (rc) return rc;
  return (int)genes_of(c, n_features);
}

size_t game_workspace_size(const game_config* c, int64_t n_patterns, int32_t n_features) {
  if (check_config(c, n_features)) return 0;
  if (n_patterns < 1) {
    fail(GAME_EINVAL, "n_patterns < 1");
    return 0;
  }
  return layout(c, n_features).total;
}

int game_create(const game_config* c, const float* X, const float* t, int64_t NP, int32_t N,
                void* ws, size_t ws_bytes, void* stream, game_t* out) {
  if (!out) return fail(GAME_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = check_config(c, N);
  if (rc) return rc;
  if (NP < 1) return fail(GAME_EINVAL, "n_patterns < 1");
  if ((NP + kTileRows - 1) / kTileRows > (int64_t)INT32_MAX)
    return fail(GAME_EINVAL, "n_patterns too large");
  if (!X || !t) return fail(GAME_EINVAL, "X or t is NULL");
  if (!ws) return fail(GAME_EWORKSPACE, "workspace is NULL");
  if (!aligned(ws, kAlign)) return fail(GAME_EWORKSPACE, "workspace not 256-byte aligned");
  const Layout L = layout(c, N);
  if (ws_bytes < L.total)
    return fail(GAME_EWORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
  game_ctx* h = new game_ctx{};
  h->cfg = *c;
  h->X = X;
  h->t = t;
  h->NP = NP;
  h->N = N;
  h->K = (int32_t)genes_of(c, N);
  h->stream = (hipStream_t)stream;
  char* base = (char*)ws;
  h->state = (RunState*)(base + L.state);
  h->pop[0] = (float*)(base + L.pop0);
  h->pop[1] = (float*)(base + L.pop1);
  h->fit32 = (float*)(base + L.fit32);
  h->fit64 = (double*)(base + L.fit64);
  h->order = (int32_t*)(base + L.order);
  h->partial = (double*)(base + L.partial);
  hipError_t e = hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete h;
    return hip_fail(e, "hipStreamCreateWithFlags");
  }
  e = launch_set_state(h->state, 0, c->max_generations, c->target, 1, h->stream);
  if (e != hipSuccess) {
    hipStreamDestroy(h->capture_stream);
    delete h;
    return hip_fail(e, "launch_set_state");
  }
  *out = h;
  return GAME_OK;
}

int game_destroy(game_t h) {
  if (!h) return fail(GAME_EINVAL, "handle is NULL");
  if (h->graph) hipGraphExecDestroy(h->graph);
  if (h->capture_stream) hipStreamDestroy(h->capture_stream);
  delete h;
  return GAME_OK;
}

int game_fitness(game_t h, const float* genes, int32_t n, float* f32, double* f64) {
  if (!h) return fail(GAME_EINVAL, "handle is NULL");
  if (!genes || !f32) return fail(GAME_EINVAL, "genes or fitness is NULL");
  if (n < 1 || n > h->cfg.population)
    return fail(GAME_EINVAL, "n %d not in 1..population (%d)", n, h->cfg.population);
  FitArgs fa = fit_args(h, h->X, h->t, h->NP, genes, n);
  GAME_HIP(launch_fitness_f32(fa, h->cfg.basis, h->cfg.degree, h->stream));
  GAME_HIP(launch_finish(h->partial, fa.ld_partial, n, fa.n_splits, h->NP, h->cfg.error_fn, f32, f64, h->stream));
  return GAME_OK;
}

int game_evaluate(game_t h, const float* X, const float* t, int64_t NP, const float* genes,
                  int32_t n, double* err64) {
  if (!h) return fail(GAME_EINVAL, "handle is NULL");
  if (!X || !t || !genes || !err64) return fail(GAME_EINVAL, "NULL argument");
  if (NP < 1) return fail(GAME_EINVAL, "n_patterns < 1");
  if ((NP + kTileRows - 1) / kTileRows > (int64_t)INT32_MAX)
    return fail(GAME_EINVAL, "n_patterns too large");
  if (n < 1 || n > h->cfg.population)
    return fail(GAME_EINVAL, "n %d not in 1..population (%d)", n, h->cfg.population);
  FitArgs fa = fit_args(h, X, t, NP, genes, n);
  GAME_HIP(launch_fitness_f32(fa, h->cfg.basis, h->cfg.degree, h->stream));
  GAME_HIP(launch_finish(h->partial, fa.ld_partial, n, fa.n_splits, NP, h->cfg.error_fn, nullptr, err64,
                         h->stream));
  return GAME_OK;
}

int game_init_population(game_t h) {
  if (!h) return fail(GAME_EINVAL, "handle is NULL");
  GAME_HIP(launch_init_genes(h->cfg.seed, h->cfg.init_mode, h->cfg.population, h->K, h->pop[0],
                             h->stream));
  GAME_HIP(launch_set_state(h->state, 0, h->cfg.max_generations, h->cfg.target, 1, h->stream));
  h->initialized = true;
  return GAME_OK;
}

int game_step(game_t h) {
  if (!h) return fail(GAME_EINVAL, "handle is NULL");
  if (!h->initialized) return fail(GAME_ESTATE, "population not initialised");
  return enqueue_step(h, h->stream);
}

int game_run(game_t h, int32_t max_gen, double target, int32_t* gens_done, float* best_genes,
             double* best_err) {
  if (!h) return fail(GAME_EINVAL, "handle is NULL");
  if (!h->initialized) return fail(GAME_ESTATE, "population not initialised");
  if (max_gen >= 0) h->cfg.max_generations = max_gen;
  if (target >= 0) h->cfg.target = target;
  GAME_HIP(launch_set_state(h->state, 0, h->cfg.max_generations, h->cfg.target, 0, h->stream));
  RunState st{};
  GAME_HIP(hipMemcpyAsync(&st, h->state, sizeof st, hipMemcpyDeviceToHost, h->stream));
  GAME_HIP(hipStreamSynchronize(h->stream));
  if (!h->graph) {
    // Capture a fixed number of generations once; every kernel reads the
    // generation counter and the stop flag from device memory, so the same
    // graph serves every replay and does nothing once stopped.
    const int steps = 8;
    GAME_HIP(hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeThreadLocal));
    int rc = GAME_OK;
    for (int i = 0; i < steps && rc == GAME_OK; ++i) rc = enqueue_step(h, h->capture_stream);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(h->capture_stream, &g);
    if (rc) {
      if (g) hipGraphDestroy(g);
      return rc;
    }
    if (ec != hipSuccess) return hip_fail(ec, "hipStreamEndCapture");
    const hipError_t ei = hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (ei != hipSuccess) {
      h->graph = nullptr;
      return hip_fail(ei, "hipGraphInstantiate");
    }
    h->graph_steps = steps;
  }
  if (!st.stop) {
    const int64_t evals = (int64_t)h->cfg.max_generations - st.gen + 1;
    const int64_t launches = evals <= 0 ? 1 : (evals + h->graph_steps - 1) / h->graph_steps;
    for (int64_t i = 0; i < launches; ++i) GAME_HIP(hipGraphLaunch(h->graph, h->stream));
  }
  GAME_HIP(hipMemcpyAsync(&st, h->state, sizeof st, hipMemcpyDeviceToHost, h->stream));
  GAME_HIP(hipStreamSynchronize(h->stream));
  if (gens_done) *gens_done = st.gen;
  if (best_err) *best_err = st.best_err;
  if (best_genes && st.best >= 0) {
    const float* src = h->pop[st.gen & 1] + (int64_t)st.best * h->K;
    GAME_HIP(hipMemcpyAsync(best_genes, src, sizeof(float) * h->K, hipMemcpyDeviceToHost,
                            h->stream));
    GAME_HIP(hipStreamSynchronize(h->stream));
  }
  return GAME_OK;
}

int game_get_population(game_t h, float* genes, float* fitness) {
  if (!h) return fail(GAME_EINVAL, "handle is NULL");
  if (!genes) return fail(GAME_EINVAL, "genes is NULL");
  const int64_t n = (int64_t)h->cfg.population * h->K;
  hipLaunchKernelGGL(copy_current_kernel, dim3((unsigned)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024)),
                     dim3(256), 0, h->stream, h->state, h->pop[0], h->pop[1], n, genes);
  GAME_HIP(hipGetLastError());
  if (fitness)
    GAME_HIP(hipMemcpyAsync(fitness, h->fit32, sizeof(float) * h->cfg.population,
                            hipMemcpyDeviceToDevice, h->stream));
  return GAME_OK;
}

int game_set_population(game_t h, const float* genes, int32_t generation) {
  if (!h) return fail(GAME_EINVAL, "handle is NULL");
  if (!genes) return fail(GAME_EINVAL, "genes is NULL");
  if (generation < 0) return fail(GAME_EINVAL, "generation < 0");
  GAME_HIP(hipMemcpyAsync(h->pop[generation & 1], genes,
                          sizeof(float) * h->cfg.population * h->K, hipMemcpyDeviceToDevice,
                          h->stream));
  GAME_HIP(launch_set_state(h->state, generation, h->cfg.max_generations, h->cfg.target, 1,
                            h->stream));
  h->initialized = true;
  return GAME_OK;
}

int game_get_state(game_t h, int32_t* generation, int32_t* stopped, int32_t* best_index,
                   double* best_error) {
  if (!h) return fail(GAME_EINVAL, "handle is NULL");
  RunState st{};
  GAME_HIP(hipMemcpyAsync(&st, h->state, sizeof st, hipMemcpyDeviceToHost, h->stream));
  GAME_HIP(hipStreamSynchronize(h->stream));
  if (generation) *generation = st.gen;
  if (stopped) *stopped = st.stop;
  if (best_index) *best_index = st.best;
  if (best_error) *best_error = st.best_err;
  return GAME_OK;
}

int game_rank(const float* fitness, int32_t n, int32_t* order, void* stream) {
  if (!fitness || !order) return fail(GAME_EINVAL, "NULL argument");
  if (n < 1 || n > kMaxPopulation) return fail(GAME_EINVAL, "n %d not in 1..%d", n, kMaxPopulation);
  GAME_HIP(launch_rank(fitness, n, order, (hipStream_t)stream));
  return GAME_OK;
}

size_t game_ga_workspace_size(const game_config* c) {
  if (!c) {
    fail(GAME_EINVAL, "config is NULL");
    return 0;
  }
  if (c->population < 2 || c->population > kMaxPopulation) {
    fail(GAME_EINVAL, "population %d not in 2..%d", c->population, kMaxPopulation);
    return 0;
  }
  return align_up((size_t)c->population * sizeof(int32_t));
}

int game_ga_next(const game_config* c, int32_t K, const float* pop, const float* fitness,
                 int32_t generation, float* out, void* ws, size_t ws_bytes, void* stream) {
  int rc = check_config(c, 1);
  if (rc) return rc;
  if (K < 2 || K > kMaxGenes) return fail(GAME_EINVAL, "n_genes %d not in 2..%d", K, kMaxGenes);
  if (!pop || !fitness || !out) return fail(GAME_EINVAL, "NULL argument");
  if (generation < 1) return fail(GAME_EINVAL, "generation %d < 1", generation);
  const size_t need = game_ga_workspace_size(c);
  if (!ws || !aligned(ws, kAlign) || ws_bytes < need)
    return fail(GAME_EWORKSPACE, "workspace must be 256-byte aligned with %zu bytes", need);
  const size_t bytes = (size_t)c->population * K * sizeof(float);
  if ((const char*)out < (const char*)pop + bytes && (const char*)pop < (const char*)out + bytes)
    return fail(GAME_EINVAL, "out overlaps pop");
  hipStream_t s = (hipStream_t)stream;
  int32_t* order = (int32_t*)ws;
  GAME_HIP(launch_rank(fitness, c->population, order, s));
  GAArgs ga = ga_args(c, K);
  ga.pop_a = pop;
  ga.out_a = out;
  ga.fitness = fitness;
  ga.order = order;
  ga.generation = generation;
  GAME_HIP(launch_ga_next(ga, s));
  return GAME_OK;
}

int game_init_genes(const game_config* c, int32_t K, float* out, void* stream) {
  if (!c || !out) return fail(GAME_EINVAL, "NULL argument");
  if (c->population < 1 || c->population > kMaxPopulation)
    return fail(GAME_EINVAL, "population %d not in 1..%d", c->population, kMaxPopulation);
  if (K < 1 || K > kMaxGenes) return fail(GAME_EINVAL, "n_genes %d not in 1..%d", K, kMaxGenes);
  if (c->init_mode < 0 || c->init_mode > 2) return fail(GAME_EINVAL, "init_mode not in 0..2");
  GAME_HIP(launch_init_genes(c->seed, c->init_mode, c->population, K, out, (hipStream_t)stream));
  return GAME_OK;
}

const char* game_last_error(void) { return g_error.c_str(); }

}  // extern "C"
