// Host runtime of libgame: configuration checks, workspace carving, kernel
// launches on the caller's stream, and the graph-captured training loop.
// The library allocates no device memory: every buffer comes from the
// caller's workspace.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

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
  if (c->tournament_k < 1 || c->tournament_k > c->population)
    return fail(GAME_EINVAL, "tournament_k %d not in 1..population (%d)", c->tournament_k,
                c->population);
  if (c->elitism < 0 || c->elitism >= c->population)
    return fail(GAME_EINVAL, "elitism %d not in 0..population-1", c->elitism);
  if (c->elite_mode != 0 && c->elite_mode != 1)
    return fail(GAME_EINVAL, "elite_mode %d not 0 or 1", c->elite_mode);
  if (c->init_mode < 0 || c->init_mode > 2)
    return fail(GAME_EINVAL, "init_mode %d not in 0..2", c->init_mode);
  if (c->error_fn < 0 || c->error_fn > 3)
    return fail(GAME_EINVAL, "error_fn %d not in 0..3", c->error_fn);
  if (c->precision != GAME_FP32 && c->precision != GAME_BF16)
    return fail(GAME_EINVAL, "precision %d not 0 (FP32) or 1 (BF16)", c->precision);
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
  if (c->selection < 0 || c->selection > 2)
    return fail(GAME_EINVAL, "selection %d not in 0..2", c->selection);
  if (n_features < 1) return fail(GAME_EINVAL, "n_features %d < 1", n_features);
  if (genes_of(c, n_features) > kMaxGenes)
    return fail(GAME_EINVAL, "B*N*d+1 = %lld genes exceeds %d", (long long)genes_of(c, n_features),
                kMaxGenes);
  return GAME_OK;
}

struct Layout {
  size_t state, pop0, pop1, fit32, fit64, order, cum, partial, rescore, cs, total;
};

// The trig expansion's (cos x, sin x) table is kept for float32 runs (the
// BF16 kernel evaluates them itself).
bool keeps_trig_table(const game_config* c) {
  return c->basis == GAME_TRIG && c->precision == GAME_FP32;
}

Layout layout(const game_config* c, int64_t n_patterns, int32_t n_features) {
  const size_t P = (size_t)c->population;
  const size_t K = (size_t)genes_of(c, n_features);
  const size_t Ppad = (P + kMaxTileCols - 1) / kMaxTileCols * kMaxTileCols;
  Layout L{};
  size_t off = 0;
  L.state = off; off += align_up(sizeof(RunState));
  L.pop0 = off; off += align_up(P * K * sizeof(float));
  L.pop1 = off; off += align_up(P * K * sizeof(float));
  L.fit32 = off; off += align_up(P * sizeof(float));
  L.fit64 = off; off += align_up(P * sizeof(double));
  L.order = off; off += align_up(P * sizeof(int32_t));
  L.cum = off; off += align_up(P * sizeof(double));
  L.partial = off;
  off += align_up(std::max(Ppad * kMaxSplits, (size_t)kSplitCapacity) * sizeof(double));
  L.rescore = off; off += align_up(64 * sizeof(double));
  L.cs = off;
  if (keeps_trig_table(c)) off += align_up((size_t)n_patterns * n_features * 2 * sizeof(float));
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
  double* cum;              // roulette wheel of the current generation
  double* partial;
  double* rescore;          // float64 error of the last re-scored elite
  const float* cs;          // (cos x, sin x) of the data set (trig, float32), or null
  bool initialized;
  hipGraphExec_t graph;
  int graph_steps;
  game_surrogate_ctx* sur;  // attached fitness surrogate (screening), or null
  RunState* host_state;     // two pinned host slots for the stop checks of game_run
  hipEvent_t chunk_done[2];
};

struct game_surrogate_ctx {
  game_surrogate_config cfg;
  int32_t n_in;
  int32_t H;
  int32_t max_batch;
  int64_t n_params;
  hipStream_t stream;
  float* params;
  float* grads;
  float* m;
  float* v;
  SurrogateState* st;
  // training minibatch
  float *Xb, *tb, *Z1, *H1, *Z2, *H2, *y, *dy, *dZ2, *dZ1;
  // predictions over up to max_batch rows
  float *H1c, *H2c, *yc;
  // archive of exact evaluations
  float *arch_genes, *arch_target;
  // input statistics (per gene: mean, inverse standard deviation) and the
  // standardised copies of the candidates and of the audit sample
  float *mu, *inv, *cand_x, *audit_x;
  double* gpart;
  // screening
  float* cand;
  int32_t* rank;
  uint64_t* sorted;
  float *audit_genes, *audit_pred, *audit_exact, *H1a, *H2a;
  // split-K partial products of the weight gradients
  float* kpart;              // [k ranges][n_params] weight-gradient ranges
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
  a.degree = h->cfg.degree;
  a.basis = h->cfg.basis;
  a.cs = X == h->X && NP == h->NP ? h->cs : nullptr;
  if (h->cfg.precision == GAME_BF16) plan_fitness_bf16(a, h->cfg.degree, h->cfg.basis);
  else plan_fitness(a, h->cfg.degree, h->cfg.basis, true);
  return a;
}

hipError_t launch_fitness(const game_ctx* h, const FitArgs& a, hipStream_t s) {
  if (h->cfg.precision == GAME_BF16) return launch_fitness_bf16(a, h->cfg.basis, h->cfg.degree, s);
  return launch_fitness_f32(a, h->cfg.basis, h->cfg.degree, s);
}

// Float64 error of n chromosomes over (X, t); partials use the workspace.
hipError_t rescore64(const game_ctx* h, const float* X, const float* t, int64_t NP,
                     const float* genes, int32_t n, double* out, hipStream_t s) {
  Rescore64Args r{};
  r.X = X;
  r.t = t;
  r.genes = genes;
  r.partial = h->partial;
  r.NP = NP;
  r.N = h->N;
  r.K = h->K;
  r.n = n;
  int64_t blocks = (NP + 255) / 256;
  const int64_t cap = (int64_t)kMaxSplits * kMaxTileCols / (n < 1 ? 1 : n);
  if (blocks > 256) blocks = 256;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  r.blocks = (int32_t)blocks;
  r.error_fn = h->cfg.error_fn;
  r.R = h->cfg.tmse_R;
  return launch_rescore64(r, h->cfg.basis, h->cfg.degree, out, s);
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
  g.selection = c->selection;
  return g;
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

// ----------------------------------------------------------- surrogate
struct SurLayout {
  size_t st, params, grads, m, v, Xb, tb, Z1, H1, Z2, H2, y, dy, dZ2, dZ1, H1c, H2c, yc, ag, at,
      cand, rank, sorted, aug, aup, aue, H1a, H2a, kpart, mu, inv, candx, audx, gpart, total;
  int64_t n_params;
};

SurLayout sur_layout(const game_surrogate_config* c, int32_t n_in, int32_t max_batch) {
  SurLayout L{};
  const size_t H = c->hidden, B = c->minibatch, C = max_batch, A = c->audit;
  L.n_params = (int64_t)H * n_in + H + (int64_t)H * H + H + H + 1;
  const size_t P = (size_t)L.n_params * sizeof(float);
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off += align_up(bytes); return o; };
  L.st = take(sizeof(SurrogateState));
  L.params = take(P);
  L.grads = take(P);
  L.m = take(P);
  L.v = take(P);
  L.Xb = take(B * n_in * 4);
  L.tb = take(B * 4);
  L.Z1 = take(B * H * 4);
  L.H1 = take(B * H * 4);
  L.Z2 = take(B * H * 4);
  L.H2 = take(B * H * 4);
  L.y = take(B * 4);
  L.dy = take(B * 4);
  L.dZ2 = take(B * H * 4);
  L.dZ1 = take(B * H * 4);
  L.H1c = take(C * H * 4);
  L.H2c = take(C * H * 4);
  L.yc = take(C * 4);
  L.ag = take((size_t)c->archive * n_in * 4);
  L.at = take((size_t)c->archive * 4);
  L.cand = take(C * n_in * 4);
  L.rank = take(C * 4);
  L.sorted = take((size_t)sort_chunks((int64_t)C) * kSortChunk * 8);
  L.aug = take(A * n_in * 4);
  L.aup = take(A * 4);
  L.aue = take(A * 4);
  L.H1a = take(A * H * 4);
  L.H2a = take(A * H * 4);
  L.kpart = take((size_t)gemm_k_split((int)B) * P);
  L.mu = take((size_t)n_in * 4);
  L.inv = take((size_t)n_in * 4);
  L.candx = take(C * n_in * 4);
  L.audx = take(A * n_in * 4);
  L.gpart = take((size_t)2 * kMomentBlocks * n_in * 8);
  L.total = off;
  return L;
}

int check_surrogate(const game_surrogate_config* c, int32_t n_in, int32_t max_batch) {
  if (!c) return fail(GAME_EINVAL, "surrogate config is NULL");
  if (c->hidden < 1 || c->hidden > 4096) return fail(GAME_EINVAL, "hidden not in 1..4096");
  if (c->archive < 1) return fail(GAME_EINVAL, "archive < 1");
  if (c->minibatch < 1 || c->minibatch > (1 << 20)) return fail(GAME_EINVAL, "minibatch out of range");
  if (c->train_steps < 0 || c->train_steps > 1024) return fail(GAME_EINVAL, "train_steps out of range");
  if (!(c->lr >= 0.f)) return fail(GAME_EINVAL, "lr < 0");
  if (c->oversample < 1 || c->oversample > 64) return fail(GAME_EINVAL, "oversample not in 1..64");
  if (c->audit < 2 || c->audit > 1024) return fail(GAME_EINVAL, "audit not in 2..1024");
  if (n_in < 1 || n_in > kMaxGenes) return fail(GAME_EINVAL, "n_genes out of range");
  if (max_batch < 1) return fail(GAME_EINVAL, "max_batch < 1");
  return GAME_OK;
}

GemmArgs gemm(const float* A, int64_t lda_m, int64_t lda_k, const float* B, int64_t ldb_n,
              int64_t ldb_k, float* C, int64_t ldc, int M, int N, int K, const float* bias, int act,
              float* Z, const float* aux, int64_t ld_aux, const int32_t* skip) {
  GemmArgs g{};
  g.A = A; g.lda_m = lda_m; g.lda_k = lda_k;
  g.B = B; g.ldb_n = ldb_n; g.ldb_k = ldb_k;
  g.C = C; g.ldc = ldc; g.M = M; g.N = N; g.K = K;
  g.bias = bias; g.act = act; g.Z = Z; g.aux = aux; g.ld_aux = ld_aux; g.skip = skip;
  return g;
}

struct SurParams {
  float *W1, *b1, *W2, *b2, *w3, *b3;
};

SurParams split_params(const game_surrogate_ctx* s, float* base) {
  const int64_t H = s->H, n = s->n_in;
  SurParams p{};
  p.W1 = base;
  p.b1 = p.W1 + H * n;
  p.W2 = p.b1 + H;
  p.b2 = p.W2 + H * H;
  p.w3 = p.b2 + H;
  p.b3 = p.w3 + H;
  return p;
}

// Forward over n rows of X [n x n_in]; stores Z1/Z2 when given (training).
// Forward pass over n rows of X; with t set (training) the output layer
// also writes dy and dZ2 for the loss mean((y - t)^2).
int sur_forward(game_surrogate_ctx* s, const float* X, int n, float* Z1, float* H1, float* Z2,
                float* H2, float* y, const int32_t* skip, hipStream_t st,
                const float* t = nullptr, int32_t* step = nullptr) {
  const bool bf16 = !s->cfg.fp32_operands;
  const SurParams p = split_params(s, s->params);
  const int H = s->H, ni = s->n_in;
  GAME_HIP(launch_gemm(gemm(X, ni, 1, p.W1, ni, 1, H1, H, n, H, ni, p.b1, 1, Z1, nullptr, 0, skip),
                       bf16, st));
  GAME_HIP(launch_gemm(gemm(H1, H, 1, p.W2, H, 1, H2, H, n, H, H, p.b2, 1, Z2, nullptr, 0, skip),
                       bf16, st));
  GAME_HIP(launch_out_layer(H2, p.w3, p.b3, n, H, y, t, Z2, t ? s->dy : nullptr,
                            t ? s->dZ2 : nullptr, step, skip, st));
  return GAME_OK;
}

// Gradients of mean((y - t)^2) over the n rows in s->Xb / s->tb, as *ks
// ranges in s->kpart ([range][n_params], parameter order; the gradient is
// their sum in range order); for_adam: this is a training step (advances
// the step count).
int sur_gradients(game_surrogate_ctx* s, int n, const int32_t* skip, hipStream_t st,
                  bool for_adam, int* ks_out) {
  const bool bf16 = !s->cfg.fp32_operands;
  const int H = s->H, ni = s->n_in;
  int rc = sur_forward(s, s->Xb, n, s->Z1, s->H1, s->Z2, s->H2, s->y, skip, st, s->tb,
                       for_adam ? &s->st->step : nullptr);
  if (rc) return rc;
  const SurParams p = split_params(s, s->params);
  const SurParams gp = split_params(s, s->kpart);
  // Weight gradients sum over the n minibatch rows in ks ranges (n <=
  // cfg.minibatch, for which kpart is sized).  Each bias gradient is the
  // row sum of the product's A operand.
  const int ks = gemm_k_split(n);
  *ks_out = ks;
  auto wgrad = [&](GemmArgs g, float* bias_grad) {
    g.part = g.C;
    g.rowsum_part = bias_grad;
    g.part_ld = s->n_params;
    g.k_split = ks;
    return g;
  };
  // One launch: dw3 = dy^T H2 and db3 = sum dy; dW2 = dZ2^T H1 and db2 =
  // column sums of dZ2; dZ1 = (dZ2 W2) * gelu'(Z1).
  const GemmArgs prods[3] = {
      wgrad(gemm(s->dy, 0, 1, s->H2, 1, H, gp.w3, H, 1, H, n, nullptr, 0, nullptr, nullptr, 0,
                 skip), gp.b3),
      wgrad(gemm(s->dZ2, 1, H, s->H1, 1, H, gp.W2, H, H, H, n, nullptr, 0, nullptr, nullptr, 0,
                 skip), gp.b2),
      gemm(s->dZ2, H, 1, p.W2, 1, H, s->dZ1, H, n, H, H, nullptr, 2, nullptr, s->Z1, H, skip)};
  GAME_HIP(launch_gemm_multi(prods, 3, bf16, st));
  // dW1 = dZ1^T X, db1 = column sums of dZ1
  GAME_HIP(launch_gemm(wgrad(gemm(s->dZ1, 1, H, s->Xb, 1, ni, gp.W1, ni, H, ni, n, nullptr, 0,
                                  nullptr, nullptr, 0, skip), gp.b1),
                       bf16, st));
  return GAME_OK;
}

// Screened generation tail (after the evaluation of the current population):
// archive it, train, generate oversampled offspring, score them with the
// network, audit a random sample exactly, and fill the next population with
// the best-predicted offspring (or the plain offspring when the audit's rank
// correlation is too low).
int enqueue_screening(game_ctx* h, hipStream_t s) {
  game_surrogate_ctx* sr = h->sur;
  const game_surrogate_config& c = sr->cfg;
  const int32_t* stop = &h->state->stop;
  const int P = h->cfg.population, E = h->cfg.elitism, K = h->K;
  ArchiveArgs aa{};
  aa.run = h->state;
  aa.pop0 = h->pop[0];
  aa.pop1 = h->pop[1];
  aa.fit64 = h->fit64;
  aa.P = P;
  aa.K = K;
  aa.genes = sr->arch_genes;
  aa.target = sr->arch_target;
  aa.capacity = c.archive;
  aa.st = sr->st;
  GAME_HIP(launch_archive_append(aa, s));
  GAME_HIP(launch_archive_stats(sr->arch_target, sr->st, h->state, P, c.archive, s));
  GAME_HIP(launch_gene_stats(sr->arch_genes, K, c.archive, sr->st, h->state, sr->gpart, sr->mu,
                             sr->inv, s));
  // Each Adam update shares its launch with the next step's minibatch draw.
  if (c.train_steps > 0)
    GAME_HIP(launch_sample_minibatch(sr->arch_genes, sr->arch_target, K, sr->st, h->state, c.seed,
                                     0, c.minibatch, sr->mu, sr->inv, sr->Xb, sr->tb, s));
  for (int step = 0; step < c.train_steps; ++step) {
    int ks = 1;
    int rc = sur_gradients(sr, c.minibatch, stop, s, true, &ks);
    if (rc) return rc;
    if (step + 1 < c.train_steps)
      GAME_HIP(launch_adam_sample(sr->params, sr->kpart, ks, sr->m, sr->v, sr->n_params, c.lr,
                                  sr->st, stop, sr->arch_genes, sr->arch_target, K, h->state,
                                  c.seed, step + 1, c.minibatch, sr->mu, sr->inv, sr->Xb, sr->tb,
                                  s));
    else
      GAME_HIP(launch_adam(sr->params, sr->kpart, ks, sr->m, sr->v, sr->n_params, c.lr, sr->st,
                           stop, s));
  }
  const int C = c.oversample * (P - E);
  GAArgs ga = ga_args(&h->cfg, K);
  ga.pop_a = h->pop[0];
  ga.pop_b = h->pop[1];
  ga.out_a = h->pop[0];
  ga.out_b = h->pop[1];
  ga.fitness = h->fit32;
  ga.order = h->order;
  ga.gen_ptr = &h->state->gen;
  ga.stop = stop;
  ga.n_slots = E + C;
  ga.children = sr->cand;
  ga.cum = h->cum;
  GAME_HIP(launch_ga_next(ga, s));
  // The audit decides first: the network and the exact fitness score a
  // random sample of the candidates, and only when their rank correlation
  // passes does the network score and rank every candidate.
  GAME_HIP(launch_audit_pick(sr->cand, C, K, h->state, c.seed, c.audit, sr->mu, sr->inv,
                             sr->audit_genes, sr->audit_x, s));
  int rc = sur_forward(sr, sr->audit_x, c.audit, nullptr, sr->H1a, nullptr, sr->H2a,
                       sr->audit_pred, stop, s);
  if (rc) return rc;
  FitArgs fa = fit_args(h, h->X, h->t, h->NP, sr->audit_genes, c.audit);
  fa.stop = stop;
  GAME_HIP(launch_fitness(h, fa, s));
  GAME_HIP(launch_finish(h->partial, fa.ld_partial, c.audit, fa.n_splits, h->NP, h->cfg.error_fn,
                         sr->audit_exact, nullptr, s));
  GAME_HIP(launch_spearman_gate(sr->audit_pred, sr->audit_exact, c.audit, c.rho_min,
                                c.min_archive, h->state, sr->st, s));
  const int32_t* skip = &sr->st->skip;
  GAME_HIP(launch_standardize(sr->cand, C, K, sr->mu, sr->inv, sr->cand_x, skip, s));
  rc = sur_forward(sr, sr->cand_x, C, nullptr, sr->H1c, nullptr, sr->H2c, sr->yc, skip, s);
  if (rc) return rc;
  GAME_HIP(launch_rank_sorted(sr->yc, C, sr->sorted, sr->rank, skip, s));
  GAME_HIP(launch_gather_next(sr->cand, sr->rank, C, K, E, P, h->state, sr->st, h->pop[0],
                              h->pop[1], s));
  return GAME_OK;
}

// The rest of a generation after its stop test: the roulette wheel when
// selecting by roulette, then the genetic step (or, with a surrogate, the
// screened generation tail) building pop[gen & 1] for the advanced counter.
// Every kernel does nothing once the run has stopped.
int enqueue_tail(game_ctx* h, hipStream_t s) {
  if (h->cfg.selection == GAME_ROULETTE)
    GAME_HIP(launch_roulette_cum(h->fit32, h->cfg.population, h->cum, &h->state->stop, s));
  if (h->sur) return enqueue_screening(h, s);
  GAArgs ga = ga_args(&h->cfg, h->K);
  ga.cum = h->cum;
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

// One generation of the loop on stream s: evaluate pop[gen & 1], finish and
// rank, stop test, then build pop[(gen + 1) & 1].
int enqueue_step(game_ctx* h, hipStream_t s) {
  FitArgs fa = fit_args(h, h->X, h->t, h->NP, h->pop[0], h->cfg.population);
  fa.genes_alt = h->pop[1];
  fa.gen_sel = &h->state->gen;
  fa.stop = &h->state->stop;
  fa.stop_seen = &h->state->stop_seen;
  GAME_HIP(launch_fitness(h, fa, s));
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
  GAME_HIP(launch_reduce_fitness(ra, s));
  GAME_HIP(launch_finish_rank(ra, s));
  return enqueue_tail(h, s);
}

__global__ void copy_current_kernel(const RunState* st, const float* pop0, const float* pop1,
                                    int64_t n, float* out) {
  const float* src = (st->gen & 1) ? pop1 : pop0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = src[i];
}

// Queues up to n_chunks chunks of generations (enqueue() queues one) with
// two chunks in flight: after each chunk the n run states are copied to one
// of two pinned host slots and an event is recorded; before queuing chunk i
// the host waits for chunk i - 2's copy and stops queuing once every run had
// stopped by then.  Chunks queued after a stop do nothing (every kernel reads
// the device stop flag), so at most two chunks run idle.
template <class F>
int queue_chunks(hipStream_t s, int64_t n_chunks, const RunState* dev, int n, RunState* slots,
                 hipEvent_t* done, F&& enqueue) {
  for (int64_t i = 0; i < n_chunks; ++i) {
    RunState* slot = slots + (i & 1) * n;
    if (i >= 2) {
      GAME_HIP(hipEventSynchronize(done[i & 1]));
      bool all = true;
      for (int r = 0; r < n && all; ++r) all = slot[r].stop != 0;
      if (all) break;
    }
    const int rc = enqueue();
    if (rc) return rc;
    GAME_HIP(hipMemcpyAsync(slot, dev, sizeof(RunState) * n, hipMemcpyDeviceToHost, s));
    GAME_HIP(hipEventRecord(done[i & 1], s));
  }
  return GAME_OK;
}

// Pinned host slots and events for queue_chunks over n run states.
int create_chunk_sync(int n, RunState** slots, hipEvent_t* done) {
  *slots = nullptr;
  done[0] = done[1] = nullptr;
  GAME_HIP(hipHostMalloc((void**)slots, 2 * sizeof(RunState) * n, hipHostMallocDefault));
  for (int i = 0; i < 2; ++i)
    GAME_HIP(hipEventCreateWithFlags(&done[i], hipEventDisableTiming));
  return GAME_OK;
}

void destroy_chunk_sync(RunState* slots, hipEvent_t* done) {
  for (int i = 0; i < 2; ++i)
    if (done[i]) (void)hipEventDestroy(done[i]);
  if (slots) (void)hipHostFree(slots);
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
  return layout(c, n_patterns, n_features).total;
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
  const Layout L = layout(c, NP, N);
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
  h->cum = (double*)(base + L.cum);
  h->rescore = (double*)(base + L.rescore);
  hipError_t e = hipSuccess;
  if (keeps_trig_table(c)) {
    float* cs = (float*)(base + L.cs);
    e = launch_trig_cs(X, NP, N, cs, h->stream);
    if (e != hipSuccess) {
      delete h;
      return hip_fail(e, "launch_trig_cs");
    }
    h->cs = cs;
  }
  e = hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete h;
    return hip_fail(e, "hipStreamCreateWithFlags");
  }
  rc = create_chunk_sync(1, &h->host_state, h->chunk_done);
  if (rc == GAME_OK) {
    e = launch_set_state(h->state, 0, c->max_generations, c->target, 1, h->stream);
    if (e != hipSuccess) rc = hip_fail(e, "launch_set_state");
  }
  if (rc) {
    destroy_chunk_sync(h->host_state, h->chunk_done);
    (void)hipStreamDestroy(h->capture_stream);
    delete h;
    return rc;
  }
  *out = h;
  return GAME_OK;
}

int game_destroy(game_t h) {
  if (!h) return fail(GAME_EINVAL, "handle is NULL");
  if (h->graph) (void)hipGraphExecDestroy(h->graph);
  if (h->capture_stream) (void)hipStreamDestroy(h->capture_stream);
  destroy_chunk_sync(h->host_state, h->chunk_done);
  delete h;
  return GAME_OK;
}

int game_fitness(game_t h, const float* genes, int32_t n, float* f32, double* f64) {
  if (!h) return fail(GAME_EINVAL, "handle is NULL");
  if (!genes || !f32) return fail(GAME_EINVAL, "genes or fitness is NULL");
  if (n < 1 || n > h->cfg.population)
    return fail(GAME_EINVAL, "n %d not in 1..population (%d)", n, h->cfg.population);
  FitArgs fa = fit_args(h, h->X, h->t, h->NP, genes, n);
  GAME_HIP(launch_fitness(h, fa, h->stream));
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
  GAME_HIP(launch_fitness(h, fa, h->stream));
  GAME_HIP(launch_finish(h->partial, fa.ld_partial, n, fa.n_splits, NP, h->cfg.error_fn, nullptr, err64,
                         h->stream));
  return GAME_OK;
}

int game_rescore64(game_t h, const float* X, const float* t, int64_t NP, const float* genes,
                   int32_t n, double* err64) {
  if (!h) return fail(GAME_EINVAL, "handle is NULL");
  if (!genes || !err64) return fail(GAME_EINVAL, "NULL argument");
  if ((X == nullptr) != (t == nullptr)) return fail(GAME_EINVAL, "X and t must both be set or NULL");
  if (!X) {
    X = h->X;
    t = h->t;
    NP = h->NP;
  }
  if (NP < 1) return fail(GAME_EINVAL, "n_patterns < 1");
  if (n < 1 || n > kMaxTileCols * kMaxSplits)
    return fail(GAME_EINVAL, "n %d not in 1..%d", n, kMaxTileCols * kMaxSplits);
  if (n > h->cfg.population)
    return fail(GAME_EINVAL, "n %d not in 1..population (%d)", n, h->cfg.population);
  GAME_HIP(rescore64(h, X, t, NP, genes, n, err64, h->stream));
  return GAME_OK;
}

namespace {

static int predict_common(game_t h, const float* X, const float* t, int64_t NP, const float* genes,
                          int32_t n, float threshold, float* out, int64_t* counts) {
  if (!h) return fail(GAME_EINVAL, "handle is NULL");
  if (!genes || (!out && !counts)) return fail(GAME_EINVAL, "NULL argument");
  if (counts && ((X == nullptr) != (t == nullptr)))
    return fail(GAME_EINVAL, "X and t must both be set or NULL");
  if (!X) {
    X = h->X;
    t = counts ? h->t : nullptr;
    NP = h->NP;
  }
  if (NP < 1) return fail(GAME_EINVAL, "n_patterns < 1");
  if (n < 1 || n > 65535) return fail(GAME_EINVAL, "n %d not in 1..65535", n);
  if (!(threshold == threshold)) return fail(GAME_EINVAL, "threshold is NaN");
  PredictArgs a{};
  a.X = X;
  a.t = t;
  a.genes = genes;
  a.NP = NP;
  a.N = h->N;
  a.K = h->K;
  a.degree = h->cfg.degree;
  a.n = n;
  a.threshold = threshold;
  a.out = out;
  a.counts = counts;
  GAME_HIP(launch_predict(a, h->cfg.basis, h->stream));
  return GAME_OK;
}

}  // namespace

int game_predict(game_t h, const float* X, int64_t NP, const float* genes, int32_t n,
                 float* out) {
  if (!out) return fail(GAME_EINVAL, "out is NULL");
  return predict_common(h, X, nullptr, NP, genes, n, 0.5f, out, nullptr);
}

int game_classify(game_t h, const float* X, const float* t, int64_t NP, const float* genes,
                  int32_t n, float threshold, int64_t* counts) {
  if (!counts) return fail(GAME_EINVAL, "counts is NULL");
  return predict_common(h, X, t, NP, genes, n, threshold, nullptr, counts);
}

int game_trig_sums(const float* X, int64_t NP, int32_t N, int32_t degree, float* Z,
                   void* stream) {
  if (!X || !Z) return fail(GAME_EINVAL, "NULL argument");
  if (NP < 1 || N < 1) return fail(GAME_EINVAL, "n_patterns and n_features must be >= 1");
  if (degree < 1 || degree > kMaxDegree)
    return fail(GAME_EINVAL, "degree %d not in 1..%d", degree, kMaxDegree);
  if ((NP + 255) / 256 > (int64_t)INT32_MAX) return fail(GAME_EINVAL, "n_patterns too large");
  GAME_HIP(launch_trig_sums(X, NP, N, degree, Z, (hipStream_t)stream));
  return GAME_OK;
}

int game_merit(const int64_t* c, double* m) {
  if (!c || !m) return fail(GAME_EINVAL, "NULL argument");
  const double tp = (double)c[0], fp = (double)c[1], tn = (double)c[2], fn = (double)c[3];
  const double n = tp + fp + tn + fn;
  m[0] = n > 0 ? (tp + tn) / n : NAN;
  m[1] = tp + fn > 0 ? tp / (tp + fn) : NAN;
  m[2] = fp + tn > 0 ? fp / (fp + tn) : NAN;
  m[3] = tp + fp > 0 ? fp / (tp + fp) : NAN;
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
  RunState st{};
  GAME_HIP(hipMemcpyAsync(&st, h->state, sizeof st, hipMemcpyDeviceToHost, h->stream));
  GAME_HIP(hipStreamSynchronize(h->stream));
  // A run stopped on its last evaluation continues from it when that
  // evaluation meets neither new criterion: the stop test's other branch
  // (the counter advances), then the rest of that generation, exactly as
  // one uninterrupted run would have gone on.
  const bool resume = st.stop && st.evaluated == st.gen &&
                      !(st.best_err <= h->cfg.target || st.gen >= h->cfg.max_generations);
  GAME_HIP(launch_set_state(h->state, 0, h->cfg.max_generations, h->cfg.target, resume ? 2 : 0,
                            h->stream));
  if (resume) {
    const int rc = enqueue_tail(h, h->stream);
    if (rc) return rc;
    st.stop = 0;
    st.gen += 1;
  }
  // Evaluations left (at least one: a run past its limit evaluates once and
  // stops).
  const int64_t evals = std::max<int64_t>(1, (int64_t)h->cfg.max_generations - st.gen + 1);
  if (h->sur && !st.stop) {
    // A screened generation is a few hundred short launches; the stream runs
    // them back to back faster than a graph replays them, so generations
    // are queued directly, 8 per chunk.
    int64_t left = evals;
    const int rc = queue_chunks(h->stream, (evals + 7) / 8, h->state, 1, h->host_state,
                                h->chunk_done, [&]() {
                                  for (int i = 0; i < 8 && left > 0; ++i, --left) {
                                    const int r = enqueue_step(h, h->stream);
                                    if (r) return r;
                                  }
                                  return (int)GAME_OK;
                                });
    if (rc) return rc;
  } else if (!st.stop) {
    if (!h->graph) {
      // Capture a fixed number of generations once; every kernel reads the
      // generation counter and the stop flag from device memory, so the
      // same graph serves every replay and does nothing once stopped.
      const int steps = 8;
      GAME_HIP(hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeThreadLocal));
      int rc = GAME_OK;
      for (int i = 0; i < steps && rc == GAME_OK; ++i) rc = enqueue_step(h, h->capture_stream);
      hipGraph_t g = nullptr;
      const hipError_t ec = hipStreamEndCapture(h->capture_stream, &g);
      if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      if (ec != hipSuccess) return hip_fail(ec, "hipStreamEndCapture");
      const hipError_t ei = hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ei != hipSuccess) {
        h->graph = nullptr;
        return hip_fail(ei, "hipGraphInstantiate");
      }
      h->graph_steps = steps;
    }
    // Two replays (16 generations) per chunk.
    const int64_t launches = (evals + h->graph_steps - 1) / h->graph_steps;
    const int rc = queue_chunks(h->stream, (launches + 1) / 2, h->state, 1, h->host_state,
                                h->chunk_done, [&]() {
                                  for (int i = 0; i < 2; ++i) {
                                    const hipError_t e = hipGraphLaunch(h->graph, h->stream);
                                    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
                                  }
                                  return (int)GAME_OK;
                                });
    if (rc) return rc;
  }
  GAME_HIP(hipMemcpyAsync(&st, h->state, sizeof st, hipMemcpyDeviceToHost, h->stream));
  GAME_HIP(hipStreamSynchronize(h->stream));
  if (gens_done) *gens_done = st.gen;
  if (best_err) *best_err = st.best_err;
  if (st.best >= 0 && h->cfg.precision != GAME_FP32) {
    // Reduced-precision run: the elite's reported error is its float64 re-score.
    const float* src = h->pop[st.gen & 1] + (int64_t)st.best * h->K;
    GAME_HIP(rescore64(h, h->X, h->t, h->NP, src, 1, h->rescore, h->stream));
    double v = 0.0;
    GAME_HIP(hipMemcpyAsync(&v, h->rescore, sizeof v, hipMemcpyDeviceToHost, h->stream));
    GAME_HIP(hipStreamSynchronize(h->stream));
    if (best_err) *best_err = v;
  }
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
  return align_up((size_t)c->population * sizeof(int32_t)) +
         align_up((size_t)c->population * sizeof(double));
}

namespace {

// The genetic step after validation: rank order and roulette sums in `ws`
// (game_ga_workspace_size bytes), then the next generation.
static int ga_next_on(const game_config* c, int32_t K, const float* pop, const float* fitness,
               int32_t generation, float* out, void* ws, hipStream_t s) {
  int32_t* order = (int32_t*)ws;
  double* cum = (double*)((char*)ws + align_up((size_t)c->population * sizeof(int32_t)));
  GAME_HIP(launch_rank(fitness, c->population, order, s));
  if (c->selection == GAME_ROULETTE)
    GAME_HIP(launch_roulette_cum(fitness, c->population, cum, nullptr, s));
  GAArgs ga = ga_args(c, K);
  ga.cum = cum;
  ga.pop_a = pop;
  ga.out_a = out;
  ga.fitness = fitness;
  ga.order = order;
  ga.generation = generation;
  GAME_HIP(launch_ga_next(ga, s));
  return GAME_OK;
}

static int check_ga_next(const game_config* c, int32_t K, const float* pop, const float* fitness,
                  int32_t generation, const float* out) {
  int rc = check_config(c, 1);
  if (rc) return rc;
  if (K < 2 || K > kMaxGenes) return fail(GAME_EINVAL, "n_genes %d not in 2..%d", K, kMaxGenes);
  if (!pop || !fitness || !out) return fail(GAME_EINVAL, "NULL argument");
  if (generation < 1) return fail(GAME_EINVAL, "generation %d < 1", generation);
  const size_t bytes = (size_t)c->population * K * sizeof(float);
  if ((const char*)out < (const char*)pop + bytes && (const char*)pop < (const char*)out + bytes)
    return fail(GAME_EINVAL, "out overlaps pop");
  return GAME_OK;
}

}  // namespace

int game_ga_next(const game_config* c, int32_t K, const float* pop, const float* fitness,
                 int32_t generation, float* out, void* ws, size_t ws_bytes, void* stream) {
  int rc = check_ga_next(c, K, pop, fitness, generation, out);
  if (rc) return rc;
  const size_t need = game_ga_workspace_size(c);
  if (!ws || !aligned(ws, kAlign) || ws_bytes < need)
    return fail(GAME_EWORKSPACE, "workspace must be 256-byte aligned with %zu bytes", need);
  return ga_next_on(c, K, pop, fitness, generation, out, ws, (hipStream_t)stream);
}

// ------------------------------------------------ fixed-scratch genetic step
// The scratch of game_ga_next_static: room for the rank order and the
// roulette sums of the largest population, laid out as game_ga_next lays
// out its workspace.  Each device holds its own copy until the process
// ends.  Host code never passes the array's name to a kernel or a copy (on
// the host it is only a stand-in for the symbol): it uses the device
// address hipGetSymbolAddress returns for the current device.
constexpr size_t kStaticScratchBytes =
    ((size_t)kMaxPopulation * sizeof(int32_t) + kAlign - 1) / kAlign * kAlign +
    (size_t)kMaxPopulation * sizeof(double);
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxScratchDevices];  // address of `scratch` on each device, once looked up

// Device address of the current device's scratch, looked up on its first use.
static int current_scratch(void** out) {
  int dev = 0;
  GAME_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxScratchDevices)
    return fail(GAME_EINVAL, "device %d: the fixed scratch serves devices 0..%d", dev,
                kMaxScratchDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    GAME_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(GAME_EHIP, "hipGetSymbolAddress returned NULL for the scratch array");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return GAME_OK;
}

}  // namespace

int game_ga_next_static(const game_config* c, int32_t K, const float* pop, const float* fitness,
                        int32_t generation, float* out, void* stream) {
  int rc = check_ga_next(c, K, pop, fitness, generation, out);
  if (rc) return rc;
  const size_t need = game_ga_workspace_size(c);
  if (need > kStaticScratchBytes)
    return fail(GAME_EINVAL, "population %d needs %zu scratch bytes; the fixed scratch holds %zu",
                c->population, need, kStaticScratchBytes);
  void* ws = nullptr;
  rc = current_scratch(&ws);
  if (rc) return rc;
  return ga_next_on(c, K, pop, fitness, generation, out, ws, (hipStream_t)stream);
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

// ---------------------------------------------------------------- surrogate
int game_surrogate_config_default(game_surrogate_config* c) {
  if (!c) return fail(GAME_EINVAL, "config is NULL");
  memset(c, 0, sizeof *c);
  c->hidden = 256;
  c->fp32_operands = 0;
  // Tuned on the 1M x 32, degree-8 problem with population 4,096 for the
  // time to reach a target error, with the inputs standardised per gene: a
  // window of the last four generations, 48 Adam steps at 2e-3 per
  // generation (the audit's rank correlation above 0.8 from the fifth
  // generation on), 256 audited children (standard error of the
  // correlation about 0.02).
  c->archive = 16384;
  c->minibatch = 1024;
  c->train_steps = 48;
  c->lr = 2e-3f;
  c->oversample = 8;
  c->audit = 256;
  c->rho_min = 0.8f;
  c->min_archive = 4096;
  c->seed = 0;
  return GAME_OK;
}

size_t game_surrogate_workspace_size(const game_surrogate_config* c, int32_t n_genes,
                                     int32_t max_batch) {
  if (check_surrogate(c, n_genes, max_batch)) return 0;
  return sur_layout(c, n_genes, max_batch).total;
}

int game_surrogate_create(const game_surrogate_config* c, int32_t n_genes, int32_t max_batch,
                          void* ws, size_t ws_bytes, void* stream, game_surrogate_t* out) {
  if (!out) return fail(GAME_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = check_surrogate(c, n_genes, max_batch);
  if (rc) return rc;
  if (!ws) return fail(GAME_EWORKSPACE, "workspace is NULL");
  if (!aligned(ws, kAlign)) return fail(GAME_EWORKSPACE, "workspace not 256-byte aligned");
  const SurLayout L = sur_layout(c, n_genes, max_batch);
  if (ws_bytes < L.total)
    return fail(GAME_EWORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
  char* b = (char*)ws;
  game_surrogate_ctx* s = new game_surrogate_ctx{};
  s->cfg = *c;
  s->n_in = n_genes;
  s->H = c->hidden;
  s->max_batch = max_batch;
  s->n_params = L.n_params;
  s->stream = (hipStream_t)stream;
  s->st = (SurrogateState*)(b + L.st);
  s->params = (float*)(b + L.params);
  s->grads = (float*)(b + L.grads);
  s->m = (float*)(b + L.m);
  s->v = (float*)(b + L.v);
  s->Xb = (float*)(b + L.Xb);
  s->tb = (float*)(b + L.tb);
  s->Z1 = (float*)(b + L.Z1);
  s->H1 = (float*)(b + L.H1);
  s->Z2 = (float*)(b + L.Z2);
  s->H2 = (float*)(b + L.H2);
  s->y = (float*)(b + L.y);
  s->dy = (float*)(b + L.dy);
  s->dZ2 = (float*)(b + L.dZ2);
  s->dZ1 = (float*)(b + L.dZ1);
  s->H1c = (float*)(b + L.H1c);
  s->H2c = (float*)(b + L.H2c);
  s->yc = (float*)(b + L.yc);
  s->arch_genes = (float*)(b + L.ag);
  s->arch_target = (float*)(b + L.at);
  s->cand = (float*)(b + L.cand);
  s->rank = (int32_t*)(b + L.rank);
  s->sorted = (uint64_t*)(b + L.sorted);
  s->audit_genes = (float*)(b + L.aug);
  s->audit_pred = (float*)(b + L.aup);
  s->audit_exact = (float*)(b + L.aue);
  s->H1a = (float*)(b + L.H1a);
  s->H2a = (float*)(b + L.H2a);
  s->kpart = (float*)(b + L.kpart);
  s->mu = (float*)(b + L.mu);
  s->inv = (float*)(b + L.inv);
  s->cand_x = (float*)(b + L.candx);
  s->audit_x = (float*)(b + L.audx);
  s->gpart = (double*)(b + L.gpart);
  hipError_t e = launch_fill_zero((float*)s->st, sizeof(SurrogateState) / sizeof(float), s->stream);
  // input statistics start as the identity (mean 0, inverse deviation 1)
  if (e == hipSuccess) e = launch_fill_zero(s->mu, n_genes, s->stream);
  if (e == hipSuccess) e = launch_fill(s->inv, n_genes, 1.f, s->stream);
  if (e == hipSuccess) e = launch_fill_zero(s->m, s->n_params, s->stream);
  if (e == hipSuccess) e = launch_fill_zero(s->v, s->n_params, s->stream);
  if (e == hipSuccess) e = launch_mlp_init(s->params, n_genes, s->H, c->seed, s->stream);
  if (e != hipSuccess) {
    delete s;
    return hip_fail(e, "surrogate init");
  }
  *out = s;
  return GAME_OK;
}

int game_surrogate_destroy(game_surrogate_t s) {
  if (!s) return fail(GAME_EINVAL, "surrogate is NULL");
  delete s;
  return GAME_OK;
}

int64_t game_surrogate_num_params(game_surrogate_t s) {
  if (!s) return fail(GAME_EINVAL, "surrogate is NULL");
  return s->n_params;
}

int game_surrogate_get_input_stats(game_surrogate_t s, float* mean, float* inv_std) {
  if (!s || !mean || !inv_std) return fail(GAME_EINVAL, "NULL argument");
  GAME_HIP(hipMemcpyAsync(mean, s->mu, sizeof(float) * s->n_in, hipMemcpyDeviceToDevice,
                          s->stream));
  GAME_HIP(hipMemcpyAsync(inv_std, s->inv, sizeof(float) * s->n_in, hipMemcpyDeviceToDevice,
                          s->stream));
  return GAME_OK;
}

int game_surrogate_get_params(game_surrogate_t s, float* params) {
  if (!s || !params) return fail(GAME_EINVAL, "NULL argument");
  GAME_HIP(hipMemcpyAsync(params, s->params, sizeof(float) * s->n_params, hipMemcpyDeviceToDevice,
                          s->stream));
  return GAME_OK;
}

int game_surrogate_set_params(game_surrogate_t s, const float* params) {
  if (!s || !params) return fail(GAME_EINVAL, "NULL argument");
  GAME_HIP(hipMemcpyAsync(s->params, params, sizeof(float) * s->n_params, hipMemcpyDeviceToDevice,
                          s->stream));
  return GAME_OK;
}

int game_surrogate_predict(game_surrogate_t s, const float* genes, int32_t n, float* y) {
  if (!s || !genes || !y) return fail(GAME_EINVAL, "NULL argument");
  if (n < 1 || n > s->max_batch) return fail(GAME_EINVAL, "n %d not in 1..%d", n, s->max_batch);
  GAME_HIP(launch_standardize(genes, n, s->n_in, s->mu, s->inv, s->cand_x, nullptr, s->stream));
  int rc = sur_forward(s, s->cand_x, n, nullptr, s->H1c, nullptr, s->H2c, y, nullptr, s->stream);
  return rc;
}

int game_surrogate_gradients(game_surrogate_t s, const float* genes, const float* target, int32_t n,
                             float* grads, float* y) {
  if (!s || !genes || !target || !grads) return fail(GAME_EINVAL, "NULL argument");
  if (n < 1 || n > s->cfg.minibatch)
    return fail(GAME_EINVAL, "n %d not in 1..minibatch (%d)", n, s->cfg.minibatch);
  GAME_HIP(launch_standardize(genes, n, s->n_in, s->mu, s->inv, s->Xb, nullptr, s->stream));
  GAME_HIP(hipMemcpyAsync(s->tb, target, sizeof(float) * n, hipMemcpyDeviceToDevice, s->stream));
  int ks = 1;
  int rc = sur_gradients(s, n, nullptr, s->stream, false, &ks);
  if (rc) return rc;
  GAME_HIP(launch_sum_ranges(s->grads, s->kpart, ks, s->n_params, s->stream));
  GAME_HIP(hipMemcpyAsync(grads, s->grads, sizeof(float) * s->n_params, hipMemcpyDeviceToDevice,
                          s->stream));
  if (y) GAME_HIP(hipMemcpyAsync(y, s->y, sizeof(float) * n, hipMemcpyDeviceToDevice, s->stream));
  return GAME_OK;
}

int game_surrogate_train_step(game_surrogate_t s, const float* genes, const float* target,
                              int32_t n) {
  if (!s || !genes || !target) return fail(GAME_EINVAL, "NULL argument");
  if (n < 1 || n > s->cfg.minibatch)
    return fail(GAME_EINVAL, "n %d not in 1..minibatch (%d)", n, s->cfg.minibatch);
  GAME_HIP(launch_standardize(genes, n, s->n_in, s->mu, s->inv, s->Xb, nullptr, s->stream));
  GAME_HIP(hipMemcpyAsync(s->tb, target, sizeof(float) * n, hipMemcpyDeviceToDevice, s->stream));
  int ks = 1;
  int rc = sur_gradients(s, n, nullptr, s->stream, true, &ks);
  if (rc) return rc;
  GAME_HIP(launch_adam(s->params, s->kpart, ks, s->m, s->v, s->n_params, s->cfg.lr, s->st, nullptr,
                       s->stream));
  return GAME_OK;
}

int game_attach_surrogate(game_t h, game_surrogate_t s) {
  if (!h) return fail(GAME_EINVAL, "handle is NULL");
  if (s) {
    if (s->n_in != h->K)
      return fail(GAME_EINVAL, "surrogate takes %d genes, the run has %d", s->n_in, h->K);
    const int C = s->cfg.oversample * (h->cfg.population - h->cfg.elitism);
    if (C > s->max_batch)
      return fail(GAME_EINVAL, "oversampled offspring (%d) exceed max_batch (%d)", C, s->max_batch);
    if (s->cfg.audit > h->cfg.population)
      return fail(GAME_EINVAL, "audit (%d) exceeds the population", s->cfg.audit);
    if (s->stream != h->stream) return fail(GAME_EINVAL, "surrogate and run use different streams");
  }
  h->sur = s;
  if (h->graph) {
    (void)hipGraphExecDestroy(h->graph);
    h->graph = nullptr;
  }
  return GAME_OK;
}

int game_surrogate_stats(game_surrogate_t s, float* rho, int32_t* use, int32_t* screened,
                         int32_t* archive_count, int32_t* adam_steps) {
  if (!s) return fail(GAME_EINVAL, "surrogate is NULL");
  SurrogateState st{};
  GAME_HIP(hipMemcpyAsync(&st, s->st, sizeof st, hipMemcpyDeviceToHost, s->stream));
  GAME_HIP(hipStreamSynchronize(s->stream));
  if (rho) *rho = st.rho;
  if (use) *use = st.use;
  if (screened) *screened = st.screened;
  if (archive_count) *archive_count = st.count;
  if (adam_steps) *adam_steps = st.step;
  return GAME_OK;
}

// ------------------------------------------------------------------ batches
}  // extern "C"

struct game_batch_ctx {
  int32_t n_runs;
  std::vector<BatchRun> runs;
  std::vector<game_config> cfgs;
  BatchRun* runs_dev;
  BatchItem* items_dev;
  int32_t* counter;
  int32_t* rank_block_run;
  int32_t* ga_wave_run;
  RunState* states;
  int64_t item_capacity;
  int32_t n_items;
  int32_t n_rank_blocks;
  int32_t n_ga_waves;
  int32_t max_pop;
  int32_t grid;
  int32_t tiles_per_item;         // the common value of run_tiles, or 0 when they differ
  std::vector<int32_t> run_tiles; // patterns per item of each run, in 256-row tiles
  int32_t queue_begin[kQueues + 1];
  int32_t max_gen;
  size_t lds;
  hipStream_t stream;
  hipStream_t capture_stream;
  hipGraphExec_t graph;
  int graph_steps;
  bool initialized;
  bool any_roulette;
  RunState* host_states;    // two pinned host slots of n_runs states (game_batch_run)
  hipEvent_t chunk_done[2];
};

namespace {

struct BatchLayout {
  size_t runs, items, counter, rank_map, ga_map, states, total;
  std::vector<size_t> pop0, pop1, fit32, fit64, order, cum, partial, cs;
  int64_t item_capacity;
  int32_t n_rank_blocks, n_ga_waves;
};

int check_run(const game_run_desc& r, int i) {
  const int rc = check_config(&r.cfg, r.n_features);
  if (rc) {
    const std::string msg = g_error;
    return fail(rc, "run %d: %s", i, msg.c_str());
  }
  if (r.cfg.precision != GAME_FP32) return fail(GAME_EINVAL, "run %d: batches run in FP32", i);
  if (r.n_patterns < 1) return fail(GAME_EINVAL, "run %d: n_patterns < 1", i);
  if ((r.n_patterns + kTileRows - 1) / kTileRows > (int64_t)INT32_MAX)
    return fail(GAME_EINVAL, "run %d: n_patterns too large", i);
  return GAME_OK;
}

BatchLayout batch_layout(const game_run_desc* runs, int32_t n) {
  BatchLayout L{};
  int64_t cap = 0;
  int32_t rb = 0, gw = 0;
  for (int i = 0; i < n; ++i) {
    const int P = runs[i].cfg.population;
    cap += (int64_t)((P + kTileCols - 1) / kTileCols) * kMaxSplits;
    rb += (P + kRankPerBlock - 1) / kRankPerBlock;
    gw += runs[i].cfg.elitism + (P - runs[i].cfg.elitism + 1) / 2;
  }
  L.item_capacity = cap;
  L.n_rank_blocks = rb;
  L.n_ga_waves = gw;
  size_t off = 0;
  L.runs = off; off += align_up(sizeof(BatchRun) * n);
  L.items = off; off += align_up(sizeof(BatchItem) * cap);
  L.counter = off; off += align_up(sizeof(int32_t) * kQueues);
  L.rank_map = off; off += align_up(sizeof(int32_t) * rb);
  L.ga_map = off; off += align_up(sizeof(int32_t) * gw);
  L.states = off; off += align_up(sizeof(RunState) * n);
  for (int i = 0; i < n; ++i) {
    const size_t P = runs[i].cfg.population;
    const size_t K = (size_t)genes_of(&runs[i].cfg, runs[i].n_features);
    const size_t Ppad = (P + kTileCols - 1) / kTileCols * kTileCols;
    L.pop0.push_back(off); off += align_up(P * K * sizeof(float));
    L.pop1.push_back(off); off += align_up(P * K * sizeof(float));
    L.fit32.push_back(off); off += align_up(P * sizeof(float));
    L.fit64.push_back(off); off += align_up(P * sizeof(double));
    L.order.push_back(off); off += align_up(P * sizeof(int32_t));
    L.cum.push_back(off); off += align_up(P * sizeof(double));
    L.partial.push_back(off); off += align_up(Ppad * kMaxSplits * sizeof(double));
    L.cs.push_back(off);
    if (runs[i].cfg.basis == GAME_TRIG)
      off += align_up((size_t)runs[i].n_patterns * runs[i].n_features * 2 * sizeof(float));
  }
  L.total = off;
  return L;
}

// Work decomposition: run r's patterns are cut into splits of about
// tiles[r] 256-row tiles; items are (run, chromosome tile, split), heaviest
// first so the queue ends with small items.
int build_items(game_batch_ctx* b, const std::vector<int32_t>& tiles_of_run) {
  // Groups: every chromosome tile of one (run, split), which read the same
  // patterns.  Dealt largest first to the least-loaded of the kXcds queues
  // of the run's expansion family (one fitness launch per family).
  struct Group {
    int32_t run, split;
    int64_t cost;
  };
  std::vector<Group> groups;
  for (int r = 0; r < b->n_runs; ++r) {
    BatchRun& run = b->runs[r];
    const int tiles = tiles_of_run[r];
    int splits = (run.n_tiles + tiles - 1) / tiles;
    if (splits > kMaxSplits) splits = kMaxSplits;
    if (splits < 1) splits = 1;
    run.tiles_per_split = (run.n_tiles + splits - 1) / splits;
    run.n_splits = (run.n_tiles + run.tiles_per_split - 1) / run.tiles_per_split;
    for (int sp = 0; sp < run.n_splits; ++sp) {
      const int64_t rows = std::min(run.tiles_per_split, run.n_tiles - sp * run.tiles_per_split);
      groups.push_back({r, sp, rows * run.Q * run.D * run.n_ctiles});
    }
  }
  std::stable_sort(groups.begin(), groups.end(),
                   [](const Group& x, const Group& y) { return x.cost > y.cost; });
  std::vector<std::vector<int32_t>> dealt(kQueues);
  int64_t load[kQueues] = {};
  for (int32_t g = 0; g < (int32_t)groups.size(); ++g) {
    int64_t* fam = load + b->runs[groups[g].run].basis * kXcds;
    const int q = (int)(std::min_element(fam, fam + kXcds) - load);
    dealt[q].push_back(g);
    load[q] += groups[g].cost;
  }
  std::vector<BatchItem> items;
  for (int q = 0; q < kQueues; ++q) {
    b->queue_begin[q] = (int32_t)items.size();
    for (const int32_t g : dealt[q]) {
      const BatchRun& run = b->runs[groups[g].run];
      const int rows = std::min(run.tiles_per_split,
                                run.n_tiles - groups[g].split * run.tiles_per_split);
      for (int c = 0; c < run.n_ctiles; ++c)
        items.push_back({groups[g].run, c, groups[g].split, rows * run.Q * run.D});
    }
  }
  b->queue_begin[kQueues] = (int32_t)items.size();
  if ((int64_t)items.size() > b->item_capacity) return fail(GAME_EINVAL, "too many items");
  GAME_HIP(hipMemcpyAsync(b->items_dev, items.data(), sizeof(BatchItem) * items.size(),
                          hipMemcpyHostToDevice, b->stream));
  GAME_HIP(hipMemcpyAsync(b->runs_dev, b->runs.data(), sizeof(BatchRun) * b->runs.size(),
                          hipMemcpyHostToDevice, b->stream));
  GAME_HIP(hipStreamSynchronize(b->stream));
  b->n_items = (int32_t)items.size();
  b->run_tiles = tiles_of_run;
  b->tiles_per_item = tiles_of_run.empty() ? 0 : tiles_of_run[0];
  for (const int32_t t : tiles_of_run)
    if (t != b->tiles_per_item) b->tiles_per_item = 0;
  if (b->graph) {
    (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
  }
  return GAME_OK;
}

int build_items(game_batch_ctx* b, int32_t tiles) {
  return build_items(b, std::vector<int32_t>(b->n_runs, tiles));
}

BatchArgs batch_args(const game_batch_ctx* b) {
  BatchArgs a{};
  a.runs = b->runs_dev;
  a.items = b->items_dev;
  a.counter = b->counter;
  a.rank_block_run = b->rank_block_run;
  a.ga_wave_run = b->ga_wave_run;
  a.n_runs = b->n_runs;
  a.n_items = b->n_items;
  a.n_rank_blocks = b->n_rank_blocks;
  a.n_ga_waves = b->n_ga_waves;
  a.max_population = b->max_pop;
  a.grid = b->grid;
  for (int q = 0; q <= kQueues; ++q) a.queue_begin[q] = b->queue_begin[q];
  return a;
}

int enqueue_batch_step(game_batch_ctx* b, hipStream_t s) {
  const BatchArgs a = batch_args(b);
  GAME_HIP(launch_fitness_batch(a, b->lds, s));
  GAME_HIP(launch_reduce_fitness_batch(a, s));
  GAME_HIP(launch_finish_rank_batch(a, s));
  if (b->any_roulette) GAME_HIP(launch_roulette_cum_batch(a, s));
  GAME_HIP(launch_ga_next_batch(a, s));
  return GAME_OK;
}

}  // namespace

extern "C" {

size_t game_batch_workspace_size(const game_run_desc* runs, int32_t n_runs) {
  if (!runs || n_runs < 1) {
    fail(GAME_EINVAL, "no runs");
    return 0;
  }
  for (int i = 0; i < n_runs; ++i)
    if (check_run(runs[i], i)) return 0;
  return batch_layout(runs, n_runs).total;
}

int game_batch_create(const game_run_desc* runs, int32_t n_runs, void* ws, size_t ws_bytes,
                      void* stream, game_batch_t* out) {
  if (!out) return fail(GAME_EINVAL, "out is NULL");
  *out = nullptr;
  if (!runs || n_runs < 1) return fail(GAME_EINVAL, "no runs");
  for (int i = 0; i < n_runs; ++i) {
    const int rc = check_run(runs[i], i);
    if (rc) return rc;
    if (!runs[i].X_dev || !runs[i].t_dev) return fail(GAME_EINVAL, "run %d: X or t is NULL", i);
  }
  if (!ws) return fail(GAME_EWORKSPACE, "workspace is NULL");
  if (!aligned(ws, kAlign)) return fail(GAME_EWORKSPACE, "workspace not 256-byte aligned");
  const BatchLayout L = batch_layout(runs, n_runs);
  if (ws_bytes < L.total)
    return fail(GAME_EWORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
  char* base = (char*)ws;
  game_batch_ctx* b = new game_batch_ctx{};
  b->n_runs = n_runs;
  b->stream = (hipStream_t)stream;
  b->runs_dev = (BatchRun*)(base + L.runs);
  b->items_dev = (BatchItem*)(base + L.items);
  b->counter = (int32_t*)(base + L.counter);
  b->rank_block_run = (int32_t*)(base + L.rank_map);
  b->ga_wave_run = (int32_t*)(base + L.ga_map);
  b->states = (RunState*)(base + L.states);
  b->item_capacity = L.item_capacity;
  b->n_rank_blocks = L.n_rank_blocks;
  b->n_ga_waves = L.n_ga_waves;
  b->grid = 512;
  std::vector<int32_t> rank_map, ga_map;
  size_t lds = 4 * 64 * sizeof(double);
  for (int i = 0; i < n_runs; ++i) {
    const game_config& c = runs[i].cfg;
    b->cfgs.push_back(c);
    FitArgs fa{};
    fa.NP = runs[i].n_patterns;
    fa.N = runs[i].n_features;
    fa.n_chrom = c.population;
    plan_fitness(fa, c.degree, c.basis, false);
    lds = std::max(lds, fitness_lds_bytes(fa, c.degree));
    BatchRun r{};
    r.X = runs[i].X_dev;
    r.t = runs[i].t_dev;
    r.NP = runs[i].n_patterns;
    r.N = runs[i].n_features;
    r.K = (int32_t)genes_of(&c, r.N);
    r.basis = c.basis;
    r.D = c.degree;
    r.U = fa.U;
    r.Q = fa.Q;
    r.pairs_per_chunk = fa.pairs_per_chunk;
    r.n_chunks = fa.n_chunks;
    r.n_ctiles = fa.n_ctiles;
    r.ld_partial = fa.ld_partial;
    r.n_tiles = fa.n_tiles;
    r.error_fn = c.error_fn;
    r.R = c.tmse_R;
    r.pop0 = (float*)(base + L.pop0[i]);
    r.pop1 = (float*)(base + L.pop1[i]);
    r.fit32 = (float*)(base + L.fit32[i]);
    r.fit64 = (double*)(base + L.fit64[i]);
    r.order = (int32_t*)(base + L.order[i]);
    r.partial = (double*)(base + L.partial[i]);
    r.cs = c.basis == GAME_TRIG ? (const float*)(base + L.cs[i]) : nullptr;
    r.state = b->states + i;
    r.P = c.population;
    r.k = c.tournament_k;
    r.E = c.elitism;
    r.elite_mode = c.elite_mode;
    r.thr_cross = coin_threshold(c.p_crossover);
    r.thr_mut = coin_threshold(c.p_mutation);
    r.sigma = c.sigma_mutation;
    r.seed = c.seed;
    r.selection = c.selection;
    r.cum = (double*)(base + L.cum[i]);
    r.rank_block0 = (int32_t)rank_map.size();
    for (int k = 0; k < (c.population + kRankPerBlock - 1) / kRankPerBlock; ++k) rank_map.push_back(i);
    r.ga_wave0 = (int32_t)ga_map.size();
    for (int k = 0; k < c.elitism + (c.population - c.elitism + 1) / 2; ++k) ga_map.push_back(i);
    b->runs.push_back(r);
    b->max_pop = std::max(b->max_pop, c.population);
    if (c.selection == GAME_ROULETTE) b->any_roulette = true;
    b->max_gen = std::max(b->max_gen, c.max_generations);
  }
  b->lds = lds;
  int rc = GAME_OK;
  hipError_t e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking);
  if (e != hipSuccess) rc = hip_fail(e, "hipStreamCreateWithFlags");
  if (!rc) {
    e = hipMemcpyAsync(b->rank_block_run, rank_map.data(), sizeof(int32_t) * rank_map.size(),
                       hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(b->ga_wave_run, ga_map.data(), sizeof(int32_t) * ga_map.size(),
                         hipMemcpyHostToDevice, b->stream);
    if (e != hipSuccess) rc = hip_fail(e, "hipMemcpyAsync");
  }
  // (cos x, sin x) of every pattern and feature of the trigonometric runs,
  // once for the batch's lifetime (the data sets do not change).
  for (int i = 0; i < n_runs && !rc; ++i) {
    const BatchRun& r = b->runs[i];
    if (!r.cs) continue;
    e = launch_trig_cs(r.X, r.NP, r.N, const_cast<float*>(r.cs), b->stream);
    if (e != hipSuccess) rc = hip_fail(e, "launch_trig_cs");
  }
  if (!rc) rc = create_chunk_sync(n_runs, &b->host_states, b->chunk_done);
  if (!rc) rc = build_items(b, 8);
  if (rc) {
    destroy_chunk_sync(b->host_states, b->chunk_done);
    if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    delete b;
    return rc;
  }
  *out = b;
  return GAME_OK;
}

int game_batch_destroy(game_batch_t b) {
  if (!b) return fail(GAME_EINVAL, "batch is NULL");
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
  destroy_chunk_sync(b->host_states, b->chunk_done);
  delete b;
  return GAME_OK;
}

int game_batch_tune(game_batch_t b, int32_t tiles_per_item, int32_t grid) {
  if (!b) return fail(GAME_EINVAL, "batch is NULL");
  if (tiles_per_item < 1 || grid < 1 || grid > 65536)
    return fail(GAME_EINVAL, "tiles_per_item >= 1 and 1 <= grid <= 65536");
  b->grid = grid;
  return build_items(b, tiles_per_item);
}

namespace {

// Average duration (ms) of `reps` fitness launches of the current work list
// after one untimed launch (HIP events on the batch's stream).
int time_batch_fitness(game_batch_ctx* b, int32_t reps, hipEvent_t e0, hipEvent_t e1, float* ms) {
  const BatchArgs a = batch_args(b);
  hipError_t e = launch_batch_reset(a, b->stream);
  if (e == hipSuccess) e = launch_fitness_batch(a, b->lds, b->stream);
  if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
  for (int i = 0; i < reps && e == hipSuccess; ++i) {
    e = launch_batch_reset(a, b->stream);
    if (e == hipSuccess) e = launch_fitness_batch(a, b->lds, b->stream);
  }
  if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  if (e != hipSuccess) return hip_fail(e, "autotune launch");
  *ms = t / reps;
  return GAME_OK;
}

const int kTuneTiles[] = {1, 2, 4, 8, 16, 32, 64, 128};
const int kTuneGrids[] = {256, 512, 1024};

}  // namespace

int game_batch_tune_runs(game_batch_t b, const int32_t* tiles_per_item, int32_t grid) {
  if (!b || !tiles_per_item) return fail(GAME_EINVAL, "NULL argument");
  if (grid < 1 || grid > 65536) return fail(GAME_EINVAL, "grid %d not in 1..65536", grid);
  std::vector<int32_t> t(tiles_per_item, tiles_per_item + b->n_runs);
  for (int r = 0; r < b->n_runs; ++r)
    if (t[r] < 1) return fail(GAME_EINVAL, "run %d: tiles_per_item %d < 1", r, t[r]);
  b->grid = grid;
  return build_items(b, t);
}

int game_batch_get_tuning(game_batch_t b, int32_t* tiles_per_item, int32_t* grid) {
  if (!b || !tiles_per_item) return fail(GAME_EINVAL, "NULL argument");
  std::copy(b->run_tiles.begin(), b->run_tiles.end(), tiles_per_item);
  if (grid) *grid = b->grid;
  return GAME_OK;
}

int game_batch_autotune(game_batch_t b, int32_t reps, int32_t* best_tiles, int32_t* best_grid,
                        float* best_ms, float* times_ms) {
  if (!b) return fail(GAME_EINVAL, "batch is NULL");
  if (reps < 1) return fail(GAME_EINVAL, "reps < 1");
  hipEvent_t e0, e1;
  GAME_HIP(hipEventCreate(&e0));
  GAME_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  int bt = 8, bg = 512, idx = 0;
  int rc = GAME_OK;
  for (int tiles : kTuneTiles) {
    for (int grid : kTuneGrids) {
      b->grid = grid;
      rc = build_items(b, tiles);
      float ms = 0.f;
      if (!rc) rc = time_batch_fitness(b, reps, e0, e1, &ms);
      if (rc) break;
      if (times_ms) times_ms[idx] = ms;
      ++idx;
      if (ms < best) {
        best = ms;
        bt = tiles;
        bg = grid;
      }
    }
    if (rc) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  b->grid = bg;
  rc = build_items(b, bt);
  if (rc) return rc;
  GAME_HIP(launch_batch_reset(batch_args(b), b->stream));
  if (best_tiles) *best_tiles = bt;
  if (best_grid) *best_grid = bg;
  if (best_ms) *best_ms = best;
  return GAME_OK;
}

int game_batch_autotune_buckets(game_batch_t b, int32_t reps, const int32_t* bucket_of_run,
                                int32_t n_buckets, int32_t* tiles_per_bucket, int32_t* grid,
                                float* best_ms) {
  if (!b || !bucket_of_run || !tiles_per_bucket) return fail(GAME_EINVAL, "NULL argument");
  if (reps < 1) return fail(GAME_EINVAL, "reps < 1");
  if (n_buckets < 1 || n_buckets > 64) return fail(GAME_EINVAL, "n_buckets not in 1..64");
  for (int r = 0; r < b->n_runs; ++r)
    if (bucket_of_run[r] < 0 || bucket_of_run[r] >= n_buckets)
      return fail(GAME_EINVAL, "run %d: bucket %d not in 0..%d", r, bucket_of_run[r], n_buckets - 1);
  int32_t t0 = 8, g0 = 512;
  float best = 0.f;
  int rc = game_batch_autotune(b, reps, &t0, &g0, &best, nullptr);
  if (rc) return rc;
  std::vector<int32_t> bt(n_buckets, t0);
  auto runs_tiles = [&](const std::vector<int32_t>& per_bucket) {
    std::vector<int32_t> t(b->n_runs);
    for (int r = 0; r < b->n_runs; ++r) t[r] = per_bucket[bucket_of_run[r]];
    return t;
  };
  hipEvent_t e0, e1;
  GAME_HIP(hipEventCreate(&e0));
  GAME_HIP(hipEventCreate(&e1));
  b->grid = g0;
  rc = build_items(b, runs_tiles(bt));
  if (!rc) rc = time_batch_fitness(b, reps, e0, e1, &best);
  for (int k = 0; k < n_buckets && !rc; ++k) {
    bool used = false;
    for (int r = 0; r < b->n_runs; ++r) used = used || bucket_of_run[r] == k;
    if (!used) continue;
    const int32_t keep = bt[k];
    for (int tiles : kTuneTiles) {
      if (tiles == keep) continue;
      std::vector<int32_t> trial = bt;
      trial[k] = tiles;
      rc = build_items(b, runs_tiles(trial));
      float ms = 0.f;
      if (!rc) rc = time_batch_fitness(b, reps, e0, e1, &ms);
      if (rc) break;
      if (ms < best) {
        best = ms;
        bt = trial;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  rc = build_items(b, runs_tiles(bt));
  if (rc) return rc;
  GAME_HIP(launch_batch_reset(batch_args(b), b->stream));
  std::copy(bt.begin(), bt.end(), tiles_per_bucket);
  if (grid) *grid = g0;
  if (best_ms) *best_ms = best;
  return GAME_OK;
}

int game_batch_init(game_batch_t b) {
  if (!b) return fail(GAME_EINVAL, "batch is NULL");
  for (int r = 0; r < b->n_runs; ++r) {
    const game_config& c = b->cfgs[r];
    GAME_HIP(launch_init_genes(c.seed, c.init_mode, c.population, b->runs[r].K, b->runs[r].pop0,
                               b->stream));
    GAME_HIP(launch_set_state(b->states + r, 0, c.max_generations, c.target, 1, b->stream));
  }
  GAME_HIP(launch_batch_reset(batch_args(b), b->stream));
  b->initialized = true;
  return GAME_OK;
}

int game_batch_step(game_batch_t b) {
  if (!b) return fail(GAME_EINVAL, "batch is NULL");
  if (!b->initialized) return fail(GAME_ESTATE, "batch not initialised");
  return enqueue_batch_step(b, b->stream);
}

int game_batch_evaluate(game_batch_t b) {
  if (!b) return fail(GAME_EINVAL, "batch is NULL");
  if (!b->initialized) return fail(GAME_ESTATE, "batch not initialised");
  const BatchArgs a = batch_args(b);
  GAME_HIP(launch_batch_reset(a, b->stream));
  GAME_HIP(launch_fitness_batch(a, b->lds, b->stream));
  GAME_HIP(launch_reduce_fitness_batch(a, b->stream));
  // the queues are re-armed for the next generation's launch
  GAME_HIP(launch_batch_reset(a, b->stream));
  return GAME_OK;
}

int game_batch_run(game_batch_t b, int32_t* gens_done, double* best_err) {
  if (!b) return fail(GAME_EINVAL, "batch is NULL");
  if (!b->initialized) return fail(GAME_ESTATE, "batch not initialised");
  std::vector<RunState> st(b->n_runs);
  GAME_HIP(hipMemcpyAsync(st.data(), b->states, sizeof(RunState) * b->n_runs,
                          hipMemcpyDeviceToHost, b->stream));
  GAME_HIP(hipStreamSynchronize(b->stream));
  int min_gen = INT32_MAX;
  for (const RunState& x : st)
    if (!x.stop) min_gen = std::min(min_gen, x.gen);
  if (min_gen != INT32_MAX) {
    if (!b->graph) {
      const int steps = 4;
      GAME_HIP(hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal));
      int rc = GAME_OK;
      for (int i = 0; i < steps && rc == GAME_OK; ++i) rc = enqueue_batch_step(b, b->capture_stream);
      hipGraph_t g = nullptr;
      const hipError_t ec = hipStreamEndCapture(b->capture_stream, &g);
      if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      if (ec != hipSuccess) return hip_fail(ec, "hipStreamEndCapture");
      const hipError_t ei = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ei != hipSuccess) {
        b->graph = nullptr;
        return hip_fail(ei, "hipGraphInstantiate");
      }
      b->graph_steps = steps;
    }
    // Two replays (8 generations) per chunk, until every run has stopped.
    const int64_t evals = std::max<int64_t>(1, (int64_t)b->max_gen - min_gen + 1);
    const int64_t launches = (evals + b->graph_steps - 1) / b->graph_steps;
    const int rc = queue_chunks(b->stream, (launches + 1) / 2, b->states, b->n_runs,
                                b->host_states, b->chunk_done, [&]() {
                                  for (int i = 0; i < 2; ++i) {
                                    const hipError_t e = hipGraphLaunch(b->graph, b->stream);
                                    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
                                  }
                                  return (int)GAME_OK;
                                });
    if (rc) return rc;
  }
  GAME_HIP(hipMemcpyAsync(st.data(), b->states, sizeof(RunState) * b->n_runs,
                          hipMemcpyDeviceToHost, b->stream));
  GAME_HIP(hipStreamSynchronize(b->stream));
  for (int r = 0; r < b->n_runs; ++r) {
    if (gens_done) gens_done[r] = st[r].gen;
    if (best_err) best_err[r] = st[r].best_err;
  }
  return GAME_OK;
}

int game_batch_get_population(game_batch_t b, int32_t run, float* genes, float* fitness) {
  if (!b) return fail(GAME_EINVAL, "batch is NULL");
  if (run < 0 || run >= b->n_runs) return fail(GAME_EINVAL, "run %d out of range", run);
  if (!genes) return fail(GAME_EINVAL, "genes is NULL");
  const BatchRun& r = b->runs[run];
  const int64_t n = (int64_t)r.P * r.K;
  hipLaunchKernelGGL(copy_current_kernel,
                     dim3((unsigned)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024)), dim3(256),
                     0, b->stream, b->states + run, r.pop0, r.pop1, n, genes);
  GAME_HIP(hipGetLastError());
  if (fitness)
    GAME_HIP(hipMemcpyAsync(fitness, r.fit32, sizeof(float) * r.P, hipMemcpyDeviceToDevice,
                            b->stream));
  return GAME_OK;
}

int game_batch_num_items(game_batch_t b, int32_t* n_items, int32_t* tiles_per_item, int32_t* grid) {
  if (!b) return fail(GAME_EINVAL, "batch is NULL");
  if (n_items) *n_items = b->n_items;
  if (tiles_per_item) *tiles_per_item = b->tiles_per_item;
  if (grid) *grid = b->grid;
  return GAME_OK;
}

const char* game_last_error(void) { return g_error.c_str(); }

}  // extern "C"
