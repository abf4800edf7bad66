// Internal declarations shared by libgame's translation units (not part of
// the C ABI; see include/game.h for that).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace game {

// Sum over splits of chromosome i's partials, called by all 64 lanes of a
// wave: lane l adds splits l, l+64, ... in order, then a butterfly adds the
// lane sums.  Partner lanes add the same two values (a + b == b + a), so
// every lane ends with the same, scheduling-independent value.
__device__ __forceinline__ double wave_split_sum(const double* partial, int64_t ld, int n_splits,
                                                 int i) {
  double s = 0.0;
  for (int k = (int)(threadIdx.x & 63); k < n_splits; k += 64) s += partial[(int64_t)k * ld + i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  return s;
}

// Error of a split sum: mean over the NP patterns, root for RMSE, NaN -> +inf.
__device__ __forceinline__ double error_from_sum(double s, int64_t NP, int error_fn) {
  double v = s / (double)NP;
  if (error_fn == 1) v = sqrt(v);
  if (isnan(v)) v = INFINITY;
  return v;
}


constexpr int kWave = 64;
constexpr int kMaxDegree = 16;
constexpr int kMaxPopulation = 8192;
constexpr int kMaxGenes = 4097;
constexpr int kMaxSplits = 64;
// A single run's partial sums hold max(Ppad * kMaxSplits, kSplitCapacity)
// doubles, so a launch over few chromosome tiles may cut the patterns into
// more splits (up to kSplitCapacity / ld_partial) and still fill the GPU.
constexpr int kSplitCapacity = 65536;
inline int max_splits(int ld_partial) {
  const int c = kSplitCapacity / (ld_partial < 1 ? 1 : ld_partial);
  return c > kMaxSplits ? c : kMaxSplits;
}

// Fitness tile geometry: a workgroup of 4 waves covers 256 patterns x 64
// chromosomes; each wave 64 patterns (two 32-row MFMA blocks) x 64
// chromosomes (two 32-column MFMA blocks).
constexpr int kTileRows = 256;
constexpr int kTileCols = 64;
constexpr int kFitThreads = 256;
// Largest K kept in LDS at once, in MFMA K-steps per lane half: a
// chromosome tile whose genes fit is staged once; otherwise its genes pass
// through two LDS buffers in chunks of at most kChunkSteps K-steps, the next
// chunk's copy in flight while the current one is used.  kMaxChunkSteps for
// 64-chromosome tiles (two workgroups share a CU's LDS), kMaxWideSteps for
// 128-chromosome ones (128 rows x 319 floats = 159.5 KB of one CU).
constexpr int kMaxChunkSteps = 128;
constexpr int kMaxWideSteps = 159;
constexpr int kChunkSteps = 64;

// Device-side state of a run.  Only the rank kernel writes gen/stop/best.
struct RunState {
  int32_t gen;          // index of the population to be evaluated next
  int32_t stop;         // 1 once a stop criterion held
  int32_t best;         // best index of the last evaluation
  int32_t max_gen;      // stop when gen >= max_gen after an evaluation
  double best_err;      // float64 error of `best`
  double target;        // stop when best_err <= target
  int32_t evaluated;    // generation of the last evaluation, -1 if none
  int32_t stop_seen;    // stop flag as the generation's fitness launch saw it
  int32_t pad[6];
};

// Problem view for the fitness kernels.
struct FitArgs {
  const float* X;           // [NP x N] row-major
  const float* t;           // [NP]
  const float* genes;       // [n_chrom x K] canonical layout
  const float* genes_alt;   // second buffer of a ping-pong pair (or null)
  const int32_t* gen_sel;   // when set, genes_alt is used if (*gen_sel & 1)
  const int32_t* stop;      // when set and nonzero the kernel returns
  int32_t* stop_seen;       // when set, block 0 records *stop here
  double* partial;          // [n_splits x ld_partial] float64 SSE partials
  int64_t NP;
  int32_t N;
  int32_t K;
  int32_t n_chrom;
  int32_t U;                // sub-features B*N
  int32_t Q;                // feature pairs ceil(U/2)
  int32_t pairs_per_chunk;
  int32_t n_chunks;
  int32_t n_ctiles;
  int32_t ld_partial;       // n_ctiles * tile_cols
  int32_t n_splits;
  int32_t tiles_per_split;
  int32_t n_tiles;
  int32_t xcd_remap;
  int32_t error_fn;
  float R;
  int32_t degree;           // d
  int32_t basis;            // expansion family (the kernels take it as a template parameter)
  const float* cs;          // trig only: [NP x N] pairs (cos x, sin x) of X, or null
  int32_t tile_cols;        // chromosomes per FP32 tile: 64, or 128 (genes in one chunk)
};

// Fitness-kernel variant of the trigonometric expansion that reads the
// stored (cos x, sin x) table FitArgs::cs.
constexpr int kTrigTable = 4;

// Grid/chunk planning shared by every float32 fitness launch.  wide allows
// 128-chromosome tiles (single runs); the batched kernel's items are 64
// chromosomes wide.
void plan_fitness(FitArgs& a, int degree, int basis, bool wide);
size_t fitness_lds_bytes(const FitArgs& a, int degree);

hipError_t launch_fitness_f32(const FitArgs& a, int basis, int degree, hipStream_t s);
// BF16 operands, FP32 accumulation: 128-chromosome tiles; in its plan Q
// counts groups of sub-features and pairs_per_chunk the groups per chunk.
void plan_fitness_bf16(FitArgs& a, int degree, int basis);
hipError_t launch_fitness_bf16(const FitArgs& a, int basis, int degree, hipStream_t s);
constexpr int kMaxTileCols = 128;

// Float64 re-score of n chromosomes over a data set.
// Per-pattern cos/sin sums of the shared-gene model: Z [NP x 2d].
// The trigonometric expansion's seeds of a data set, once: cs[2(k N + i)]
// = cos x_ki, cs[2(k N + i) + 1] = sin x_ki (float32 sincosf, the call the
// fitness kernels make when no table is given).
hipError_t launch_trig_cs(const float* X, int64_t NP, int N, float* cs, hipStream_t s);
hipError_t launch_trig_sums(const float* X, int64_t NP, int N, int d, float* Z, hipStream_t s);

// Outputs (counts == nullptr) or classification counts of n chromosomes.
struct PredictArgs {
  const float* X;           // [NP x N]
  const float* t;           // [NP] class labels (classification)
  const float* genes;       // [n x K]
  int64_t NP;
  int32_t N, K, degree, n;
  float threshold;          // predicted class 1 when Out >= threshold
  float* out;               // [n x NP] (prediction)
  int64_t* counts;          // [n x 4]: TP, FP, TN, FN (classification)
};
hipError_t launch_predict(const PredictArgs& a, int basis, hipStream_t s);

struct Rescore64Args {
  const float* X;
  const float* t;
  const float* genes;
  double* partial;          // [blocks x n]
  int64_t NP;
  int32_t N;
  int32_t K;
  int32_t n;
  int32_t blocks;
  int32_t error_fn;
  double R;
};
hipError_t launch_rescore64(const Rescore64Args& a, int basis, int degree, double* out,
                            hipStream_t s);
hipError_t launch_finish(const double* partial, int32_t ld, int32_t n, int32_t n_splits, int64_t NP,
                         int32_t error_fn, float* f32, double* f64, hipStream_t s);
hipError_t launch_init_genes(uint64_t seed, int32_t mode, int32_t P, int32_t K, float* out,
                             hipStream_t s);
hipError_t launch_rank(const float* fit, int32_t n, int32_t* order, hipStream_t s);

struct GAArgs {
  const float* pop_a;       // previous generation (or ping-pong buffer 0)
  const float* pop_b;       // ping-pong buffer 1 (or null)
  float* out_a;             // next generation (or ping-pong buffer 0)
  float* out_b;             // ping-pong buffer 1 (or null)
  const float* fitness;     // [P] float32 of the previous generation
  const int32_t* order;     // [P] rank order of `fitness`
  const int32_t* gen_ptr;   // when set: generation = *gen_ptr, buffers by parity
  const int32_t* stop;
  int32_t generation;       // used when gen_ptr is null
  int32_t P;
  int32_t K;
  int32_t k;
  int32_t E;
  int32_t elite_mode;
  uint64_t thr_cross;
  uint64_t thr_mut;
  float sigma;
  uint64_t seed;
  int32_t n_slots;          // output slots incl. elites; 0 means P
  float* children;          // when set, child slot s goes to row s - E here
  int32_t selection;        // 0 tournament, 1 linear ranking, 2 roulette
  const double* cum;        // roulette: cumulative weights [P]
};
// Roulette wheel of one generation: cum[i] = sum_{j<=i} 1/(f_j + 1e-12).
hipError_t launch_roulette_cum(const float* fit, int32_t P, double* cum, const int32_t* stop,
                               hipStream_t s);
hipError_t launch_ga_next(const GAArgs& a, hipStream_t s);

// Evaluation epilogue of a run: float64 errors, rank, best, stop test.
// Grid: ceil(P / kRankPerBlock) workgroups of kRankThreads.
struct RankArgs {
  const double* partial;
  int32_t ld_partial;
  int32_t n_splits;
  int64_t NP;
  int32_t P;
  int32_t error_fn;
  float* fit32;
  double* fit64;
  int32_t* order;
  RunState* state;
};
hipError_t launch_finish_rank(const RankArgs& a, hipStream_t s);
// fit64/fit32 of every chromosome from the split partials (one wave per
// chromosome, wave_split_sum order); runs before finish_rank.
hipError_t launch_reduce_fitness(const RankArgs& a, hipStream_t s);
constexpr int kRankThreads = 1024;
constexpr int kRankPerBlock = 64;
hipError_t launch_set_state(RunState* st, int32_t gen, int32_t max_gen, double target,
                            int32_t reset, hipStream_t s);

// ---------------------------------------------------------------- batches
// One run of a batch: its data, its fitness plan (float32 kernel geometry),
// its population buffers and its genetic parameters.
struct BatchRun {
  const float* X;
  const float* t;
  const float* cs;          // trigonometric runs: (cos x, sin x) per pattern and feature
  int64_t NP;
  int32_t N;
  int32_t K;
  int32_t basis;
  int32_t D;
  int32_t U;
  int32_t Q;
  int32_t pairs_per_chunk;
  int32_t n_chunks;
  int32_t n_ctiles;
  int32_t ld_partial;
  int32_t n_splits;
  int32_t tiles_per_split;
  int32_t n_tiles;
  int32_t error_fn;
  float R;
  float* pop0;
  float* pop1;
  float* fit32;
  double* fit64;
  int32_t* order;
  double* partial;
  RunState* state;
  int32_t P;
  int32_t k;
  int32_t E;
  int32_t elite_mode;
  uint64_t thr_cross;
  uint64_t thr_mut;
  float sigma;
  uint64_t seed;
  int32_t selection;
  double* cum;              // roulette weights [P]
  int32_t rank_block0;      // first rank workgroup of this run
  int32_t ga_wave0;         // first genetic-step wave of this run
};

// A unit of fitness work: one 64-chromosome tile of one run over one split
// of its patterns.
struct BatchItem {
  int32_t run;
  int32_t ctile;
  int32_t split;
  int32_t cost;             // relative work, for ordering
};

// The batched fitness work list is split by expansion family, one launch per
// family present, and each family's items into one queue per XCD (8 on
// MI355X); workgroup b starts on queue b % 8, the XCD the hardware dispatches
// it to, and takes work from the family's other queues once its own is empty.
constexpr int kXcds = 8;
constexpr int kFamilies = 4;
constexpr int kQueues = kFamilies * kXcds;  // queue f * kXcds + q: family f, XCD q
static_assert(kQueues <= 64, "the queue heads are re-armed by one wave");

struct BatchArgs {
  const BatchRun* runs;
  const BatchItem* items;
  int32_t* counter;         // kQueues queue heads of the fitness launches
  const int32_t* rank_block_run;
  const int32_t* ga_wave_run;
  int32_t n_runs;
  int32_t n_items;
  int32_t n_rank_blocks;
  int32_t n_ga_waves;
  int32_t max_population;
  int32_t grid;             // persistent fitness workgroups
  int32_t queue_begin[kQueues + 1];  // queue q holds items [queue_begin[q], queue_begin[q+1])
};
hipError_t launch_fitness_batch(const BatchArgs& a, size_t lds_bytes, hipStream_t s);
hipError_t launch_finish_rank_batch(const BatchArgs& a, hipStream_t s);
hipError_t launch_reduce_fitness_batch(const BatchArgs& a, hipStream_t s);
hipError_t launch_ga_next_batch(const BatchArgs& a, hipStream_t s);
hipError_t launch_batch_reset(const BatchArgs& a, hipStream_t s);
hipError_t launch_roulette_cum_batch(const BatchArgs& a, hipStream_t s);

// ---------------------------------------------------------------- surrogate
struct GemmArgs {
  const float* A;           // A(m, k) = A[m * lda_m + k * lda_k]
  const float* B;           // B(n, k) = B[n * ldb_n + k * ldb_k]
  float* C;                 // C[m * ldc + n]
  const float* bias;        // [N] or null
  float* Z;                 // pre-activation out (act 1) or null
  const float* aux;         // act 2: C *= gelu'(aux[m * ld_aux + n])
  int64_t lda_m, lda_k, ldb_n, ldb_k, ldc, ld_aux;
  int32_t M, N, K;
  int32_t act;              // 0 none, 1 GELU, 2 times GELU'(aux)
  const int32_t* skip;      // when set and nonzero the launch does nothing
  // Split products (weight gradients over a minibatch).  When part is set,
  // K is cut into k_split ranges of whole 16-value steps and range z writes
  // its raw sum to part[z * part_ld + m * ldc + n] (no bias, no epilogue);
  // with rowsum_part set it also writes sum_k A(m, k) over its range to
  // rowsum_part[z * part_ld + m].  Readers add the ranges in order z = 0, 1, ...
  float* part;
  float* rowsum_part;
  int64_t part_ld;
  int32_t k_split;
};
// Ranges for a split product of length K: at most 512 K values each (one
// load round per wave of the small-product kernel), at most 8 ranges.
inline int gemm_k_split(int K) {
  const int r = (K + 511) / 512;
  return r < 1 ? 1 : (r > 8 ? 8 : r);
}
hipError_t launch_gemm(const GemmArgs& g, bool bf16, hipStream_t s);
// Up to 3 independent minibatch-sized products in one launch.
hipError_t launch_gemm_multi(const GemmArgs* gs, int n, bool bf16, hipStream_t s);
// Output layer (and with t set, its backward); see out_layer_kernel.
hipError_t launch_out_layer(const float* H2, const float* w3, const float* b3, int B, int H,
                            float* y, const float* t, const float* Z2, float* dy, float* dZ2,
                            int32_t* step, const int32_t* skip, hipStream_t s);
hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s);
hipError_t launch_fill(float* p, int64_t n, float value, hipStream_t s);

struct SurrogateState {
  int32_t step;             // Adam steps taken
  int32_t head;             // archive ring position of the next append
  int32_t count;            // archive entries
  float mean, inv_std;      // standardisation of the archive targets
  float rho;                // Spearman correlation of the last audit
  int32_t use;              // 1 when this generation's offspring are screened
  int32_t screened;         // generations screened so far
  int32_t skip;             // 1 when the candidates need no full scoring (stopped or not used)
  int32_t pad[7];
};
// Gradient of parameter i: the sum of the ks split ranges part[z * n + i]
// in order z = 0, 1, ...
__device__ __forceinline__ float sum_ranges(const float* part, int ks, int64_t n, int64_t i) {
  float gi = part[i];
  for (int z = 1; z < ks; ++z) gi += part[(int64_t)z * n + i];
  return gi;
}

// Adam (Kingma & Ba) with bias correction, parameter i, at Adam step `step`
// (1 for the first update).  The moment updates are explicit FMAs, so the
// result does not depend on the translation unit's contraction setting.
__device__ __forceinline__ void adam_update(float* p, const float* part, int ks, float* m, float* v,
                                            int64_t n, float lr, int step, int64_t i) {
  const float c1 = 1.f - powf(0.9f, (float)step);
  const float c2 = 1.f - powf(0.999f, (float)step);
  const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
  const float gi = sum_ranges(part, ks, n, i);
  const float mi = fmaf(beta1, m[i], (1.f - beta1) * gi);
  const float vi = fmaf(beta2, v[i], ((1.f - beta2) * gi) * gi);
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Adam on n parameters whose gradient is the sum of ks ranges
// part[z * n + i], added in order z = 0, 1, ...
hipError_t launch_adam(float* p, const float* part, int ks, float* m, float* v, int64_t n,
                       float lr, SurrogateState* st, const int32_t* skip, hipStream_t s);
// g[i] = sum over z < ks of part[z * n + i], in order.
hipError_t launch_sum_ranges(float* g, const float* part, int ks, int64_t n, hipStream_t s);

// Surrogate kernels built with the Philox draws (stream 3).
hipError_t launch_mlp_init(float* params, int n_in, int hidden, uint64_t seed, hipStream_t s);
struct ArchiveArgs {
  const RunState* run;      // the evaluated generation is run->evaluated
  const float* pop0;
  const float* pop1;
  const double* fit64;
  int32_t P;
  int32_t K;
  float* genes;             // [capacity x K]
  float* target;            // [capacity] log error
  int32_t capacity;
  SurrogateState* st;
};
hipError_t launch_archive_append(const ArchiveArgs& a, hipStream_t s);
hipError_t launch_archive_stats(const float* target, SurrogateState* st, const RunState* run,
                                int P, int capacity, hipStream_t s);
// Network inputs are standardised genes, (g - mu) * inv per gene (two
// float32 roundings); mu and inv come from the archive (launch_gene_stats).
hipError_t launch_sample_minibatch(const float* genes, const float* target, int32_t K,
                                   const SurrogateState* st, const RunState* run, uint64_t seed,
                                   int32_t step, int32_t B, const float* mu, const float* inv,
                                   float* Xb, float* tb, hipStream_t s);
// The Adam update of a training step and the minibatch draw of the next one
// (independent work) in one launch.
hipError_t launch_adam_sample(float* p, const float* part, int ks, float* m, float* v, int64_t n,
                              float lr, SurrogateState* st, const int32_t* skip, const float* genes,
                              const float* target, int32_t K, const RunState* run, uint64_t seed,
                              int32_t next_step, int32_t B, const float* mu, const float* inv,
                              float* Xb, float* tb, hipStream_t s);
// Audit sample: raw genes (for the exact evaluation) and their standardised
// copy (for the network).
hipError_t launch_audit_pick(const float* cand, int32_t C, int32_t K, const RunState* run,
                             uint64_t seed, int32_t A, const float* mu, const float* inv,
                             float* genes, float* x, hipStream_t s);
// Per-gene mean and inverse standard deviation of the archive's rows
// (float64 moments summed in a fixed order, population form, the standard
// deviation floored at kInputStdFloor): part holds 2 * kMomentBlocks * K
// doubles.
constexpr int kMomentBlocks = 256;   // a multiple of kMomentRows (16)
constexpr double kInputStdFloor = 1e-3;
hipError_t launch_gene_stats(const float* genes, int32_t K, int32_t capacity,
                             const SurrogateState* st, const RunState* run, double* part,
                             float* mu, float* inv, hipStream_t s);
// dst[r * K + g] = (src[r * K + g] - mu[g]) * inv[g] for n rows (nothing
// when *skip is set).
hipError_t launch_standardize(const float* src, int32_t n, int32_t K, const float* mu,
                              const float* inv, float* dst, const int32_t* skip, hipStream_t s);
hipError_t launch_spearman_gate(const float* pred, const float* exact, int32_t A, float rho_min,
                                int32_t min_archive, const RunState* run, SurrogateState* st,
                                hipStream_t s);
// Rank by (value, index) of up to ~10^6 values: chunks of kSortChunk keys
// sorted in LDS, then each value's rank summed over binary searches of the
// sorted chunks.  sorted holds sort_chunks(n) * kSortChunk keys.
constexpr int kSortChunk = 8192;
inline int sort_chunks(int64_t n) { return (int)((n + kSortChunk - 1) / kSortChunk); }
hipError_t launch_rank_sorted(const float* v, int32_t n, uint64_t* sorted, int32_t* rank,
                              const int32_t* skip, hipStream_t s);
hipError_t launch_gather_next(const float* cand, const int32_t* rank, int32_t C, int32_t K,
                              int32_t E, int32_t P, const RunState* run, const SurrogateState* st,
                              float* pop0, float* pop1, hipStream_t s);

}  // namespace game
