/*
 * game.h - C ABI of libgame, GAME genetic-algorithm fitness on AMD Instinct
 * MI355X (gfx950).
 *
 * Method: Cavuoti et al., "Astrophysical data mining with GPU. A case study:
 * genetic classification of globular clusters" (GAME).  A chromosome's genes
 * weight a per-feature polynomial expansion of degree d (Eq. 1; Eq. 8 for
 * the trigonometric one), summed over the N features of a pattern plus one
 * bias (Eq. 2); its fitness is the error of those outputs against the
 * targets over all NP patterns (MSE Eq. 4, RMSE Eq. 5, TMSE Eq. 10).  The
 * genetic loop of Sec. 4.1 (generate, evaluate and sort, test the stop
 * criteria, evolve) runs entirely on the device.
 *
 * Conventions shared by every entry point:
 *  - Every function returns GAME_OK (0) or a negative game_status and never
 *    throws; game_last_error() gives a message for the calling thread.
 *  - "_dev" pointers are device memory owned by the caller (the library
 *    never allocates device memory); "_host" pointers are host memory.
 *  - Work is queued on the caller's HIP stream (hipStream_t passed as
 *    void*; NULL is the default stream) and is asynchronous unless a
 *    function says it synchronises.
 *  - Matrices are row-major float32.  X is [n_patterns x n_features], the
 *    targets t are [n_patterns].
 *  - Gene layout (canonical, K = B*N*d + 1 genes): gene 0 is the bias a_0;
 *    gene 1 + i*B*d + b*d + (j-1) multiplies phi_{b,j}(f_i) for feature i
 *    (0-based), block b (B = 2 only for GAME_TRIG: b = 0 cos(jx), b = 1
 *    sin(jx)) and degree j = 1..d.  A population is [P x K] row-major.
 *  - A handle is used by one host thread at a time; calls on one handle
 *    are ordered by its stream.
 */
#ifndef GAME_H
#define GAME_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct game_ctx* game_t;

typedef enum {
  GAME_OK = 0,
  GAME_EINVAL = -1,     /* an argument or the configuration is invalid     */
  GAME_EWORKSPACE = -2, /* the workspace is missing, too small or unaligned */
  GAME_EHIP = -3,       /* a HIP runtime call failed                        */
  GAME_ESTATE = -4      /* the call is not valid in the handle's state      */
} game_status;

/* Expansion families: Eq. 1 leaves g(x) free; Eq. 8 is the trigonometric
 * one the paper uses.  Chebyshev T_j, Legendre P_j, powers x^j, cos/sin(jx). */
typedef enum { GAME_CHEBYSHEV = 0, GAME_LEGENDRE = 1, GAME_POWER = 2, GAME_TRIG = 3 } game_basis;

/* Error functions: MSE (Eq. 4), RMSE (Eq. 5), TMSE (Eq. 10).  TMSE counts
 * a pattern's squared residual only when |t - Out| > R (the reading under
 * which the paper's worked example holds); GAME_TMSE_SQUARED compares the
 * squared residual with R as Eq. 10 is printed. */
typedef enum { GAME_MSE = 0, GAME_RMSE = 1, GAME_TMSE = 2, GAME_TMSE_SQUARED = 3 } game_error_fn;

/* Arithmetic of the fitness contraction: FP32 MFMA, or BF16 operands (genes
 * and expansion values rounded to nearest even) with FP32 accumulation and
 * a compensated reduction.  With GAME_BF16, game_run reports the elite's
 * error re-scored in float64 (game_rescore64). */
typedef enum { GAME_FP32 = 0, GAME_BF16 = 1 } game_precision;

/* Initial population (the three random modes listed in Sec. 2): normal in
 * [-1, 1] (sigma 1/3, clamped), uniform in [-1, 1), uniform in [0, 1). */
typedef enum { GAME_INIT_NORMAL = 0, GAME_INIT_UNIFORM = 1, GAME_INIT_UNIT = 2 } game_init;

/* Parent selection: a tournament of tournament_k draws with replacement
 * (lowest (fitness, index) wins), or the two criteria named in Sec. 2:
 * linear ranking with selection pressure 2 (rank r of P has weight P - r;
 * integer draw (u32 * P(P+1)/2) >> 32 located in the cumulative weights)
 * and roulette wheel (weight 1/(error + 1e-12) in float64, cumulative sum
 * left to right, first index above (u32 2^-32) * total; infinite or NaN
 * errors weigh 0; a wheel of zero total draws uniformly). */
typedef enum { GAME_TOURNAMENT = 0, GAME_RANKING = 1, GAME_ROULETTE = 2 } game_selection;

/* Run configuration (the user options of Sec. 2 and the parameters of
 * Sec. 5).  Genetic operators: tournament selection of size tournament_k
 * with replacement (lowest (fitness, index) wins); one-point crossover with
 * probability p_crossover and cut in [1, K-1]; per-gene Gaussian mutation
 * g <- clamp(g + sigma_mutation * z, -1, 1) with probability p_mutation;
 * elitism keeps `elitism` chromosomes unchanged (elite_mode 0: that many
 * copies of the winner, as the paper words it; 1: the best `elitism`).
 * Every random draw is Philox4x64-10 keyed by (seed, stream) with counter
 * (generation, unit, block, 0). */
typedef struct {
  int32_t basis;          /* game_basis                                   */
  int32_t degree;         /* d, 1..16                                     */
  int32_t population;     /* P, 2..8192                                   */
  int32_t tournament_k;   /* 1..population (paper: 4)                     */
  int32_t elitism;        /* 0..population-1 (paper: 2)                   */
  int32_t elite_mode;     /* 0 or 1                                       */
  int32_t init_mode;      /* game_init                                    */
  int32_t error_fn;       /* game_error_fn                                */
  int32_t precision;      /* game_precision                               */
  float p_crossover;      /* [0, 1] (paper: 0.9)                          */
  float p_mutation;       /* [0, 1] (paper: 0.2)                          */
  float sigma_mutation;   /* >= 0                                         */
  float tmse_R;           /* TMSE threshold R in (0, 1) (paper: 0.49)     */
  uint64_t seed;
  int32_t max_generations;/* stop after this many evolution steps        */
  double target;          /* stop when the best error <= target (0.001)  */
  int32_t selection;      /* game_selection                               */
} game_config;

/* Fills *cfg with the defaults: Chebyshev, d = 4, P = 50, tournament of
 * k = 3, elitism 2 (mode 0), normal init, MSE, FP32, p_c 0.9, p_m 0.05,
 * sigma 0.1, R 0.49, seed 0, 100 generations, target 0.001.  Returns
 * GAME_EINVAL on NULL. */
int game_config_default(game_config* cfg);

/* K = B*N*d + 1 for this configuration and feature count (Eq. 2 with
 * per-feature genes), or GAME_EINVAL. */
int game_num_genes(const game_config* cfg, int32_t n_features);

/* Bytes of device workspace game_create needs for this problem; 0 when the
 * configuration is invalid (see game_last_error()). */
size_t game_workspace_size(const game_config* cfg, int64_t n_patterns, int32_t n_features);

/* Creates a handle over a resident data set (the patterns of Sec. 2).
 * X_dev, t_dev and workspace_dev must stay valid and X_dev/t_dev unchanged
 * until game_destroy.  workspace_dev must be 256-byte aligned and at least
 * game_workspace_size() bytes.  Validates the configuration (GAME_EINVAL),
 * the workspace (GAME_EWORKSPACE).  The population is not initialised.  For
 * a float32 run of the trigonometric expansion (Eq. 8), cos x and sin x of
 * every pattern and feature are computed here once, into the workspace
 * (n_patterns x n_features x 8 bytes of it), queued on hip_stream: the
 * trigonometric terms are evaluated once per data set, not in every
 * generation (Sec. 4.1). */
int game_create(const game_config* cfg, const float* X_dev, const float* t_dev,
                int64_t n_patterns, int32_t n_features, void* workspace_dev,
                size_t workspace_bytes, void* hip_stream, game_t* out);

int game_destroy(game_t h);

/* Fitness of n chromosomes genes_dev [n x K] over the handle's data set
 * with the handle's error function (Eqs. 2-5, 10): fitness_dev [n] float32
 * and, if fitness64_dev is not NULL, the same values as float64.  Sums are
 * accumulated in float64 in a fixed order (deterministic).  A chromosome
 * whose error is NaN gets +inf.  1 <= n <= population. */
int game_fitness(game_t h, const float* genes_dev, int32_t n, float* fitness_dev,
                 double* fitness64_dev);

/* Error of n chromosomes on another data set of the same feature count
 * (the "test" use case of Sec. 2): err64_dev [n] float64.  X_dev/t_dev as
 * in game_create; 1 <= n <= population. */
int game_evaluate(game_t h, const float* X_dev, const float* t_dev, int64_t n_patterns,
                  const float* genes_dev, int32_t n, double* err64_dev);

/* Float64 error of n chromosomes genes_dev [n x K] (Eqs. 2-5, 10 evaluated
 * in double precision on the vector ALUs), err64_dev [n]: the elite's final
 * re-score after a BF16 run, or an exact audit of any result.  X_dev/t_dev
 * NULL means the handle's own data set (n_patterns is then ignored);
 * 1 <= n <= population.  Deterministic (fixed-order sums). */
int game_rescore64(game_t h, const float* X_dev, const float* t_dev, int64_t n_patterns,
                   const float* genes_dev, int32_t n, double* err64_dev);

/* The "run" use case of Sec. 2: the model output Out (Eq. 2) of n
 * chromosomes genes_dev [n x K] on n_patterns patterns X_dev, into out_dev
 * [n x n_patterns] float32, chromosome-major.  X_dev NULL means the handle's
 * own data set (n_patterns is then ignored).  Evaluated in float32 on the
 * vector ALUs in canonical gene order, whatever cfg.precision is.
 * 1 <= n <= 65535. */
int game_predict(game_t h, const float* X_dev, int64_t n_patterns, const float* genes_dev,
                 int32_t n, float* out_dev);

/* Classification counts of n chromosomes on a labelled set (Sec. 5 figures
 * of merit): a pattern is predicted as class 1 when Out >= threshold (the
 * same float32 Out as game_predict) and belongs to class 1 when t > 0.5.
 * counts_dev [n x 4] int64: true positives, false positives, true
 * negatives, false negatives.  X_dev/t_dev both NULL means the handle's own
 * data set. */
int game_classify(game_t h, const float* X_dev, const float* t_dev, int64_t n_patterns,
                  const float* genes_dev, int32_t n, float threshold, int64_t* counts_dev);

/* The paper's own model (Eq. 9) shares the genes a_j, b_j over all
 * features; its per-pattern sums do not depend on the genes and are
 * computed once per data set (Sec. 4.1).  Z_dev [n_patterns x 2*degree]
 * float32: column j-1 holds sum_i cos(j x_i), column degree+j-1 holds
 * sum_i sin(j x_i), j = 1..degree, x_i = X_dev[k * n_features + i] in
 * radians (any range), evaluated in float64 and rounded once.  A run of
 * the shared model is a run with basis GAME_POWER, degree 1 on Z_dev as a
 * data set of 2*degree features: its chromosome is then
 * [a_0, a_1..a_d, b_1..b_d] (2d+1 genes, Eq. 7).  1 <= degree <= 16.
 * Queued on hip_stream (NULL: the null stream); stateless. */
int game_trig_sums(const float* X_dev, int64_t n_patterns, int32_t n_features, int32_t degree,
                   float* Z_dev, void* hip_stream);

/* Figures of merit of Sec. 5 from host counts[4] (TP, FP, TN, FN):
 * merit[0] accuracy (TP+TN)/all, merit[1] completeness TP/(TP+FN),
 * merit[2] contamination FP/(FP+TN) (the fraction of class-0 patterns
 * classified as class 1), merit[3] FP/(TP+FP) (the other common
 * convention).  A ratio with a zero denominator is NaN. */
int game_merit(const int64_t* counts, double* merit);

/* Generation 0: random genes per cfg.init_mode (stream 0, unit =
 * chromosome, block = gene).  Resets the generation counter and stop flag. */
int game_init_population(game_t h);

/* One iteration of the loop of Sec. 4.1 on the stream: evaluate the
 * current population, rank it, test the stop criteria (best error <=
 * cfg.target or generation >= cfg.max_generations) and, unless stopped,
 * build the next generation.  Once stopped, further steps do nothing. */
int game_step(game_t h);

/* The training loop of Sec. 4.1 (evaluate and sort, test the stop
 * criteria, evolve) run to its stop criteria, the error threshold or the
 * maximum number of iterations of Sec. 5.  The loop is captured in a HIP
 * graph of 8 generations (no host round trip per generation); replays are
 * queued two at a time with two such chunks in flight, and queuing ends once
 * the device stop flag, copied back after each chunk, shows the run stopped
 * (chunks queued meanwhile do nothing).  With a surrogate attached the
 * generations are queued on the stream directly, 8 per chunk, with the same
 * stop checks (its few hundred short launches per generation run faster
 * that way).  Synchronises the stream.  max_generations < 0 and target < 0
 * keep the configured values; a run that stopped on earlier limits resumes
 * when its last evaluation no longer meets the new ones, and continues from
 * that evaluation exactly as one uninterrupted run would have; otherwise
 * nothing runs and the current results are reported.  Outputs (each may be NULL): the number of
 * evolution steps applied since the last init/set, the best chromosome [K]
 * and its float64 error. */
int game_run(game_t h, int32_t max_generations, double target, int32_t* generations_done,
             float* best_genes_host, double* best_error_host);

/* The "train" use case of Sec. 2 ends with the trained population stored:
 * copies of the current population [P x K] and, if fitness_dev is not NULL,
 * its fitness [P] as last evaluated (on the stream). */
int game_get_population(game_t h, float* genes_dev, float* fitness_dev);

/* Restores a stored population (the "train" use case's output, Sec. 2) to
 * resume training from it: genes_dev [P x K] becomes the current population
 * and the generation counter is set to `generation` (>= 0); the stop flag
 * clears.  The next generation's draws are those of generation + 1, so a
 * run resumed from the population and counter of step g continues exactly
 * as the uninterrupted run. */
int game_set_population(game_t h, const float* genes_dev, int32_t generation);

/* Synchronises the stream and reports the generation counter, the stop
 * flag, the best index of the last evaluation and its float64 error. */
int game_get_state(game_t h, int32_t* generation, int32_t* stopped, int32_t* best_index,
                   double* best_error);

/* Rank order of n fitness values (the "sort the best chromosomes" step of
 * Sec. 4.1): order_dev[r] is the index of rank r by (fitness ascending,
 * index ascending), NaN counted as +inf and -0 as +0.  1 <= n <= 8192. */
int game_rank(const float* fitness_dev, int32_t n, int32_t* order_dev, void* hip_stream);

/* Stateless genetic step: builds generation `generation` (>= 1) in
 * out_dev [P x K] from pop_dev [P x K] and its float32 fitness_dev [P],
 * with cfg's operators and seed (elitism, tournament, one-point crossover,
 * Gaussian mutation).  Bit-exact for given inputs.  workspace_dev: at least
 * game_ga_workspace_size(cfg) bytes, 256-byte aligned.  out_dev must not
 * overlap pop_dev. */
size_t game_ga_workspace_size(const game_config* cfg);
int game_ga_next(const game_config* cfg, int32_t n_genes, const float* pop_dev,
                 const float* fitness_dev, int32_t generation, float* out_dev,
                 void* workspace_dev, size_t workspace_bytes, void* hip_stream);

/* game_ga_next for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same genetic step with the same results bit for bit, but its rank
 * order and roulette sums live in a fixed scratch array inside the library
 * (98,304 bytes on each device that runs it, held until the process ends)
 * instead of a caller workspace, and it allocates nothing.  Arguments as in
 * game_ga_next without the workspace; population up to 8192 (a larger one
 * is GAME_EINVAL).  All calls on one device share that device's scratch and
 * nothing in it carries over between calls: calls that overlap on one
 * device (several streams or host threads) race, so the caller orders them.
 * Runs on the current device, which must be the stream's. */
int game_ga_next_static(const game_config* cfg, int32_t n_genes, const float* pop_dev,
                        const float* fitness_dev, int32_t generation, float* out_dev,
                        void* hip_stream);

/* Stateless generation-0 population [P x n_genes] (cfg.init_mode, cfg.seed). */
int game_init_genes(const game_config* cfg, int32_t n_genes, float* out_dev, void* hip_stream);

/* ------------------------------------------------------------------------
 * Fitness surrogate: a multilayer perceptron (genes -> standardised log
 * error; two hidden layers of `hidden` units with GELU, one output) trained
 * on the GPU with Adam from an archive of the exact evaluations the GA
 * makes.  The network's inputs are the genes standardised per gene,
 * x = (g - mean) * inv_std in float32 (two roundings), with the mean and
 * the inverse standard deviation (population form, deviation floored at
 * 1e-3) of the archived chromosomes, recomputed after every archived
 * generation; a new surrogate starts with mean 0 and inv_std 1.  Attached to a run it pre-screens offspring: each generation
 * builds oversample x (P - E) children with the same draws as the plain
 * genetic step (the first P - E of them are exactly the plain offspring),
 * scores them with the network, and keeps the P - E best-predicted ones.
 * An audit sample of `audit` randomly chosen children is scored exactly;
 * when the Spearman rank correlation between its predicted and exact
 * errors is below rho_min, or the archive holds fewer than min_archive
 * chromosomes, that generation keeps the plain offspring instead.  Exact
 * fitness remains the only selection criterion inside the population.
 * ---------------------------------------------------------------------- */
typedef struct game_surrogate_ctx* game_surrogate_t;

typedef struct {
  int32_t hidden;         /* units per hidden layer (256)                     */
  int32_t fp32_operands;  /* 0: BF16 operands, FP32 accumulation; 1: FP32      */
  int32_t archive;        /* archive capacity in chromosomes (16384)          */
  int32_t minibatch;      /* rows per Adam step (1024)                        */
  int32_t train_steps;    /* Adam steps per generation (48)                   */
  float lr;               /* Adam learning rate (2e-3)                        */
  int32_t oversample;     /* children generated per kept child (8)            */
  int32_t audit;          /* children scored exactly per generation (256)     */
  float rho_min;          /* rank correlation needed to screen (0.8)          */
  int32_t min_archive;    /* archive size needed to screen (4096)             */
  uint64_t seed;          /* initial weights and sampling draws (stream 3)    */
} game_surrogate_config;

int game_surrogate_config_default(game_surrogate_config* cfg);

/* Workspace bytes for a surrogate over n_genes inputs that predicts up to
 * max_batch rows at once (>= oversample x (P - E) to be attached). */
size_t game_surrogate_workspace_size(const game_surrogate_config* cfg, int32_t n_genes,
                                     int32_t max_batch);

/* Creates the network with its initial weights (uniform in
 * [-1/sqrt(fan_in), 1/sqrt(fan_in)) from Philox stream 3, zero biases) and
 * zero Adam moments, on the stream. */
int game_surrogate_create(const game_surrogate_config* cfg, int32_t n_genes, int32_t max_batch,
                          void* workspace_dev, size_t workspace_bytes, void* hip_stream,
                          game_surrogate_t* out);
int game_surrogate_destroy(game_surrogate_t s);

/* The input statistics in use: mean_dev [n_genes] and inv_std_dev
 * [n_genes] float32 (on the stream). */
int game_surrogate_get_input_stats(game_surrogate_t s, float* mean_dev, float* inv_std_dev);

/* Number of parameters; they are one float32 vector in the order W1
 * [hidden x n_genes], b1, W2 [hidden x hidden], b2, w3 [hidden], b3. */
int64_t game_surrogate_num_params(game_surrogate_t s);
int game_surrogate_get_params(game_surrogate_t s, float* params_dev);
int game_surrogate_set_params(game_surrogate_t s, const float* params_dev);

/* Predictions y_dev [n] for genes_dev [n x n_genes] (standardised with the
 * current input statistics), 1 <= n <= max_batch.
 * A row's prediction does not depend on n or on the other rows: every
 * product sums in one fixed order whatever the batch size. */
int game_surrogate_predict(game_surrogate_t s, const float* genes_dev, int32_t n, float* y_dev);

/* Gradients grads_dev [num_params] of mean((y - target)^2) over n rows
 * (1 <= n <= minibatch), and the predictions y_dev [n] if not NULL. */
int game_surrogate_gradients(game_surrogate_t s, const float* genes_dev, const float* target_dev,
                             int32_t n, float* grads_dev, float* y_dev);

/* One Adam step (beta 0.9 / 0.999, eps 1e-8, bias-corrected) on those
 * gradients. */
int game_surrogate_train_step(game_surrogate_t s, const float* genes_dev, const float* target_dev,
                              int32_t n);

/* Attaches (or, with NULL, detaches) a surrogate to a run: its generations
 * then screen offspring as described above.  The surrogate must have
 * n_genes = K, max_batch >= oversample x (P - E), audit <= P and the same
 * stream. */
int game_attach_surrogate(game_t h, game_surrogate_t s);

/* Synchronises and reports: rank correlation of the last audit, whether the
 * last generation was screened, generations screened so far, archive
 * size, Adam steps taken. */
int game_surrogate_stats(game_surrogate_t s, float* rho, int32_t* screened_last,
                         int32_t* screened_total, int32_t* archive_count, int32_t* adam_steps);

/* ------------------------------------------------------------------------
 * Batches: many independent runs of uneven sizes advanced together.  Each
 * generation is one persistent fitness launch over a work list of (run,
 * 64-chromosome tile, pattern split) items drained through atomic queues
 * (one per XCD; the tiles of one split share a queue, hence one L2), one
 * rank/stop-test launch and one genetic-step launch for all runs;
 * game_batch_run replays a captured HIP graph of such generations.  Every
 * run follows exactly the trajectory it would follow alone (same draws,
 * same fixed-order sums).  FP32 precision only.
 * ---------------------------------------------------------------------- */
typedef struct game_batch_ctx* game_batch_t;

typedef struct {
  const float* X_dev;     /* [n_patterns x n_features], caller-owned          */
  const float* t_dev;     /* [n_patterns]                                     */
  int64_t n_patterns;
  int32_t n_features;
  int32_t reserved;       /* set to 0                                         */
  game_config cfg;        /* the run's own configuration (precision FP32)     */
} game_run_desc;

/* Workspace bytes for a batch of n_runs runs (0 if a run is invalid). */
size_t game_batch_workspace_size(const game_run_desc* runs, int32_t n_runs);

/* Creates a batch over caller-owned data; the workspace (256-byte aligned,
 * game_batch_workspace_size bytes) holds every run's populations, fitness,
 * partial sums and the work list, and for each run of the trigonometric
 * expansion (Eq. 8) cos x and sin x of its patterns (n_patterns x
 * n_features x 8 bytes), computed here once.  X_dev and t_dev of every run
 * must stay valid and unchanged until game_batch_destroy.  Copies the
 * descriptors; synchronises the stream once.  The default decomposition is
 * 8 tiles of 256 patterns per item and 512 persistent workgroups.  The
 * fitness of a generation is one persistent launch for the polynomial
 * families and one for the trigonometric runs, if any. */
int game_batch_create(const game_run_desc* runs, int32_t n_runs, void* workspace_dev,
                      size_t workspace_bytes, void* hip_stream, game_batch_t* out);
int game_batch_destroy(game_batch_t b);

/* Sets the work decomposition: patterns per item in 256-row tiles, and the
 * number of persistent fitness workgroups.  Synchronises the stream. */
int game_batch_tune(game_batch_t b, int32_t tiles_per_item, int32_t grid);

/* The batch autotuner: times the batch's fitness launch (HIP events, reps
 * launches each) for every tiles_per_item in {1,2,4,8,16,32,64,128} and grid
 * in {256,512,1024}, keeps the fastest and reports it; times_ms (may be
 * NULL) receives the GAME_AUTOTUNE_CANDIDATES averages in that order (tiles
 * outer, grid inner).  Leaves the populations as they were.  Synchronises
 * the stream. */
#define GAME_AUTOTUNE_CANDIDATES 24
int game_batch_autotune(game_batch_t b, int32_t reps, int32_t* tiles_per_item, int32_t* grid,
                        float* best_ms, float* times_ms);

/* Per-run work decomposition: run i's patterns are cut into items of
 * tiles_per_item[i] (>= 1) 256-row tiles, host array [n_runs]; grid
 * persistent fitness workgroups (1..65536).  Synchronises the stream. */
int game_batch_tune_runs(game_batch_t b, const int32_t* tiles_per_item, int32_t grid);

/* The decomposition in use: tiles_per_item [n_runs] (host) and the grid. */
int game_batch_get_tuning(game_batch_t b, int32_t* tiles_per_item, int32_t* grid);

/* The autotuner by shape bucket: run i belongs to bucket bucket_of_run[i]
 * (0..n_buckets-1, n_buckets <= 64).  Starting from the best uniform
 * decomposition (game_batch_autotune), each used bucket in turn tries every
 * tiles_per_item of the uniform search with the other buckets fixed and
 * keeps the fastest fitness launch (HIP events, reps launches each).  The
 * result is set and returned: tiles_per_bucket [n_buckets] (host), the grid
 * and its average launch time.  Leaves the populations as they were.
 * Synchronises the stream. */
int game_batch_autotune_buckets(game_batch_t b, int32_t reps, const int32_t* bucket_of_run,
                                int32_t n_buckets, int32_t* tiles_per_bucket, int32_t* grid,
                                float* best_ms);

/* Generation 0 of every run (its own init_mode and seed). */
int game_batch_init(game_batch_t b);

/* One generation of every run that has not stopped (three launches). */
int game_batch_step(game_batch_t b);

/* The evaluation half of a generation (Sec. 4.1, evaluate): the fitness of
 * every running run's current population in one persistent launch, then
 * the per-run fixed-order sums into each run's fitness [P] (as
 * game_batch_get_population returns it); no ranking, stop test or genetic
 * step.  The same work list and results as the evaluation inside
 * game_batch_step. */
int game_batch_evaluate(game_batch_t b);

/* Runs every run until its stop criterion holds (its own max_generations
 * and target, Sec. 5), by replays of a captured graph of 4 generations,
 * queued two at a time with two such chunks in flight until the run states
 * copied back after a chunk show every run stopped; synchronises.  Outputs
 * per run (may be NULL): evolution steps applied, best float64 error of the
 * last evaluation. */
int game_batch_run(game_batch_t b, int32_t* generations_done_host, double* best_error_host);

/* Current population [P x K] of one run and its last fitness [P]. */
int game_batch_get_population(game_batch_t b, int32_t run, float* genes_dev, float* fitness_dev);

/* Current work decomposition: number of items, tiles per item (0 when the
 * runs' values differ), grid. */
int game_batch_num_items(game_batch_t b, int32_t* n_items, int32_t* tiles_per_item, int32_t* grid);

/* Message for the last failing call on this thread ("" if none). */
const char* game_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GAME_H */
