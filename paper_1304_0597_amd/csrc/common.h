// Internal declarations shared by libgame's translation units (not part of
// the C ABI; see include/game.h for that).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace game {

constexpr int kWave = 64;
constexpr int kMaxDegree = 16;
constexpr int kMaxPopulation = 8192;
constexpr int kMaxGenes = 4097;
constexpr int kMaxSplits = 64;

// Fitness tile geometry: a workgroup of 4 waves covers 256 patterns x 64
// chromosomes; each wave 64 patterns (two 32-row MFMA blocks) x 64
// chromosomes (two 32-column MFMA blocks).
constexpr int kTileRows = 256;
constexpr int kTileCols = 64;
constexpr int kFitThreads = 256;
// Largest K-chunk kept in LDS at once, in MFMA K-steps per lane half.
constexpr int kMaxChunkSteps = 128;

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
  int32_t ld_partial;       // n_ctiles * 64
  int32_t n_splits;
  int32_t tiles_per_split;
  int32_t n_tiles;
  int32_t xcd_remap;
  int32_t error_fn;
  float R;
};

// Grid/chunk planning shared by every fitness launch.
void plan_fitness(FitArgs& a, int degree, int basis);
size_t fitness_lds_bytes(const FitArgs& a, int degree);

hipError_t launch_fitness_f32(const FitArgs& a, int basis, int degree, hipStream_t s);
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
};
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
constexpr int kRankThreads = 1024;
constexpr int kRankPerBlock = 64;
hipError_t launch_set_state(RunState* st, int32_t gen, int32_t max_gen, double target,
                            int32_t reset, hipStream_t s);

}  // namespace game
