// Fused GAME fitness in float32 on MFMA (gfx950).
//
// For chromosome p and pattern k (Eq. 2 with per-feature genes):
//   Out[k,p] = a_0(p) + sum_{i,b,j} gene_p(i,b,j) * phi_{b,j}(x_{k,i})
// and the fitness is sum_k E_k / NP with E_k = (t_k - Out[k,p])^2 (Eqs. 3-4)
// or its thresholded form (Eq. 10).  The sum over (i,b,j) is a dense
// contraction: M = patterns, N = chromosomes, K = B*N*d expansion terms.
//
// Design:
//  * v_mfma_f32_32x32x2_f32.  The A operand (patterns x K) is never stored:
//    each lane owns one pattern row and one sub-feature u = (i, b) and
//    produces phi_1..phi_d of that sub-feature with the basis's three-term
//    recurrence, one value per K-step.  K is ordered so that the two lane
//    halves of a K-step carry sub-features 2q and 2q+1 at the same degree j,
//    so a lane's recurrence never crosses a feature boundary.
//  * The B operand (K x chromosomes) is copied once per workgroup into LDS,
//    one row per chromosome in the canonical gene order (odd row stride:
//    conflict-free ds_read_b32), by LDS DMA (global_load_lds_dword), so the
//    copy costs no registers and one memory round trip.  When K does not
//    fit, it passes through two buffers in chunks of whole feature pairs,
//    the next chunk's copy in flight while the current one is used.
//  * Accumulators start at zero.  A last K-step brings in the bias and the
//    target (lane half 0: 1 x a_0(p); half 1: -t_k x 1), so the accumulators
//    end at Out - t; the epilogue squares (or applies the error function)
//    and sums the lane's 32 rows in float32, then adds into a float64
//    running sum.
//    Partials per (chromosome, split) are combined in a fixed order: the
//    result does not depend on scheduling.
//  * The trigonometric expansion (Eq. 8) is seeded with cos x and sin x of
//    the lane's feature.  For the run's own data set they come from a table
//    computed once per data set (FitArgs::cs); otherwise sincosf in every
//    chromosome tile.
//  * Wave tile 64 patterns x 32*CB chromosomes: each generated A value feeds
//    CB MFMAs per row block.  For a single run whose population exceeds 64
//    a workgroup takes 128 chromosomes (CB = 4) with eight waves, waves 0-3
//    on the even pattern tiles of its split and 4-7 on the odd ones (two
//    waves per SIMD, one gene copy per CU, up to 159 K-steps of genes before
//    they are chunked); otherwise 64 chromosomes (CB = 2) with four waves
//    and two workgroups per CU (up to 128 K-steps).  The wider tile halves
//    the recurrence and feature-load work per MFMA.
//  * Grid: (pattern split) x (chromosome tile); consecutive blocks of one
//    split are mapped onto one XCD so its L2 serves the split's rows to all
//    chromosome tiles.
#include "fitness_f32_body.h"

namespace game {

template <int BASIS, int D, int CB>
__global__ __launch_bounds__(64 * fit_waves(CB), 8 / fit_waves(CB)) void fitness_f32_kernel(FitArgs a) {
  extern __shared__ float lds[];
  if (a.stop) {
    const int32_t stopped = *a.stop;
    if (a.stop_seen && blockIdx.x == 0 && threadIdx.x == 0) *a.stop_seen = stopped;
    if (stopped) return;
  }
  const float* __restrict__ genes = a.genes;
  if (a.gen_sel && (*a.gen_sel & 1)) genes = a.genes_alt;
  const int total = gridDim.x;
  const int b = blockIdx.x;
  const int L = a.xcd_remap ? (b & 7) * (total >> 3) + (b >> 3) : b;
  const int split = L / a.n_ctiles;
  const int ctile = L - split * a.n_ctiles;
  fitness_f32_block<BASIS, D, CB>(a, genes, split, ctile, lds);
}

template <int BASIS, int D, int CB>
static hipError_t launch_cb(const FitArgs& a, hipStream_t s) {
  const size_t lds = fitness_lds_bytes(a, D);
  const int grid = a.n_ctiles * a.n_splits;
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute((const void*)fitness_f32_kernel<BASIS, D, CB>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((fitness_f32_kernel<BASIS, D, CB>), dim3(grid), dim3(64 * fit_waves(CB)), lds,
                     s, a);
  return hipGetLastError();
}

template <int BASIS, int D>
static hipError_t launch_one(const FitArgs& a, hipStream_t s) {
  if (a.tile_cols == 128) return launch_cb<BASIS, D, 4>(a, s);
  return launch_cb<BASIS, D, 2>(a, s);
}

template <int BASIS>
static hipError_t launch_basis(const FitArgs& a, int degree, hipStream_t s) {
  switch (degree) {
#define GAME_CASE(D) case D: return launch_one<BASIS, D>(a, s);
    GAME_CASE(1) GAME_CASE(2) GAME_CASE(3) GAME_CASE(4) GAME_CASE(5) GAME_CASE(6)
    GAME_CASE(7) GAME_CASE(8) GAME_CASE(9) GAME_CASE(10) GAME_CASE(11) GAME_CASE(12)
    GAME_CASE(13) GAME_CASE(14) GAME_CASE(15) GAME_CASE(16)
#undef GAME_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fitness_f32(const FitArgs& a, int basis, int degree, hipStream_t s) {
  switch (basis) {
    case 0: return launch_basis<0>(a, degree, s);
    case 1: return launch_basis<1>(a, degree, s);
    case 2: return launch_basis<2>(a, degree, s);
    case 3: return a.cs ? launch_basis<kTrigTable>(a, degree, s) : launch_basis<3>(a, degree, s);
    default: return hipErrorInvalidValue;
  }
}

size_t fitness_lds_bytes(const FitArgs& a, int degree) {
  const int cols = a.tile_cols == 128 ? 128 : kTileCols;
  const size_t w = (size_t)(a.n_chunks > 1 ? 2 : 1) * cols *
                   (2 * a.pairs_per_chunk * degree + 1) * sizeof(float);
  const size_t red = (size_t)fit_waves(cols / 32) * cols * sizeof(double);
  return w > red ? w : red;
}

void plan_fitness(FitArgs& a, int degree, int basis, bool wide) {
  a.U = (basis == 3 ? 2 : 1) * a.N;
  a.Q = (a.U + 1) / 2;
  a.tile_cols = wide && a.n_chrom > kTileCols ? 128 : kTileCols;
  // K-steps (per lane half) of genes that stay in LDS for the whole launch:
  // two 64-chromosome workgroups share a CU, a 128-chromosome one has it to
  // itself; beyond that the genes pass through two buffers in chunks.
  const int max_steps = a.tile_cols == 128 ? kMaxWideSteps : kMaxChunkSteps;
  int ppc = a.Q * degree <= max_steps ? a.Q : kChunkSteps / degree;
  if (ppc < 1) ppc = 1;
  a.pairs_per_chunk = ppc;
  a.n_chunks = (a.Q + ppc - 1) / ppc;
  a.n_ctiles = (a.n_chrom + a.tile_cols - 1) / a.tile_cols;
  a.ld_partial = a.n_ctiles * a.tile_cols;
  a.n_tiles = (int32_t)((a.NP + kTileRows - 1) / kTileRows);
  // Aim at all resident workgroups on 256 CUs in one wave of blocks: one
  // eight-wave workgroup per CU for 128-chromosome tiles, two four-wave ones
  // for 64-chromosome tiles.
  const int target = a.tile_cols == 128 ? 256 : 512;
  int splits = (target + a.n_ctiles - 1) / a.n_ctiles;
  if (splits > max_splits(a.ld_partial)) splits = max_splits(a.ld_partial);
  if (splits > a.n_tiles) splits = a.n_tiles;
  if (splits < 1) splits = 1;
  a.tiles_per_split = (a.n_tiles + splits - 1) / splits;
  a.n_splits = (a.n_tiles + a.tiles_per_split - 1) / a.tiles_per_split;
  a.xcd_remap = ((a.n_ctiles * a.n_splits) % 8) == 0 ? 1 : 0;
}

// fitness[i] = sum_s partial[s][i] / NP (wave_split_sum order), RMSE takes
// the root; NaN becomes +inf.  One wave per chromosome.
__global__ void finish_kernel(const double* __restrict__ partial, int32_t ld, int32_t n,
                              int32_t n_splits, int64_t NP, int32_t error_fn, float* f32,
                              double* f64) {
  const int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= n) return;
  const double v = error_from_sum(wave_split_sum(partial, ld, n_splits, i), NP, error_fn);
  if ((threadIdx.x & 63) == 0) {
    if (f32) f32[i] = (float)v;
    if (f64) f64[i] = v;
  }
}

hipError_t launch_finish(const double* partial, int32_t ld, int32_t n, int32_t n_splits,
                         int64_t NP, int32_t error_fn, float* f32, double* f64, hipStream_t s) {
  hipLaunchKernelGGL(finish_kernel, dim3((n + 3) / 4), dim3(256), 0, s, partial, ld, n,
                     n_splits, NP, error_fn, f32, f64);
  return hipGetLastError();
}

}  // namespace game
