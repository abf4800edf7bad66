// Batched form: the fitness of many independent GAME runs of uneven sizes
// in one persistent launch per expansion family present.
//
// The work of a generation is a list of items (run, 64-chromosome tile,
// pattern split).  The host groups the items of one (run, split) - every
// chromosome tile over the same patterns - and deals the groups of each
// family, largest first, to that family's queue with the least work, one
// queue per XCD.  A fixed grid of workgroups drains one family's queues
// through atomic heads: workgroup b serves the queue of its own XCD (b % 8)
// first, so the chromosome tiles of a split run side by side on one XCD and
// read its patterns through one L2, then takes what is left in the family's
// other queues.  Each item is the float32 fitness computation of that run's
// tile over that split - the single-run float32 body itself, with the
// family fixed at compile time and the degree picked by a uniform switch -
// and writes its float64 partial sums to the run's own partial array.  Which
// workgroup takes which item, and which launch runs first, does not affect
// any result: every item owns its output slots and the per-run finish sums
// them in a fixed order.  A workgroup leaves the loop once every queue head
// of its family has passed its queue's end.
#include "fitness_f32_body.h"

namespace game {

namespace {

// The run table and the item list do not change while a launch runs; read
// through the constant address space, their fields come in with scalar loads
// into SGPRs instead of occupying vector registers.
using ConstRun = __attribute__((address_space(4))) const BatchRun;
using ConstItem = __attribute__((address_space(4))) const BatchItem;

// The single-run float32 body for one item of run `run` (expansion BASIS:
// a family, or kTrigTable), at the run's degree: a uniform switch over the
// 16 compile-time degrees, all inlined, so the kernel makes no calls (a call
// per item would save and restore the callee's registers in private memory
// every time).  A compile-time family keeps each body's expansion step the
// fixed recurrence of that family.  Each wave takes two consecutive pattern
// tiles at a time (four 32-row blocks over 64 chromosomes): a gene value
// read from LDS then feeds four MFMAs, and chunked genes are restaged once
// per two tiles; the per-element arithmetic and each tile's float32 sum
// are the single run's.  A run's last chromosome tile with at most 32 of
// its chromosomes takes a 32-column body (one MFMA column block), so the
// empty half of the tile is not computed; its index in 32-column units is
// twice the 64-column one.
template <int BASIS>
__device__ __forceinline__ void item_body(const ConstRun* run, const float* genes,
                                          int split, int ctile, float* lds) {
  FitArgs fa{};
  fa.X = run->X;
  fa.t = run->t;
  fa.partial = run->partial;
  fa.NP = run->NP;
  fa.N = run->N;
  fa.K = run->K;
  fa.n_chrom = run->P;
  fa.U = run->U;
  fa.Q = run->Q;
  fa.pairs_per_chunk = run->pairs_per_chunk;
  fa.n_chunks = run->n_chunks;
  fa.n_ctiles = run->n_ctiles;
  fa.ld_partial = run->ld_partial;
  fa.n_splits = run->n_splits;
  fa.tiles_per_split = run->tiles_per_split;
  fa.n_tiles = run->n_tiles;
  fa.error_fn = run->error_fn;
  fa.R = run->R;
  fa.cs = run->cs;
  fa.degree = run->D;
  fa.basis = run->basis;
  const bool narrow = run->P - ctile * kTileCols <= 32;
  switch (__builtin_amdgcn_readfirstlane(run->D)) {
#define GAME_CASE(D)                                                     \
  case D:                                                                \
    if (narrow) fitness_f32_block<BASIS, D, 1, 4>(fa, genes, split, 2 * ctile, lds); \
    else fitness_f32_block<BASIS, D, 2, 4>(fa, genes, split, ctile, lds);            \
    break;
    GAME_CASE(1) GAME_CASE(2) GAME_CASE(3) GAME_CASE(4) GAME_CASE(5) GAME_CASE(6)
    GAME_CASE(7) GAME_CASE(8) GAME_CASE(9) GAME_CASE(10) GAME_CASE(11) GAME_CASE(12)
    GAME_CASE(13) GAME_CASE(14) GAME_CASE(15) GAME_CASE(16)
#undef GAME_CASE
    default: break;
  }
}

// Drains family BASIS's queues: one item at a time until every queue head of
// the family has passed its queue's end.
template <int BASIS>
__device__ __forceinline__ void drain_family(const BatchArgs& a, float* lds, int* item_sh) {
  const int32_t* begin = a.queue_begin + BASIS * kXcds;
  int32_t* head = a.counter + BASIS * kXcds;
  if (begin[kXcds] == begin[0]) return;  // no items of this family
  const int home = blockIdx.x % kXcds;
  int tried = 0;  // queues found empty so far (thread 0 only); heads only grow
  for (;;) {
    __syncthreads();  // the previous item is done with item_sh and LDS
    if (threadIdx.x == 0) {
      int got = -1;
      while (tried < kXcds) {
        const int q = (home + tried) % kXcds;
        const int i = begin[q] + atomicAdd(&head[q], 1);
        if (i < begin[q + 1]) {
          got = i;
          break;
        }
        ++tried;
      }
      *item_sh = got;
    }
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(*item_sh);
    if (it < 0) break;
    ConstItem* w = (ConstItem*)a.items + it;
    ConstRun* run = (ConstRun*)a.runs + w->run;
    const int stopped = run->state->stop;
    if (w->ctile == 0 && w->split == 0 && threadIdx.x == 0) run->state->stop_seen = stopped;
    if (stopped) continue;
    const float* genes = (run->state->gen & 1) ? run->pop1 : run->pop0;
    // the trigonometric family is seeded from the run's stored (cos x, sin x)
    item_body<BASIS == 3 ? kTrigTable : BASIS>(run, genes, w->split, w->ctile, lds);
  }
}

}  // namespace

// The three polynomial families in one launch: a workgroup that finds the
// Chebyshev queues empty goes on to the Legendre and then the power items
// while others finish, so no family waits for the last item of another.
__global__ __launch_bounds__(kFitThreads, 2) void fitness_batch_kernel(BatchArgs a) {
  extern __shared__ float lds[];
  __shared__ int item_sh;
  drain_family<0>(a, lds, &item_sh);
  drain_family<1>(a, lds, &item_sh);
  drain_family<2>(a, lds, &item_sh);
}

// The trigonometric family in a launch of its own, its expansion seeded from
// each run's (cos x, sin x) table.
__global__ __launch_bounds__(kFitThreads, 2) void fitness_batch_trig_kernel(BatchArgs a) {
  extern __shared__ float lds[];
  __shared__ int item_sh;
  drain_family<3>(a, lds, &item_sh);
}

namespace {

hipError_t launch_drain(const void* kernel, const BatchArgs& a, size_t lds_bytes, hipStream_t s) {
  if (lds_bytes > 65536) {
    const hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)lds_bytes);
    if (e != hipSuccess) return e;
  }
  void* args[] = {const_cast<BatchArgs*>(&a)};
  return hipLaunchKernel(kernel, dim3(a.grid), dim3(kFitThreads), args, lds_bytes, s);
}

}  // namespace

hipError_t launch_fitness_batch(const BatchArgs& a, size_t lds_bytes, hipStream_t s) {
  static_assert(kFamilies == 4, "families 0-2 share a launch, family 3 has its own");
  if (a.queue_begin[3 * kXcds] > a.queue_begin[0]) {
    const hipError_t e = launch_drain((const void*)fitness_batch_kernel, a, lds_bytes, s);
    if (e != hipSuccess) return e;
  }
  if (a.queue_begin[4 * kXcds] > a.queue_begin[3 * kXcds])
    return launch_drain((const void*)fitness_batch_trig_kernel, a, lds_bytes, s);
  return hipSuccess;
}

}  // namespace game
