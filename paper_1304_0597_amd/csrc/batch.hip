// Batched form: the fitness of many independent GAME runs of uneven sizes
// in one persistent launch.
//
// The work of a generation is a list of items (run, 64-chromosome tile,
// pattern split).  The host groups the items of one (run, split) - every
// chromosome tile over the same patterns - and deals the groups, largest
// first, to the queue with the least work, one queue per XCD.  A fixed grid
// of workgroups drains the queues through atomic heads: workgroup b serves
// the queue of its own XCD (b % 8) first, so the chromosome tiles of a split
// run side by side on one XCD and read its patterns through one L2, then
// takes what is left in the other queues.  Each item is the float32 fitness
// computation of that run's tile over that split (the single-run float32
// body itself, dispatched on the run's basis and degree) and writes its
// float64 partial sums to the run's own partial array.  Which workgroup
// takes which item does not affect any result: every item owns its output
// slots and the per-run finish sums them in a fixed order.  A workgroup
// leaves the loop once every queue head has passed its queue's end.
#include "fitness_f32_body.h"

namespace game {

namespace {

// The single-run float32 body for one item of run `run`, at the run's
// degree (a uniform switch over the 16 compile-time degrees, all inlined)
// with the run's expansion family read at run time: the kernel makes no
// calls (a call per item would save and restore the callee's registers in
// private memory every time).
__device__ __forceinline__ void item_body(const BatchRun* __restrict__ run, const float* genes,
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
  fa.degree = run->D;
  fa.basis = run->basis;
  switch (__builtin_amdgcn_readfirstlane(run->D)) {
#define GAME_CASE(D) \
  case D:            \
    fitness_f32_block<-1, D>(fa, genes, split, ctile, lds); \
    break;
    GAME_CASE(1) GAME_CASE(2) GAME_CASE(3) GAME_CASE(4) GAME_CASE(5) GAME_CASE(6)
    GAME_CASE(7) GAME_CASE(8) GAME_CASE(9) GAME_CASE(10) GAME_CASE(11) GAME_CASE(12)
    GAME_CASE(13) GAME_CASE(14) GAME_CASE(15) GAME_CASE(16)
#undef GAME_CASE
    default: break;
  }
}

}  // namespace

__global__ __launch_bounds__(kFitThreads, 2) void fitness_batch_kernel(BatchArgs a) {
  extern __shared__ float lds[];
  __shared__ int item_sh;
  const int home = blockIdx.x % kXcds;
  int tried = 0;  // queues found empty so far (thread 0 only); heads only grow
  for (;;) {
    __syncthreads();  // the previous item is done with item_sh and LDS
    if (threadIdx.x == 0) {
      int got = -1;
      while (tried < kXcds) {
        const int q = (home + tried) % kXcds;
        const int i = a.queue_begin[q] + atomicAdd(&a.counter[q], 1);
        if (i < a.queue_begin[q + 1]) {
          got = i;
          break;
        }
        ++tried;
      }
      item_sh = got;
    }
    __syncthreads();
    const int it = item_sh;
    if (it < 0) break;
    const BatchItem w = a.items[it];
    const BatchRun* run = a.runs + w.run;
    const int stopped = run->state->stop;
    if (w.ctile == 0 && w.split == 0 && threadIdx.x == 0) run->state->stop_seen = stopped;
    if (stopped) continue;
    const float* genes = (run->state->gen & 1) ? run->pop1 : run->pop0;
    item_body(run, genes, w.split, w.ctile, lds);
  }
}

hipError_t launch_fitness_batch(const BatchArgs& a, size_t lds_bytes, hipStream_t s) {
  if (lds_bytes > 65536) {
    const hipError_t e = hipFuncSetAttribute((const void*)fitness_batch_kernel,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)lds_bytes);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fitness_batch_kernel, dim3(a.grid), dim3(kFitThreads), lds_bytes, s, a);
  return hipGetLastError();
}

}  // namespace game
