// Genetic operators of GAME on the device: initial population, ranking,
// elitism, tournament selection, one-point crossover, Gaussian mutation, and
// the per-generation evaluation epilogue with the stop test (the loop of
// Sec. 4.1: evaluate and sort, test the stop criteria, evolve).
//
// Every random draw is Philox4x64-10 (Salmon et al., SC'11) with key
// (seed, stream) and counter (generation, unit, block, 0):
//   stream 0  initialisation   unit = chromosome, block = gene
//   stream 1  selection        unit = child pair, 32-bit words lo(o0),
//                              hi(o0), lo(o1), ... continuing over blocks:
//                              k parent-1 indices, k parent-2 indices, the
//                              crossover coin, the cut point
//   stream 2  mutation         unit = child slot, block = gene; coin lo(o0),
//                              Gaussian from the twelve 16-bit fields of
//                              o1..o3 (Irwin-Hall: z = (S - 393210) 2^-16)
// An index in [0, n) is (u32 * n) >> 32; a coin of probability p fires when
// u32 < floor(p 2^32).  Float steps are single IEEE round-to-nearest
// operations (this file is built with -ffp-contract=off, and the mutation
// uses explicit __fmul_rn / __fadd_rn), so results are bit-reproducible.
#include "common.h"

namespace game {

struct U64x4 {
  uint64_t o0, o1, o2, o3;
};

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t lo0 = M0 * c0, hi0 = __umul64hi(M0, c0);
    const uint64_t lo1 = M1 * c2, hi1 = __umul64hi(M1, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return {c0, c1, c2, c3};
}

__device__ __forceinline__ U64x4 draw(uint64_t seed, uint64_t stream, uint64_t gen, uint64_t unit,
                                      uint64_t blk) {
  return philox4x64_10(gen, unit, blk, 0, seed, stream);
}

__device__ __forceinline__ float gauss12(const U64x4& b) {
  int32_t s = 0;
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    s += (int32_t)((b.o1 >> (16 * f)) & 0xFFFF);
    s += (int32_t)((b.o2 >> (16 * f)) & 0xFFFF);
    s += (int32_t)((b.o3 >> (16 * f)) & 0xFFFF);
  }
  return (float)(s - 393210) * 0x1p-16f;  // both steps exact
}

__device__ __forceinline__ float clamp_unit(float v) {
  return v < -1.f ? -1.f : (v > 1.f ? 1.f : v);
}

__device__ __forceinline__ float rank_key_value(float f) {
  if (isnan(f)) return INFINITY;
  return f == 0.f ? 0.f : f;
}

// Order-preserving map of a canonical float to uint32.
__device__ __forceinline__ uint32_t ordered_bits(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// ------------------------------------------------------------------ init
__global__ void init_kernel(uint64_t seed, int32_t mode, int32_t P, int32_t K, float* out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)P * K) return;
  const int64_t ch = idx / K, g = idx - ch * K;
  const U64x4 b = draw(seed, 0, 0, (uint64_t)ch, (uint64_t)g);
  const uint32_t lo24 = (uint32_t)(b.o0 & 0xFFFFFFFFull) >> 8;
  float v;
  if (mode == 0) {
    v = clamp_unit(__fmul_rn((float)(1.0 / 3.0), gauss12(b)));
  } else if (mode == 1) {
    v = (float)((int32_t)lo24 - (1 << 23)) * 0x1p-23f;
  } else {
    v = (float)lo24 * 0x1p-24f;
  }
  out[idx] = v;
}

hipError_t launch_init_genes(uint64_t seed, int32_t mode, int32_t P, int32_t K, float* out,
                             hipStream_t s) {
  const int64_t n = (int64_t)P * K;
  hipLaunchKernelGGL(init_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, seed, mode,
                     P, K, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ rank
// Ranks by counting: the rank of key e is the number of keys below it (keys
// are unique: fitness bits then index).  Each workgroup holds all keys in
// LDS and ranks kRankPerBlock of them; its 16 waves each count over one
// sixteenth of the keys, every lane of a wave reading the same key.
__device__ __forceinline__ uint64_t rank_key(float f, int i) {
  return ((uint64_t)ordered_bits(rank_key_value(f)) << 32) | (uint32_t)i;
}

// keys[i] = rank_key(fit[i], i) for i < P; the workgroup's loads of up to
// four keys per thread are in flight together.
__device__ __forceinline__ void fill_rank_keys(const float* fit, int P, uint64_t* keys) {
  const int nb = blockDim.x;
  for (int i0 = threadIdx.x; i0 < P; i0 += 4 * nb) {
    float f[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) f[u] = i0 + u * nb < P ? fit[i0 + u * nb] : 0.f;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i0 + u * nb < P) keys[i0 + u * nb] = rank_key(f[u], i0 + u * nb);
  }
}

__device__ __forceinline__ int count_rank(const uint64_t* keys, int P, int e, uint32_t* cnt) {
  constexpr int parts = kRankThreads / kRankPerBlock;
  const int part = threadIdx.x / kRankPerBlock;
  uint32_t c = 0;
  if (e < P) {
    const uint64_t ke = keys[e];
    const int per = (P + parts - 1) / parts;
    const int j0 = part * per;
    const int j1 = min(j0 + per, P);
    // Eight LDS reads in flight before the first compare (a read-compare
    // loop waits out the LDS latency for every key).
    int j = j0;
    for (; j + 8 <= j1; j += 8) {
      uint64_t kj[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) kj[u] = keys[j + u];
#pragma unroll
      for (int u = 0; u < 8; ++u) c += kj[u] < ke ? 1u : 0u;
    }
    for (; j < j1; ++j) c += keys[j] < ke ? 1u : 0u;
  }
  cnt[threadIdx.x] = c;
  __syncthreads();
  int r = -1;
  if (threadIdx.x < kRankPerBlock && e < P) {
    uint32_t t = 0;
    for (int k = 0; k < parts; ++k) t += cnt[k * kRankPerBlock + threadIdx.x];
    r = (int)t;
  }
  return r;
}

__global__ __launch_bounds__(kRankThreads) void rank_kernel(const float* __restrict__ fit, int32_t n,
                                                            int32_t* __restrict__ order) {
  extern __shared__ uint64_t keys[];
  __shared__ uint32_t cnt[kRankThreads];
  fill_rank_keys(fit, n, keys);
  __syncthreads();
  const int e = blockIdx.x * kRankPerBlock + (threadIdx.x % kRankPerBlock);
  const int r = count_rank(keys, n, e, cnt);
  if (r >= 0) order[r] = e;
}

// Allows more than 64 KiB of LDS per workgroup (gfx950 has 160 KiB per CU).
static hipError_t allow_lds(const void* fn, size_t dynamic_bytes) {
  if (dynamic_bytes + kRankThreads * sizeof(uint32_t) <= 65536) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dynamic_bytes);
}

hipError_t launch_rank(const float* fit, int32_t n, int32_t* order, hipStream_t s) {
  const hipError_t e = allow_lds((const void*)rank_kernel, (size_t)n * sizeof(uint64_t));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(rank_kernel, dim3((n + kRankPerBlock - 1) / kRankPerBlock), dim3(kRankThreads),
                     (size_t)n * sizeof(uint64_t), s, fit, n, order);
  return hipGetLastError();
}

// Errors of the 64 chromosomes [blk*64, blk*64+64) from their split
// partials, one wave per chromosome at a time (16 waves per workgroup, four
// chromosomes each).  With at most 64 splits a wave first loads the
// partials of all its chromosomes (lane l: split l, as wave_split_sum reads
// it), then adds each with the same butterfly, so the loads share one round
// trip.
constexpr int kReduceWaves = 16;
__device__ void reduce_fitness_body(const RankArgs& a, int blk) {
  if (a.state->stop_seen) return;
  const int waves = blockDim.x >> 6;
  if (a.n_splits <= 64 && waves == kReduceWaves) {
    constexpr int kPer = kRankPerBlock / kReduceWaves;
    const int lane = threadIdx.x & 63;
    const int i0 = blk * kRankPerBlock + (int)(threadIdx.x >> 6);
    double v[kPer];
#pragma unroll
    for (int c = 0; c < kPer; ++c) {
      // Unconditional loads (element 0 where there is no partial), so that
      // no branch separates them.
      const int i = i0 + c * kReduceWaves;
      const bool ok = i < a.P && lane < a.n_splits;
      const double p = a.partial[ok ? (int64_t)lane * a.ld_partial + i : 0];
      v[c] = ok ? 0.0 + p : 0.0;
    }
#pragma unroll
    for (int c = 0; c < kPer; ++c) {
      const int i = i0 + c * kReduceWaves;
      if (i >= a.P) break;
      double s = v[c];
      for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
      const double e = error_from_sum(s, a.NP, a.error_fn);
      if (lane == 0) {
        a.fit64[i] = e;
        a.fit32[i] = (float)e;
      }
    }
    return;
  }
  for (int j = (int)(threadIdx.x >> 6); j < kRankPerBlock; j += waves) {
    const int i = blk * kRankPerBlock + j;
    if (i >= a.P) break;
    const double v = error_from_sum(wave_split_sum(a.partial, a.ld_partial, a.n_splits, i), a.NP,
                                    a.error_fn);
    if ((threadIdx.x & 63) == 0) {
      a.fit64[i] = v;
      a.fit32[i] = (float)v;
    }
  }
}

__global__ __launch_bounds__(64 * kReduceWaves) void reduce_fitness_kernel(RankArgs a) {
  reduce_fitness_body(a, blockIdx.x);
}

hipError_t launch_reduce_fitness(const RankArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(reduce_fitness_kernel, dim3((a.P + kRankPerBlock - 1) / kRankPerBlock),
                     dim3(64 * kReduceWaves), 0, s, a);
  return hipGetLastError();
}

// Evaluation epilogue of one generation: rank order of the errors that
// reduce_fitness wrote, best chromosome, stop test and the generation
// counter.  The stop flag that
// decides whether this launch works is the one the generation's fitness
// launch recorded, so a workgroup that sets the flag cannot make another
// workgroup of the same launch skip its share.
// Body of one rank workgroup; `blk` is the workgroup's index within the run.
__device__ void finish_rank_body(const RankArgs& a, int blk, uint64_t* keys, uint32_t* cnt) {
  RunState* st = a.state;
  if (st->stop_seen) return;
  const int P = a.P;
  const int lo = blk * kRankPerBlock;
  fill_rank_keys(a.fit32, P, keys);
  __syncthreads();
  const int e = lo + (threadIdx.x % kRankPerBlock);
  const int r = count_rank(keys, P, e, cnt);
  if (r < 0) return;
  a.order[r] = e;
  if (r == 0) {
    const double v = a.fit64[e];
    const int gen = st->gen;
    st->best = e;
    st->best_err = v;
    st->evaluated = gen;
    if (v <= st->target || gen >= st->max_gen) {
      st->stop = 1;
    } else {
      st->gen = gen + 1;
    }
  }
}

__global__ __launch_bounds__(kRankThreads) void finish_rank_kernel(RankArgs a) {
  extern __shared__ uint64_t keys[];
  __shared__ uint32_t cnt[kRankThreads];
  finish_rank_body(a, blockIdx.x, keys, cnt);
}

hipError_t launch_finish_rank(const RankArgs& a, hipStream_t s) {
  const hipError_t e = allow_lds((const void*)finish_rank_kernel, (size_t)a.P * sizeof(uint64_t));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(finish_rank_kernel, dim3((a.P + kRankPerBlock - 1) / kRankPerBlock),
                     dim3(kRankThreads), (size_t)a.P * sizeof(uint64_t), s, a);
  return hipGetLastError();
}

// reset 1: start at generation `gen`; 0: new limits only; 2: new limits,
// and a run stopped on its last evaluation continues from it: the stop flag
// clears and the generation counter advances, as the stop test does when no
// criterion holds (the caller has checked that none does).
__global__ void set_state_kernel(RunState* st, int32_t gen, int32_t max_gen, double target,
                                 int32_t reset) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (reset == 2) {
    st->stop = 0;
    st->stop_seen = 0;
    st->gen = st->gen + 1;
  }
  if (reset == 1) {
    st->gen = gen;
    st->stop = 0;
    st->stop_seen = 0;
    st->best = -1;
    st->best_err = INFINITY;
    st->evaluated = -1;
  }
  st->max_gen = max_gen;
  st->target = target;
}

hipError_t launch_set_state(RunState* st, int32_t gen, int32_t max_gen, double target,
                            int32_t reset, hipStream_t s) {
  hipLaunchKernelGGL(set_state_kernel, dim3(1), dim3(64), 0, s, st, gen, max_gen, target, reset);
  return hipGetLastError();
}

// ------------------------------------------------------------- GA step
// One wave per output group: waves [0, E) copy the elites, wave E + q builds
// the two children of pair q.  Lanes stride over genes, so reads and writes
// of a chromosome are coalesced; the pair's selection draws are computed by
// every lane (wave-uniform).
__device__ __forceinline__ float fit_at(const float* fit, int i) {
  return rank_key_value(fit[i]);
}

// The stream-1 words of one child pair, produced in order: word i is the
// low (i even) or high (i odd) half of o[(i % 8) / 2] of block i / 8.  Words
// are read in increasing order, so each block is drawn once and only the
// current block is held (wave-uniform registers, no per-lane array).
struct PairWords {
  uint64_t seed, gen, unit;
  int blk;
  U64x4 r;
  __device__ PairWords(uint64_t s, uint64_t g, uint64_t u) : seed(s), gen(g), unit(u), blk(-1) {}
  __device__ uint32_t operator()(int i) {
    const int b = i >> 3;
    if (b != blk) {
      r = draw(seed, 1, gen, unit, (uint64_t)b);
      blk = b;
    }
    const int o = (i & 7) >> 1;
    const uint64_t v = o == 0 ? r.o0 : (o == 1 ? r.o1 : (o == 2 ? r.o2 : r.o3));
    return (i & 1) ? (uint32_t)(v >> 32) : (uint32_t)v;
  }
};

// Both tournaments of a pair: words [0, k) draw parent 1's candidates and
// [k, 2k) parent 2's.  The best candidate is the lowest fitness, ties to
// the lower index, the first draw kept unless beaten.  Candidate fitness
// values are loaded eight at a time, so their loads share a round trip;
// the comparisons run in draw order.
__device__ __forceinline__ void tournament_pair(const float* fit, PairWords& w, int k, int P,
                                                int& p1, int& p2) {
  int b1 = -1, b2 = -1;
  float f1 = 0.f, f2 = 0.f;
  for (int c0 = 0; c0 < 2 * k; c0 += 8) {
    int cand[8];
    float fc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      cand[u] = c0 + u < 2 * k ? (int)(((uint64_t)w(c0 + u) * (uint64_t)P) >> 32) : 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) fc[u] = fit_at(fit, cand[u]);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = c0 + u;
      if (c >= 2 * k) break;
      if (c < k) {
        if (b1 < 0 || fc[u] < f1 || (fc[u] == f1 && cand[u] < b1)) {
          b1 = cand[u];
          f1 = fc[u];
        }
      } else if (b2 < 0 || fc[u] < f2 || (fc[u] == f2 && cand[u] < b2)) {
        b2 = cand[u];
        f2 = fc[u];
      }
    }
  }
  p1 = b1;
  p2 = b2;
}

// Linear ranking, pressure 2: rank r has weight P - r; the integer draw
// t = (u32 * P(P+1)/2) >> 32 falls in rank r's cumulative interval.
__device__ __forceinline__ int ranking_pick(const int32_t* order, int P, uint32_t u) {
  const int64_t W = (int64_t)P * (P + 1) / 2;
  const int64_t t = (int64_t)(((uint64_t)u * (uint64_t)W) >> 32);
  int lo = 0, hi = P - 1;                 // first r with cum_end(r) > t
  while (lo < hi) {
    const int r = (lo + hi) >> 1;
    const int64_t cum_end = (int64_t)(r + 1) * P - (int64_t)(r + 1) * r / 2;
    if (cum_end > t) hi = r;
    else lo = r + 1;
  }
  return order[lo];
}

// Roulette wheel: first index whose cumulative weight exceeds
// (u32 2^-32) * total; zero total draws uniformly.
__device__ __forceinline__ int roulette_pick(const double* cum, int P, uint32_t u) {
  const double total = cum[P - 1];
  if (!(total > 0.0)) return (int)(((uint64_t)u * (uint64_t)P) >> 32);
  const double target = ((double)u * 0x1p-32) * total;
  int lo = 0, hi = P;                      // first i with cum[i] > target
  while (lo < hi) {
    const int i = (lo + hi) >> 1;
    if (cum[i] > target) hi = i;
    else lo = i + 1;
  }
  return lo < P ? lo : P - 1;
}

// Roulette weights in parallel, then one fixed left-to-right float64 scan.
__device__ void roulette_cum_body(const float* fit, int P, double* cum, double* w) {
  for (int i = threadIdx.x; i < P; i += blockDim.x)
    w[i] = 1.0 / ((double)rank_key_value(fit[i]) + 1e-12);
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < P; ++i) {
      s += w[i];
      cum[i] = s;
    }
  }
}

__global__ __launch_bounds__(1024) void roulette_cum_kernel(const float* fit, int P, double* cum,
                                                            const int32_t* stop) {
  extern __shared__ double w[];
  if (stop && *stop) return;
  roulette_cum_body(fit, P, cum, w);
}

hipError_t launch_roulette_cum(const float* fit, int32_t P, double* cum, const int32_t* stop,
                               hipStream_t s) {
  const size_t lds = (size_t)P * sizeof(double);
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute((const void*)roulette_cum_kernel,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(roulette_cum_kernel, dim3(1), dim3(1024), lds, s, fit, P, cum, stop);
  return hipGetLastError();
}

// Body of one wave: output group `wid` (an elite slot, or child pair
// wid - E) of the run described by `a`.
// Pointer c ? x : y as integer arithmetic on already loaded values.  (A
// select between two fields of the argument structure is otherwise turned
// into a load through a selected field address, which keeps the whole
// structure in private memory.)
template <class T>
__device__ __forceinline__ T* pick(bool c, T* x, T* y) {
  const uintptr_t ux = (uintptr_t)x, uy = (uintptr_t)y;
  return (T*)(uy ^ ((ux ^ uy) & (uintptr_t)(-(intptr_t)c)));
}

__device__ __forceinline__ void ga_next_wave(const GAArgs& a, int wid) {
  if (a.stop && *a.stop) return;
  int gen;
  const float* __restrict__ pop;
  float* __restrict__ out;
  if (a.gen_ptr) {
    gen = *a.gen_ptr;
    pop = pick(((gen - 1) & 1) != 0, a.pop_b, a.pop_a);
    out = pick((gen & 1) != 0, a.out_b, a.out_a);
  } else {
    gen = a.generation;
    pop = a.pop_a;
    out = a.out_a;
  }
  const int lane = threadIdx.x & 63;
  const int P = a.P, K = a.K, E = a.E;
  const int n_slots = a.n_slots ? a.n_slots : P;
  const int n_pairs = (n_slots - E + 1) >> 1;
  if (wid < E) {
    const int src = a.elite_mode == 0 ? a.order[0] : a.order[wid];
    for (int g = lane; g < K; g += 64) out[(int64_t)wid * K + g] = pop[(int64_t)src * K + g];
    return;
  }
  const int q = wid - E;
  if (q >= n_pairs) return;

  // Selection words of pair q, consumed in order: parent 1, parent 2 (k
  // words each for a tournament, one for ranking or roulette), the
  // crossover coin, the cut point.
  PairWords w(a.seed, (uint64_t)gen, (uint64_t)q);
  const int k = a.selection == 0 ? a.k : 1;
  int p1, p2;
  if (a.selection == 1) {
    p1 = ranking_pick(a.order, P, w(0));
    p2 = ranking_pick(a.order, P, w(1));
  } else if (a.selection == 2) {
    p1 = roulette_pick(a.cum, P, w(0));
    p2 = roulette_pick(a.cum, P, w(1));
  } else {
    tournament_pair(a.fitness, w, k, P, p1, p2);
  }
  const bool cross = (uint64_t)w(2 * k) < a.thr_cross;
  const int cut = 1 + (int)(((uint64_t)w(2 * k + 1) * (uint64_t)(K - 1)) >> 32);

  const int sa = E + 2 * q, sb = sa + 1;
  const bool has_b = sb < n_slots;
  float* __restrict__ out_a = pick(a.children != nullptr, a.children + (int64_t)(sa - E) * K,
                                   out + (int64_t)sa * K);
  float* __restrict__ out_b = pick(a.children != nullptr, a.children + (int64_t)(sb - E) * K,
                                   out + (int64_t)sb * K);
  // The parents' genes of up to four lane strides are loaded before the
  // mutation draws, so the loads' latency overlaps the draws.
  constexpr int kStrides = 4;
  for (int g0 = lane; g0 < K; g0 += kStrides * 64) {
    float x1[kStrides], x2[kStrides];
#pragma unroll
    for (int u = 0; u < kStrides; ++u) {
      const int g = g0 + 64 * u;
      x1[u] = g < K ? pop[(int64_t)p1 * K + g] : 0.f;
      x2[u] = g < K ? pop[(int64_t)p2 * K + g] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < kStrides; ++u) {
      const int g = g0 + 64 * u;
      if (g >= K) break;
      const bool sw = cross && g >= cut;
      float ca = sw ? x2[u] : x1[u];
      float cb = sw ? x1[u] : x2[u];
      {
        const U64x4 r = draw(a.seed, 2, (uint64_t)gen, (uint64_t)sa, (uint64_t)g);
        if ((r.o0 & 0xFFFFFFFFull) < a.thr_mut)
          ca = clamp_unit(__fadd_rn(ca, __fmul_rn(a.sigma, gauss12(r))));
      }
      out_a[g] = ca;
      if (has_b) {
        const U64x4 r = draw(a.seed, 2, (uint64_t)gen, (uint64_t)sb, (uint64_t)g);
        if ((r.o0 & 0xFFFFFFFFull) < a.thr_mut)
          cb = clamp_unit(__fadd_rn(cb, __fmul_rn(a.sigma, gauss12(r))));
        out_b[g] = cb;
      }
    }
  }
}

__global__ __launch_bounds__(256) void ga_next_kernel(GAArgs a) {
  ga_next_wave(a, blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
}

hipError_t launch_ga_next(const GAArgs& a, hipStream_t s) {
  const int n_slots = a.n_slots ? a.n_slots : a.P;
  const int n_waves = a.E + ((n_slots - a.E + 1) >> 1);
  hipLaunchKernelGGL(ga_next_kernel, dim3((n_waves + 3) / 4), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------- batches
__device__ RankArgs rank_args_of(const BatchRun& r) {
  RankArgs a{};
  a.partial = r.partial;
  a.ld_partial = r.ld_partial;
  a.n_splits = r.n_splits;
  a.NP = r.NP;
  a.P = r.P;
  a.error_fn = r.error_fn;
  a.fit32 = r.fit32;
  a.fit64 = r.fit64;
  a.order = r.order;
  a.state = r.state;
  return a;
}

// Rank workgroups of every run in one launch; workgroup b serves run
// rank_block_run[b].
__global__ __launch_bounds__(kRankThreads) void finish_rank_batch_kernel(BatchArgs a) {
  extern __shared__ uint64_t keys[];
  __shared__ uint32_t cnt[kRankThreads];
  const int r = a.rank_block_run[blockIdx.x];
  const BatchRun& run = a.runs[r];
  finish_rank_body(rank_args_of(run), blockIdx.x - run.rank_block0, keys, cnt);
}

__global__ __launch_bounds__(64 * kReduceWaves) void reduce_fitness_batch_kernel(BatchArgs a) {
  const int r = a.rank_block_run[blockIdx.x];
  const BatchRun& run = a.runs[r];
  reduce_fitness_body(rank_args_of(run), blockIdx.x - run.rank_block0);
}

hipError_t launch_reduce_fitness_batch(const BatchArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(reduce_fitness_batch_kernel, dim3(a.n_rank_blocks), dim3(64 * kReduceWaves), 0,
                     s, a);
  return hipGetLastError();
}

hipError_t launch_finish_rank_batch(const BatchArgs& a, hipStream_t s) {
  const size_t lds = (size_t)a.max_population * sizeof(uint64_t);
  const hipError_t e = allow_lds((const void*)finish_rank_batch_kernel, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(finish_rank_batch_kernel, dim3(a.n_rank_blocks), dim3(kRankThreads), lds, s,
                     a);
  return hipGetLastError();
}

// Genetic-step waves of every run in one launch; also re-arms the fitness
// work queue for the next generation.
__global__ __launch_bounds__(256) void ga_next_batch_kernel(BatchArgs a) {
  if (blockIdx.x == 0 && threadIdx.x < kQueues) a.counter[threadIdx.x] = 0;
  const int gw = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (gw >= a.n_ga_waves) return;
  const int r = a.ga_wave_run[gw];
  const BatchRun& run = a.runs[r];
  GAArgs g{};
  g.pop_a = run.pop0;
  g.pop_b = run.pop1;
  g.out_a = run.pop0;
  g.out_b = run.pop1;
  g.fitness = run.fit32;
  g.order = run.order;
  g.gen_ptr = &run.state->gen;
  g.stop = &run.state->stop;
  g.P = run.P;
  g.K = run.K;
  g.k = run.k;
  g.E = run.E;
  g.elite_mode = run.elite_mode;
  g.thr_cross = run.thr_cross;
  g.thr_mut = run.thr_mut;
  g.sigma = run.sigma;
  g.seed = run.seed;
  g.selection = run.selection;
  g.cum = run.cum;
  ga_next_wave(g, gw - run.ga_wave0);
}

hipError_t launch_ga_next_batch(const BatchArgs& a, hipStream_t s) {
  const int blocks = (a.n_ga_waves + 3) / 4;
  hipLaunchKernelGGL(ga_next_batch_kernel, dim3(blocks < 1 ? 1 : blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Roulette wheels of every run that selects by roulette: workgroup r
// serves run r.
__global__ __launch_bounds__(1024) void roulette_cum_batch_kernel(BatchArgs a) {
  extern __shared__ double w[];
  const BatchRun& run = a.runs[blockIdx.x];
  if (run.selection != 2 || run.state->stop) return;
  roulette_cum_body(run.fit32, run.P, run.cum, w);
}

hipError_t launch_roulette_cum_batch(const BatchArgs& a, hipStream_t s) {
  const size_t lds = (size_t)a.max_population * sizeof(double);
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute((const void*)roulette_cum_batch_kernel,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(roulette_cum_batch_kernel, dim3(a.n_runs), dim3(1024), lds, s, a);
  return hipGetLastError();
}

__global__ void batch_reset_kernel(BatchArgs a) {
  if (blockIdx.x == 0 && threadIdx.x < kQueues) a.counter[threadIdx.x] = 0;
}

hipError_t launch_batch_reset(const BatchArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(batch_reset_kernel, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------- surrogate
// Parameters: W1 [H x n_in], b1 [H], W2 [H x H], b2 [H], w3 [H], b3 [1] in
// one flat vector.  Weight element e of tensor t is
// float32(2u - 1) * float32(1 / sqrt(fan_in)) with u = (lo32(o0) >> 8) 2^-24
// from key (seed, 3), counter (0, t, e, 0); biases start at zero.
__global__ void mlp_init_kernel(float* params, int n_in, int H, uint64_t seed) {
  const int64_t o1 = (int64_t)H * n_in, o2 = o1 + H, o3 = o2 + (int64_t)H * H, o4 = o3 + H,
                o5 = o4 + H, total = o5 + 1;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  int tensor;
  int64_t e;
  int fan;
  if (i < o1) { tensor = 0; e = i; fan = n_in; }
  else if (i < o2) { params[i] = 0.f; return; }
  else if (i < o3) { tensor = 2; e = i - o2; fan = H; }
  else if (i < o4) { params[i] = 0.f; return; }
  else if (i < o5) { tensor = 4; e = i - o4; fan = H; }
  else { params[i] = 0.f; return; }
  const U64x4 b = draw(seed, 3, 0, (uint64_t)tensor, (uint64_t)e);
  const int32_t k = (int32_t)((uint32_t)(b.o0 & 0xFFFFFFFFull) >> 8);
  const float u2 = (float)(2 * k - (1 << 24)) * 0x1p-24f;       // 2u - 1, exact
  const float scale = (float)(1.0 / sqrt((double)fan));
  params[i] = __fmul_rn(u2, scale);
}

hipError_t launch_mlp_init(float* params, int n_in, int H, uint64_t seed, hipStream_t s) {
  const int64_t total = (int64_t)H * n_in + H + (int64_t)H * H + H + H + 1;
  hipLaunchKernelGGL(mlp_init_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     params, n_in, H, seed);
  return hipGetLastError();
}

// Appends the generation just evaluated (genes and log error, the error
// clamped to [1e-30, 1e30]) at the archive's ring position.  Skipped when
// the generation's fitness launch did not run (the run had stopped).
// A generation that stopped the run is not archived: a run resumed later
// evaluates that population again and archives it then, as one uninterrupted
// run would.
__global__ void archive_append_kernel(ArchiveArgs a) {
  if (a.run->stop) return;
  const int ev = a.run->evaluated;
  const float* pop = (ev & 1) ? a.pop1 : a.pop0;
  const int head = a.st->head;
  const int64_t n = (int64_t)a.P * a.K;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(i / a.K), g = (int)(i - (int64_t)c * a.K);
    const int row = (head + c) % a.capacity;
    a.genes[(int64_t)row * a.K + g] = pop[i];
    if (g == 0) {
      double f = a.fit64[c];
      f = isnan(f) ? 1e30 : fmin(fmax(f, 1e-30), 1e30);
      a.target[row] = (float)log(f);
    }
  }
}

hipError_t launch_archive_append(const ArchiveArgs& a, hipStream_t s) {
  const int64_t n = (int64_t)a.P * a.K;
  int blocks = (int)((n + 255) / 256);
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(archive_append_kernel, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

// Advances the archive ring after an append and recomputes the mean and
// inverse standard deviation of its targets (fixed-order float64 sums).
__global__ __launch_bounds__(1024) void archive_stats_kernel(const float* target, SurrogateState* st,
                                                             const RunState* run, int P,
                                                             int capacity) {
  __shared__ double s1[1024], s2[1024];
  __shared__ int cnt;
  if (run->stop) return;
  if (threadIdx.x == 0) {
    const int c = min(st->count + P, capacity);
    st->count = c;
    st->head = (st->head + P) % capacity;
    cnt = c;
  }
  __syncthreads();
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
    const double v = target[i];
    a += v;
    b += v * v;
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int k = 512; k > 0; k >>= 1) {
    if (threadIdx.x < k) {
      s1[threadIdx.x] += s1[threadIdx.x + k];
      s2[threadIdx.x] += s2[threadIdx.x + k];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mean = s1[0] / cnt;
    const double var = fmax(s2[0] / cnt - mean * mean, 1e-12);
    st->mean = (float)mean;
    st->inv_std = (float)(1.0 / sqrt(var));
  }
}

hipError_t launch_archive_stats(const float* target, SurrogateState* st, const RunState* run,
                                int P, int capacity, hipStream_t s) {
  hipLaunchKernelGGL(archive_stats_kernel, dim3(1), dim3(1024), 0, s, target, st, run, P,
                     capacity);
  return hipGetLastError();
}

// Input statistics: every gene centred on its archive mean and scaled by
// its archive spread, so that the network resolves the small differences
// between a converging population's chromosomes.  Workgroup b sums rows
// [b * per, (b + 1) * per) of the archive per gene in float64 (one thread
// per gene, rows in order: coalesced reads of each row, 16 rows' loads in
// flight at a time); then one thread per gene adds the kMomentBlocks shares
// in workgroup order.
constexpr int kMomentRows = 16;
__global__ __launch_bounds__(1024) void gene_moments_kernel(const float* genes, int K, int capacity,
                                                           const SurrogateState* st,
                                                           const RunState* run, double* part) {
  if (run->stop) return;
  const int count = st->count;
  const int per = (capacity + kMomentBlocks - 1) / kMomentBlocks;
  const int r0 = blockIdx.x * per;
  const int r1 = min(r0 + per, count);
  for (int g = threadIdx.x; g < K; g += blockDim.x) {
    double a = 0.0, b = 0.0;
    int r = r0;
    for (; r + kMomentRows <= r1; r += kMomentRows) {
      float v[kMomentRows];
#pragma unroll
      for (int u = 0; u < kMomentRows; ++u) v[u] = genes[(int64_t)(r + u) * K + g];
#pragma unroll
      for (int u = 0; u < kMomentRows; ++u) {
        const double d = v[u];
        a += d;
        b += d * d;
      }
    }
    for (; r < r1; ++r) {
      const double v = genes[(int64_t)r * K + g];
      a += v;
      b += v * v;
    }
    part[(int64_t)blockIdx.x * K + g] = a;
    part[(int64_t)(kMomentBlocks + blockIdx.x) * K + g] = b;
  }
}

__global__ void gene_stats_kernel(const double* part, int K, const SurrogateState* st,
                                  const RunState* run, float* mu, float* inv) {
  if (run->stop) return;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int count = st->count;
  if (g >= K || count < 1) return;
  double a = 0.0, b = 0.0;
  for (int k0 = 0; k0 < kMomentBlocks; k0 += kMomentRows) {
    double pa[kMomentRows], pb[kMomentRows];
#pragma unroll
    for (int u = 0; u < kMomentRows; ++u) {
      pa[u] = part[(int64_t)(k0 + u) * K + g];
      pb[u] = part[(int64_t)(kMomentBlocks + k0 + u) * K + g];
    }
#pragma unroll
    for (int u = 0; u < kMomentRows; ++u) {
      a += pa[u];
      b += pb[u];
    }
  }
  const double m = a / count;
  const double var = fmax(b / count - m * m, 0.0);
  mu[g] = (float)m;
  inv[g] = (float)(1.0 / fmax(sqrt(var), kInputStdFloor));
}

hipError_t launch_gene_stats(const float* genes, int32_t K, int32_t capacity,
                             const SurrogateState* st, const RunState* run, double* part,
                             float* mu, float* inv, hipStream_t s) {
  const int threads = min(1024, (K + 63) / 64 * 64);
  hipLaunchKernelGGL(gene_moments_kernel, dim3(kMomentBlocks), dim3(threads), 0, s, genes, K,
                     capacity, st, run, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gene_stats_kernel, dim3((K + 255) / 256), dim3(256), 0, s, part, K, st, run,
                     mu, inv);
  return hipGetLastError();
}

__device__ __forceinline__ float standardize1(float g, float mu, float inv) {
  return __fmul_rn(__fsub_rn(g, mu), inv);
}

__global__ void standardize_kernel(const float* src, int64_t n, int K, const float* mu,
                                   const float* inv, float* dst, const int32_t* skip) {
  if (skip && *skip) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int g = (int)(i % K);
    dst[i] = standardize1(src[i], mu[g], inv[g]);
  }
}

hipError_t launch_standardize(const float* src, int32_t n, int32_t K, const float* mu,
                              const float* inv, float* dst, const int32_t* skip, hipStream_t s) {
  const int64_t total = (int64_t)n * K;
  int blocks = (int)((total + 255) / 256);
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(standardize_kernel, dim3(blocks), dim3(256), 0, s, src, total, K, mu, inv,
                     dst, skip);
  return hipGetLastError();
}

// Minibatch of B archive rows drawn with replacement: row b is
// (u32 * count) >> 32 with u32 = lo32(o0) of key (seed, 3), counter
// (generation, 1 + step, b, 0); genes and targets standardised.
__device__ __forceinline__ void sample_minibatch_body(int64_t i, const float* genes,
                                                      const float* target, int K,
                                                      const SurrogateState* st,
                                                      const RunState* run, uint64_t seed, int step,
                                                      int B, const float* mu, const float* inv,
                                                      float* Xb, float* tb) {
  if (i >= (int64_t)B * K) return;
  const int b = (int)(i / K), g = (int)(i - (int64_t)b * K);
  const U64x4 r = draw(seed, 3, (uint64_t)run->evaluated, (uint64_t)(1 + step), (uint64_t)b);
  const int idx = (int)(((r.o0 & 0xFFFFFFFFull) * (uint64_t)st->count) >> 32);
  Xb[i] = standardize1(genes[(int64_t)idx * K + g], mu[g], inv[g]);
  if (g == 0) tb[b] = (target[idx] - st->mean) * st->inv_std;
}

__global__ void sample_minibatch_kernel(const float* genes, const float* target, int K,
                                        const SurrogateState* st, const RunState* run,
                                        uint64_t seed, int step, int B, const float* mu,
                                        const float* inv, float* Xb, float* tb) {
  if (run->stop) return;
  sample_minibatch_body((int64_t)blockIdx.x * blockDim.x + threadIdx.x, genes, target, K, st, run,
                        seed, step, B, mu, inv, Xb, tb);
}

// Workgroups [0, adam_blocks) update the parameters; the rest draw the next
// step's minibatch (Xb and tb are not read by the update).
__global__ void adam_sample_kernel(float* p, const float* part, int ks, float* m, float* v,
                                   int64_t n, float lr, SurrogateState* st, const int32_t* skip,
                                   int adam_blocks, const float* genes, const float* target, int K,
                                   const RunState* run, uint64_t seed, int next_step, int B,
                                   const float* mu, const float* inv, float* Xb, float* tb) {
  if (skip && *skip) return;
  if ((int)blockIdx.x < adam_blocks) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) adam_update(p, part, ks, m, v, n, lr, st->step, i);
    return;
  }
  sample_minibatch_body((int64_t)(blockIdx.x - adam_blocks) * blockDim.x + threadIdx.x, genes,
                        target, K, st, run, seed, next_step, B, mu, inv, Xb, tb);
}

hipError_t launch_adam_sample(float* p, const float* part, int ks, float* m, float* v, int64_t n,
                              float lr, SurrogateState* st, const int32_t* skip, const float* genes,
                              const float* target, int32_t K, const RunState* run, uint64_t seed,
                              int32_t next_step, int32_t B, const float* mu, const float* inv,
                              float* Xb, float* tb, hipStream_t s) {
  const int adam_blocks = (int)((n + 255) / 256);
  const int sample_blocks = (int)(((int64_t)B * K + 255) / 256);
  hipLaunchKernelGGL(adam_sample_kernel, dim3((unsigned)(adam_blocks + sample_blocks)), dim3(256),
                     0, s, p, part, ks, m, v, n, lr, st, skip, adam_blocks, genes, target, K, run,
                     seed, next_step, B, mu, inv, Xb, tb);
  return hipGetLastError();
}

hipError_t launch_sample_minibatch(const float* genes, const float* target, int32_t K,
                                   const SurrogateState* st, const RunState* run, uint64_t seed,
                                   int32_t step, int32_t B, const float* mu, const float* inv,
                                   float* Xb, float* tb, hipStream_t s) {
  const int64_t n = (int64_t)B * K;
  hipLaunchKernelGGL(sample_minibatch_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     genes, target, K, st, run, seed, step, B, mu, inv, Xb, tb);
  return hipGetLastError();
}

// Audit sample: A candidates drawn uniformly with replacement (key
// (seed, 3), counter (generation, 0x7FFFFFFF, a, 0)); their genes are copied
// out to be scored by the network and exactly.
__global__ void audit_pick_kernel(const float* cand, int C, int K, const RunState* run,
                                  uint64_t seed, int A, const float* mu, const float* inv,
                                  float* genes, float* x) {
  if (run->stop) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)A * K) return;
  const int a = (int)(i / K), g = (int)(i - (int64_t)a * K);
  const U64x4 r = draw(seed, 3, (uint64_t)run->gen, 0x7FFFFFFFull, (uint64_t)a);
  const int idx = (int)(((r.o0 & 0xFFFFFFFFull) * (uint64_t)C) >> 32);
  const float v = cand[(int64_t)idx * K + g];
  genes[i] = v;
  x[i] = standardize1(v, mu[g], inv[g]);
}

hipError_t launch_audit_pick(const float* cand, int32_t C, int32_t K, const RunState* run,
                             uint64_t seed, int32_t A, const float* mu, const float* inv,
                             float* genes, float* x, hipStream_t s) {
  const int64_t n = (int64_t)A * K;
  hipLaunchKernelGGL(audit_pick_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, cand,
                     C, K, run, seed, A, mu, inv, genes, x);
  return hipGetLastError();
}

// Spearman correlation of the audit's predicted and exact errors (ranks by
// (value, index), Pearson of the ranks), and the screening decision: the
// offspring are screened only when the archive is large enough and the
// correlation reaches rho_min; otherwise the plain offspring are kept.
__global__ __launch_bounds__(1024) void spearman_gate_kernel(const float* pred, const float* exact,
                                                             int A, float rho_min, int min_archive,
                                                             const RunState* run,
                                                             SurrogateState* st) {
  __shared__ float ra[1024], rb[1024];
  __shared__ double sab[1024], saa[1024], sbb[1024];
  if (run->stop) {
    if (threadIdx.x == 0) st->skip = 1;
    return;
  }
  const int i = threadIdx.x;
  if (i < A) {
    const float p = rank_key_value(pred[i]), e = rank_key_value(exact[i]);
    int cp = 0, ce = 0;
    for (int j = 0; j < A; ++j) {
      const float pj = rank_key_value(pred[j]), ej = rank_key_value(exact[j]);
      cp += (pj < p || (pj == p && j < i)) ? 1 : 0;
      ce += (ej < e || (ej == e && j < i)) ? 1 : 0;
    }
    ra[i] = (float)cp;
    rb[i] = (float)ce;
  }
  __syncthreads();
  const double mean = 0.5 * (A - 1);
  const double a = i < A ? ra[i] - mean : 0.0, b = i < A ? rb[i] - mean : 0.0;
  sab[i] = a * b;
  saa[i] = a * a;
  sbb[i] = b * b;
  __syncthreads();
  for (int k = 512; k > 0; k >>= 1) {
    if (i < k) {
      sab[i] += sab[i + k];
      saa[i] += saa[i + k];
      sbb[i] += sbb[i + k];
    }
    __syncthreads();
  }
  if (i == 0) {
    const double den = sqrt(saa[0] * sbb[0]);
    const float rho = den > 0 ? (float)(sab[0] / den) : 0.f;
    st->rho = rho;
    const int use = (st->count >= min_archive && rho >= rho_min) ? 1 : 0;
    st->use = use;
    st->skip = 1 - use;
    st->screened += use;
  }
}

hipError_t launch_spearman_gate(const float* pred, const float* exact, int32_t A, float rho_min,
                                int32_t min_archive, const RunState* run, SurrogateState* st,
                                hipStream_t s) {
  hipLaunchKernelGGL(spearman_gate_kernel, dim3(1), dim3(1024), 0, s, pred, exact, A, rho_min,
                     min_archive, run, st);
  return hipGetLastError();
}

// Rank of every value by (value, index).  Each workgroup bitonic-sorts one
// chunk of kSortChunk keys in LDS (padding keys ~0 sort last and are larger
// than any real key); then each value's rank is the sum over chunks of the
// number of keys below its own, found by binary search.  Keys are unique, so
// the ranks are a permutation of 0..n-1.
__global__ __launch_bounds__(1024) void chunk_sort_kernel(const float* v, int n, uint64_t* sorted,
                                                          const int32_t* skip) {
  __shared__ uint64_t keys[kSortChunk];
  if (skip && *skip) return;
  const int base = blockIdx.x * kSortChunk;
  for (int j = threadIdx.x; j < kSortChunk; j += blockDim.x) {
    const int e = base + j;
    keys[j] = e < n ? rank_key(v[e], e) : ~0ull;
  }
  __syncthreads();
  for (int k = 2; k <= kSortChunk; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < kSortChunk / 2; t += blockDim.x) {
        const int lo = 2 * t - (t & (j - 1));     // partner index lo + j has bit j set
        const uint64_t a = keys[lo], b = keys[lo + j];
        if ((a > b) == ((lo & k) == 0)) {
          keys[lo] = b;
          keys[lo + j] = a;
        }
      }
      __syncthreads();
    }
  }
  for (int j = threadIdx.x; j < kSortChunk; j += blockDim.x) sorted[base + j] = keys[j];
}

__global__ void merge_rank_kernel(const float* v, int n, const uint64_t* sorted, int n_chunks,
                                  int32_t* rank, const int32_t* skip) {
  if (skip && *skip) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const uint64_t key = rank_key(v[e], e);
  int r = 0;
  for (int c = 0; c < n_chunks; ++c) {
    const uint64_t* s = sorted + (int64_t)c * kSortChunk;
    int lo = 0, hi = kSortChunk;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (s[mid] < key) lo = mid + 1;
      else hi = mid;
    }
    r += lo;
  }
  rank[e] = r;
}

hipError_t launch_rank_sorted(const float* v, int32_t n, uint64_t* sorted, int32_t* rank,
                              const int32_t* skip, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int nc = sort_chunks(n);
  hipLaunchKernelGGL(chunk_sort_kernel, dim3(nc), dim3(1024), 0, s, v, n, sorted, skip);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(merge_rank_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, v, n,
                     sorted, nc, rank, skip);
  return hipGetLastError();
}

// Next population's offspring slots: with screening, candidate i goes to
// slot E + rank_i when its predicted rank is below P - E; without, the
// first P - E candidates (the plain offspring) go to slots E..P-1.
__global__ void gather_next_kernel(const float* cand, const int32_t* rank, int C, int K, int E,
                                   int P, const RunState* run, const SurrogateState* st,
                                   float* pop0, float* pop1) {
  if (run->stop) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)C * K) return;
  const int c = (int)(i / K), g = (int)(i - (int64_t)c * K);
  int slot = -1;
  if (st->use) {
    if (rank[c] < P - E) slot = E + rank[c];
  } else if (c < P - E) {
    slot = E + c;
  }
  if (slot < 0) return;
  float* pop = (run->gen & 1) ? pop1 : pop0;
  pop[(int64_t)slot * K + g] = cand[i];
}

hipError_t launch_gather_next(const float* cand, const int32_t* rank, int32_t C, int32_t K,
                              int32_t E, int32_t P, const RunState* run, const SurrogateState* st,
                              float* pop0, float* pop1, hipStream_t s) {
  const int64_t n = (int64_t)C * K;
  hipLaunchKernelGGL(gather_next_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, cand,
                     rank, C, K, E, P, run, st, pop0, pop1);
  return hipGetLastError();
}

}  // namespace game
