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

__device__ __forceinline__ int count_rank(const uint64_t* keys, int P, int e, uint32_t* cnt) {
  constexpr int parts = kRankThreads / kRankPerBlock;
  const int part = threadIdx.x / kRankPerBlock;
  uint32_t c = 0;
  if (e < P) {
    const uint64_t ke = keys[e];
    const int per = (P + parts - 1) / parts;
    const int j0 = part * per;
    const int j1 = min(j0 + per, P);
    for (int j = j0; j < j1; ++j) c += keys[j] < ke ? 1u : 0u;
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
  for (int i = threadIdx.x; i < n; i += blockDim.x) keys[i] = rank_key(fit[i], i);
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

__device__ __forceinline__ double error_of(const RankArgs& a, int i) {
  double s = 0.0;
  for (int k = 0; k < a.n_splits; ++k) s += a.partial[(int64_t)k * a.ld_partial + i];
  double v = s / (double)a.NP;
  if (a.error_fn == 1) v = sqrt(v);
  if (isnan(v)) v = INFINITY;
  return v;
}

// Evaluation epilogue of one generation: errors from the float64 partials
// (the same fixed-order sums in every workgroup), rank order, best
// chromosome, stop test and the generation counter.  The stop flag that
// decides whether this launch works is the one the generation's fitness
// launch recorded, so a workgroup that sets the flag cannot make another
// workgroup of the same launch skip its share.
__global__ __launch_bounds__(kRankThreads) void finish_rank_kernel(RankArgs a) {
  extern __shared__ uint64_t keys[];
  __shared__ uint32_t cnt[kRankThreads];
  RunState* st = a.state;
  if (st->stop_seen) return;
  const int P = a.P;
  const int lo = blockIdx.x * kRankPerBlock;
  for (int i = threadIdx.x; i < P; i += blockDim.x) {
    const double v = error_of(a, i);
    const float f = (float)v;
    keys[i] = rank_key(f, i);
    if (i >= lo && i < lo + kRankPerBlock) {
      a.fit32[i] = f;
      a.fit64[i] = v;
    }
  }
  __syncthreads();
  const int e = lo + (threadIdx.x % kRankPerBlock);
  const int r = count_rank(keys, P, e, cnt);
  if (r < 0) return;
  a.order[r] = e;
  if (r == 0) {
    const double v = error_of(a, e);
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

hipError_t launch_finish_rank(const RankArgs& a, hipStream_t s) {
  const hipError_t e = allow_lds((const void*)finish_rank_kernel, (size_t)a.P * sizeof(uint64_t));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(finish_rank_kernel, dim3((a.P + kRankPerBlock - 1) / kRankPerBlock),
                     dim3(kRankThreads), (size_t)a.P * sizeof(uint64_t), s, a);
  return hipGetLastError();
}

__global__ void set_state_kernel(RunState* st, int32_t gen, int32_t max_gen, double target,
                                 int32_t reset) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (reset) {
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

__device__ __forceinline__ int tournament(const float* fit, const uint32_t* w, int k, int P) {
  int best = (int)(((uint64_t)w[0] * (uint64_t)P) >> 32);
  float fb = fit_at(fit, best);
  for (int c = 1; c < k; ++c) {
    const int cand = (int)(((uint64_t)w[c] * (uint64_t)P) >> 32);
    const float fc = fit_at(fit, cand);
    if (fc < fb || (fc == fb && cand < best)) {
      best = cand;
      fb = fc;
    }
  }
  return best;
}

constexpr int kMaxTournament = 64;

__global__ __launch_bounds__(256) void ga_next_kernel(GAArgs a) {
  if (a.stop && *a.stop) return;
  int gen;
  const float* __restrict__ pop;
  float* __restrict__ out;
  if (a.gen_ptr) {
    gen = *a.gen_ptr;
    pop = ((gen - 1) & 1) ? a.pop_b : a.pop_a;
    out = (gen & 1) ? a.out_b : a.out_a;
  } else {
    gen = a.generation;
    pop = a.pop_a;
    out = a.out_a;
  }
  const int lane = threadIdx.x & 63;
  const int wid = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int P = a.P, K = a.K, E = a.E;
  const int n_pairs = (P - E + 1) >> 1;
  if (wid < E) {
    const int src = a.elite_mode == 0 ? a.order[0] : a.order[wid];
    for (int g = lane; g < K; g += 64) out[(int64_t)wid * K + g] = pop[(int64_t)src * K + g];
    return;
  }
  const int q = wid - E;
  if (q >= n_pairs) return;

  // selection words for pair q
  uint32_t w[2 * kMaxTournament + 2];
  const int n_words = 2 * a.k + 2;
  for (int b = 0; b * 8 < n_words; ++b) {
    const U64x4 r = draw(a.seed, 1, (uint64_t)gen, (uint64_t)q, (uint64_t)b);
    const uint64_t o[4] = {r.o0, r.o1, r.o2, r.o3};
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int idx = b * 8 + i;
      if (idx < n_words) w[idx] = (i & 1) ? (uint32_t)(o[i >> 1] >> 32) : (uint32_t)o[i >> 1];
    }
  }
  const int p1 = tournament(a.fitness, w, a.k, P);
  const int p2 = tournament(a.fitness, w + a.k, a.k, P);
  const bool cross = (uint64_t)w[2 * a.k] < a.thr_cross;
  const int cut = 1 + (int)(((uint64_t)w[2 * a.k + 1] * (uint64_t)(K - 1)) >> 32);

  const int sa = E + 2 * q, sb = sa + 1;
  const bool has_b = sb < P;
  for (int g = lane; g < K; g += 64) {
    const float x1 = pop[(int64_t)p1 * K + g];
    const float x2 = pop[(int64_t)p2 * K + g];
    const bool sw = cross && g >= cut;
    float ca = sw ? x2 : x1;
    float cb = sw ? x1 : x2;
    {
      const U64x4 r = draw(a.seed, 2, (uint64_t)gen, (uint64_t)sa, (uint64_t)g);
      if ((r.o0 & 0xFFFFFFFFull) < a.thr_mut)
        ca = clamp_unit(__fadd_rn(ca, __fmul_rn(a.sigma, gauss12(r))));
    }
    out[(int64_t)sa * K + g] = ca;
    if (has_b) {
      const U64x4 r = draw(a.seed, 2, (uint64_t)gen, (uint64_t)sb, (uint64_t)g);
      if ((r.o0 & 0xFFFFFFFFull) < a.thr_mut)
        cb = clamp_unit(__fadd_rn(cb, __fmul_rn(a.sigma, gauss12(r))));
      out[(int64_t)sb * K + g] = cb;
    }
  }
}

hipError_t launch_ga_next(const GAArgs& a, hipStream_t s) {
  const int n_waves = a.E + ((a.P - a.E + 1) >> 1);
  hipLaunchKernelGGL(ga_next_kernel, dim3((n_waves + 3) / 4), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace game
