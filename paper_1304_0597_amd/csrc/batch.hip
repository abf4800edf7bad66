// Batched form: the fitness of many independent GAME runs of uneven sizes
// in one persistent launch.
//
// The work of a generation is a list of items (run, 64-chromosome tile,
// pattern split), ordered by decreasing cost on the host.  A fixed grid of
// workgroups drains the list through an atomic queue head; each item is the
// float32 fitness computation of that run's tile over that split (the same
// contraction and epilogue as the single-run float32 kernel, with the
// degree and basis read from the run's descriptor), and writes its float64
// partial sums to the run's own partial array.  Which workgroup takes which
// item does not affect any result: every item owns its output slots and the
// per-run finish sums them in a fixed order.  Every workgroup leaves the
// loop once the queue head passes the last item.
#include "common.h"

namespace game {

typedef float f32x16 __attribute__((ext_vector_type(16)));

// Legendre recurrence coefficients (2J+1)/(J+1) and J/(J+1), J = 1..16, the
// same float values the fixed-degree kernels fold in at compile time.
#define GAME_LEG(J) float(2 * (J) + 1) / float((J) + 1)
#define GAME_LEGB(J) float(J) / float((J) + 1)
__constant__ float kLegA[17] = {0.f, GAME_LEG(1), GAME_LEG(2), GAME_LEG(3), GAME_LEG(4),
                                GAME_LEG(5), GAME_LEG(6), GAME_LEG(7), GAME_LEG(8), GAME_LEG(9),
                                GAME_LEG(10), GAME_LEG(11), GAME_LEG(12), GAME_LEG(13),
                                GAME_LEG(14), GAME_LEG(15), GAME_LEG(16)};
__constant__ float kLegB[17] = {0.f, GAME_LEGB(1), GAME_LEGB(2), GAME_LEGB(3), GAME_LEGB(4),
                                GAME_LEGB(5), GAME_LEGB(6), GAME_LEGB(7), GAME_LEGB(8),
                                GAME_LEGB(9), GAME_LEGB(10), GAME_LEGB(11), GAME_LEGB(12),
                                GAME_LEGB(13), GAME_LEGB(14), GAME_LEGB(15), GAME_LEGB(16)};
#undef GAME_LEG
#undef GAME_LEGB

// Recurrences with a runtime degree index (see basis.h for the formulas).
struct RRecur {
  float prev, cur, m2;
  template <int BASIS>
  __device__ void seed(float x, int half) {
    if constexpr (BASIS == 3) {
      float s, c;
      sincosf(x, &s, &c);
      prev = half ? 0.f : 1.f;
      cur = half ? s : c;
      m2 = 2.f * c;
    } else {
      prev = 1.f;
      cur = x;
      m2 = 2.f * x;
    }
  }
  template <int BASIS>
  __device__ void advance(int J, float x) {
    if constexpr (BASIS == 1) {
      const float n = fmaf(kLegA[J] * x, cur, -kLegB[J] * prev);
      prev = cur;
      cur = n;
    } else if constexpr (BASIS == 2) {
      cur *= x;
    } else {
      const float n = fmaf(m2, cur, -prev);
      prev = cur;
      cur = n;
    }
  }
};

template <int BASIS>
__device__ void batch_item(const BatchRun& run, int ctile, int split, float* lds) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int m = lane & 31;
  const int h = lane >> 5;
  const int D = run.D;
  const int K = run.K;
  const int U = run.U;
  const int Q = run.Q;
  const int n_chrom = run.P;
  const int64_t NP = run.NP;
  const int N = run.N;
  const float* __restrict__ X = run.X;
  const float* __restrict__ t = run.t;
  const float* __restrict__ genes = (run.state->gen & 1) ? run.pop1 : run.pop0;
  const int c0 = ctile * kTileCols;
  const int ppc = run.pairs_per_chunk;
  const int n_chunks = run.n_chunks;
  const int SC = ppc * D;
  const int WS = 2 * SC + 1;

  float w0[2];
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    const int n = c0 + cb * 32 + m;
    w0[cb] = n < n_chrom ? genes[(int64_t)n * K] : 0.f;
  }

  auto stage = [&](int chunk) {
    const int g0 = chunk * ppc * 2 * D;
    const int span = 2 * SC;
    for (int idx = threadIdx.x; idx < kTileCols * span; idx += kFitThreads) {
      const int c = idx / span;
      const int g = idx - c * span;
      const int u_off = g / D;
      const int j = g - u_off * D;
      const int u = chunk * ppc * 2 + u_off;
      const int n = c0 + c;
      float v = 0.f;
      if (n < n_chrom && u < U) v = genes[(int64_t)n * K + 1 + g0 + g];
      lds[c * WS + (u_off & 1) * SC + (u_off >> 1) * D + j] = v;
    }
  };
  if (n_chunks == 1) {
    stage(0);
    __syncthreads();
  }

  auto load_x = [&](int64_t row0, int q, float (&xo)[2]) {
    const int u = 2 * q + h;
    const int f = BASIS == 3 ? q : u;
    const bool fvalid = BASIS == 3 ? true : (u < U);
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      const int64_t r = row0 + rb * 32 + m;
      xo[rb] = (r < NP && fvalid) ? X[r * N + f] : 0.f;
    }
  };

  double acc64[2] = {0.0, 0.0};
  const int tile_begin = split * run.tiles_per_split;
  const int tile_end = min(tile_begin + run.tiles_per_split, run.n_tiles);
  float xn[2] = {0.f, 0.f};
  if (tile_begin < tile_end) load_x((int64_t)tile_begin * kTileRows + wave * 64, 0, xn);
  const bool key_sq = run.error_fn == 3;
  const bool tube = run.error_fn == 2 || run.error_fn == 3;
  const float thr = run.R;

  for (int tile = tile_begin; tile < tile_end; ++tile) {
    const int64_t row0 = (int64_t)tile * kTileRows + wave * 64;
    const float t_lane = t[row0 + lane < NP ? row0 + lane : NP - 1];
    f32x16 acc[2][2];
    acc[0][0] = f32x16{};
    acc[0][1] = f32x16{};
    acc[1][0] = f32x16{};
    acc[1][1] = f32x16{};
    for (int chunk = 0; chunk < n_chunks; ++chunk) {
      if (n_chunks > 1) {
        __syncthreads();
        stage(chunk);
        __syncthreads();
      }
      const int q_begin = chunk * ppc;
      const int q_end = min(q_begin + ppc, Q);
      for (int q = q_begin; q < q_end; ++q) {
        float x[2] = {xn[0], xn[1]};
        if (q + 1 < Q) load_x(row0, q + 1, xn);
        else if (tile + 1 < tile_end) load_x(row0 + kTileRows, 0, xn);
        RRecur rc[2];
        rc[0].seed<BASIS>(x[0], h);
        rc[1].seed<BASIS>(x[1], h);
        const float* wl = lds + m * WS + h * SC + (q - q_begin) * D;
        float b0 = wl[0], b1 = wl[32 * WS];
        for (int j = 0; j < D; ++j) {
          const int jn = j + 1 < D ? j + 1 : j;
          const float nb0 = wl[jn], nb1 = wl[32 * WS + jn];
#pragma unroll
          for (int rb = 0; rb < 2; ++rb) {
            acc[rb][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(rc[rb].cur, b0, acc[rb][0], 0, 0, 0);
            acc[rb][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(rc[rb].cur, b1, acc[rb][1], 0, 0, 0);
          }
          rc[0].advance<BASIS>(j + 1, x[0]);
          rc[1].advance<BASIS>(j + 1, x[1]);
          b0 = nb0;
          b1 = nb1;
        }
      }
    }
    const bool full = row0 + 64 <= NP;
    float s[2] = {0.f, 0.f};
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int rl = rb * 32 + 8 * (i >> 2) + 4 * h + (i & 3);
        const float tv = __shfl(t_lane, rl);
        const bool ok = full || (row0 + rl < NP);
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          const float v = (acc[rb][cb][i] + w0[cb]) - tv;
          const float e = v * v;
          const float key = key_sq ? e : fabsf(v);
          const float kept = tube ? (key > thr ? e : 0.f) : e;
          s[cb] += ok ? kept : 0.f;
        }
      }
    }
    acc64[0] += (double)s[0];
    acc64[1] += (double)s[1];
  }

#pragma unroll
  for (int cb = 0; cb < 2; ++cb) acc64[cb] += __shfl_xor(acc64[cb], 32);
  __syncthreads();
  double* red = reinterpret_cast<double*>(lds);
  if (h == 0) {
    red[wave * 64 + m] = acc64[0];
    red[wave * 64 + 32 + m] = acc64[1];
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int c = threadIdx.x;
    const double v = ((red[c] + red[64 + c]) + red[128 + c]) + red[192 + c];
    run.partial[(int64_t)split * run.ld_partial + c0 + c] = v;
  }
}

__global__ __launch_bounds__(kFitThreads, 2) void fitness_batch_kernel(BatchArgs a) {
  extern __shared__ float lds[];
  __shared__ int item_sh;
  for (;;) {
    __syncthreads();  // the previous item is done with item_sh and LDS
    if (threadIdx.x == 0) item_sh = atomicAdd(a.counter, 1);
    __syncthreads();
    const int it = item_sh;
    if (it >= a.n_items) break;
    const BatchItem w = a.items[it];
    const BatchRun& run = a.runs[w.run];
    const int stopped = run.state->stop;
    if (w.ctile == 0 && w.split == 0 && threadIdx.x == 0) run.state->stop_seen = stopped;
    if (stopped) continue;
    switch (run.basis) {
      case 0: batch_item<0>(run, w.ctile, w.split, lds); break;
      case 1: batch_item<1>(run, w.ctile, w.split, lds); break;
      case 2: batch_item<2>(run, w.ctile, w.split, lds); break;
      default: batch_item<3>(run, w.ctile, w.split, lds); break;
    }
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
