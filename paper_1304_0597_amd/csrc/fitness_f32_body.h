// The float32 fitness of one chromosome tile over one pattern split: the
// body shared by the single-run kernel (fitness_f32.hip) and the batched
// persistent kernel (batch.hip).  See fitness_f32.hip for the design.
#pragma once

#include <utility>

#include "basis.h"
#include "common.h"

namespace game {

typedef float f32x16 __attribute__((ext_vector_type(16)));

// Squared residual (MSE, RMSE) or its thresholded form (TMSE, Eq. 10):
// mode 2 keeps it when |r| > R, mode 3 when r^2 > R.
template <int MODE>
__device__ __forceinline__ float error_term(float v, float R) {
  const float e = v * v;
  if constexpr (MODE == 2) return fabsf(v) > R ? e : 0.f;
  if constexpr (MODE == 3) return e > R ? e : 0.f;
  return e;
}

// Tile range [split's tiles] x chromosome tile ctile of the launch described
// by a; writes a.partial[split * ld_partial + chromosome].  genes: the
// chromosomes being scored; lds: the workgroup's dynamic LDS.
template <int BASIS, int D>
__device__ __forceinline__ void fitness_f32_block(const FitArgs& a, const float* __restrict__ genes,
                                                  int split, int ctile, float* lds) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int m = lane & 31;
  const int h = lane >> 5;
  const int c0 = ctile * kTileCols;

  const int ppc = a.pairs_per_chunk;
  const int SC = ppc * D;          // K-steps per chunk
  const int WS = 2 * SC + 1;       // LDS row stride in floats (odd)
  const int K = a.K;

  float w0[2];
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    const int n = c0 + cb * 32 + m;
    w0[cb] = n < a.n_chrom ? genes[(int64_t)n * K] : 0.f;
  }

  // Stage the genes of feature pairs [chunk*ppc, chunk*ppc + ppc) of this
  // chromosome tile: lds[c*WS + half*SC + qq*D + (j-1)].
  auto stage = [&](int chunk) {
    const int g0 = chunk * ppc * 2 * D;       // first expansion gene of the chunk
    const int span = 2 * SC;
    for (int idx = threadIdx.x; idx < kTileCols * span; idx += kFitThreads) {
      const int c = idx / span;
      const int g = idx - c * span;           // offset within the chunk
      const int u_off = g / D;
      const int j = g - u_off * D;
      const int u = chunk * ppc * 2 + u_off;
      const int n = c0 + c;
      float v = 0.f;
      if (n < a.n_chrom && u < a.U) v = genes[(int64_t)n * K + 1 + g0 + g];
      lds[c * WS + (u_off & 1) * SC + (u_off >> 1) * D + j] = v;
    }
  };

  if (a.n_chunks == 1) {
    stage(0);
    __syncthreads();
  }

  double acc64[2] = {0.0, 0.0};
  const int64_t NP = a.NP;
  const int N = a.N;
  const int tile_begin = split * a.tiles_per_split;
  const int tile_end = min(tile_begin + a.tiles_per_split, a.n_tiles);

  // x of sub-feature pair q for this lane's two rows (0 outside the data).
  auto load_x = [&](int64_t row0, int q, float (&xo)[2]) {
    const int u = 2 * q + h;
    const int f = BASIS == 3 ? q : u;
    const bool fvalid = BASIS == 3 ? true : (u < a.U);
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      const int64_t r = row0 + rb * 32 + m;
      xo[rb] = (r < NP && fvalid) ? a.X[r * N + f] : 0.f;
    }
  };

  float xn[2] = {0.f, 0.f};
  if (tile_begin < tile_end) load_x((int64_t)tile_begin * kTileRows + wave * 64, 0, xn);

  for (int tile = tile_begin; tile < tile_end; ++tile) {
    const int64_t row0 = (int64_t)tile * kTileRows + wave * 64;
    // One target per lane (the wave's 64 rows); the epilogue redistributes
    // them across lanes, so the load's latency hides behind the K loop.
    const float t_lane = a.t[row0 + lane < NP ? row0 + lane : NP - 1];
    // Accumulators start at zero (an inline constant, nothing to keep live
    // across tiles); the bias joins in the epilogue.
    f32x16 acc[2][2];
    acc[0][0] = f32x16{};
    acc[0][1] = f32x16{};
    acc[1][0] = f32x16{};
    acc[1][1] = f32x16{};

    for (int chunk = 0; chunk < a.n_chunks; ++chunk) {
      if (a.n_chunks > 1) {
        __syncthreads();
        stage(chunk);
        __syncthreads();
      }
      const int q_begin = chunk * ppc;
      const int q_end = min(q_begin + ppc, a.Q);
      for (int q = q_begin; q < q_end; ++q) {
        float x[2] = {xn[0], xn[1]};
        // prefetch the next pair, or the first pair of the next tile
        if (q + 1 < a.Q) load_x(row0, q + 1, xn);
        else if (tile + 1 < tile_end) load_x(row0 + kTileRows, 0, xn);
        Recur<BASIS> rc[2];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) rc[rb].seed(x[rb], h);
        const float* wl = lds + m * WS + h * SC + (q - q_begin) * D;
        // One K-step per degree: two MFMA columns x two row blocks, then the
        // recurrence moves every lane's A value to the next degree.
        auto kstep = [&](auto jc) {
          constexpr int j = decltype(jc)::value;
          const float b0 = wl[j];
          const float b1 = wl[32 * WS + j];
#pragma unroll
          for (int rb = 0; rb < 2; ++rb) {
            acc[rb][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(rc[rb].cur, b0, acc[rb][0], 0, 0, 0);
            acc[rb][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(rc[rb].cur, b1, acc[rb][1], 0, 0, 0);
          }
          if constexpr (j + 1 < D) {
#pragma unroll
            for (int rb = 0; rb < 2; ++rb) rc[rb].template advance<j + 1>(x[rb]);
          }
        };
        [&]<int... J>(std::integer_sequence<int, J...>) {
          (kstep(std::integral_constant<int, J>{}), ...);
        }(std::make_integer_sequence<int, D>{});
      }
    }

    // Epilogue: residual Out - t, squared (or thresholded), summed over the
    // lane's 32 rows.  Accumulator register i of row block rb holds row
    // rb*32 + 8*(i/4) + 4*h + i%4 of the wave's 64 rows.
    const bool full = row0 + 64 <= NP;
    float s[2] = {0.f, 0.f};
    auto epilogue = [&](auto mode_c) {
      constexpr int mode = decltype(mode_c)::value;
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int rl = rb * 32 + 8 * (i >> 2) + 4 * h + (i & 3);
          const float tv = __shfl(t_lane, rl);
          float e0 = error_term<mode>((acc[rb][0][i] + w0[0]) - tv, a.R);
          float e1 = error_term<mode>((acc[rb][1][i] + w0[1]) - tv, a.R);
          if (!full) {
            const bool ok = row0 + rl < NP;
            e0 = ok ? e0 : 0.f;
            e1 = ok ? e1 : 0.f;
          }
          s[0] += e0;
          s[1] += e1;
        }
      }
    };
    if (a.error_fn == 2) epilogue(std::integral_constant<int, 2>{});
    else if (a.error_fn == 3) epilogue(std::integral_constant<int, 3>{});
    else epilogue(std::integral_constant<int, 0>{});
    acc64[0] += (double)s[0];
    acc64[1] += (double)s[1];
  }

  // Combine the two lane halves (same chromosome, different rows), then the
  // four waves, in a fixed order.
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
    a.partial[(int64_t)split * a.ld_partial + c0 + c] = v;
  }
}


}  // namespace game
