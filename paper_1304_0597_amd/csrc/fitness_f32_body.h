// The float32 fitness of one chromosome tile over one pattern split: the
// body shared by the single-run kernel (fitness_f32.hip) and the batched
// persistent kernel (batch.hip).  See fitness_f32.hip for the design.
#pragma once

#include <utility>

#include "basis.h"
#include "common.h"

namespace game {

typedef float f32x16 __attribute__((ext_vector_type(16)));

// s plus the squared residual v (MSE, RMSE: one fused multiply-add) or its
// thresholded form (TMSE, Eq. 10: mode 2 keeps it when |v| > R, mode 3 when
// v^2 > R; square and sum rounded separately).  Every rounding is spelled
// out, so each instance of the body (single-run and batched) sums the same
// bits whatever the compiler would contract.
template <int MODE>
__device__ __forceinline__ float add_error_term(float s, float v, float R) {
  if constexpr (MODE == 2 || MODE == 3) {
    const float e = __fmul_rn(v, v);
    const bool keep = MODE == 2 ? fabsf(v) > R : e > R;
    return __fadd_rn(s, keep ? e : 0.f);
  }
  return __builtin_fmaf(v, v, s);
}

// A recurrence chain that yields zero at every degree: for rows past the
// data, so that their accumulators end at exactly zero.
template <class R>
__device__ __forceinline__ void zero_chain(R& r, bool keep) {
  r.cur = keep ? r.cur : 0.f;
  if constexpr (requires { r.prev; }) r.prev = keep ? r.prev : 0.f;
}

// Wave-uniform copies (readfirstlane) of launch parameters.
__device__ __forceinline__ int32_t uniform(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uniform(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ int64_t uniform(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <class T>
__device__ __forceinline__ T* uniform(T* p) {
  return reinterpret_cast<T*>(uniform((int64_t)reinterpret_cast<uintptr_t>(p)));
}

// A pointer to global memory as such: its loads are global_load rather than
// flat_load, whose completion an LDS wait would also have to cover.
typedef const float __attribute__((address_space(1)))* gptr_f32;
__device__ __forceinline__ gptr_f32 global_f32(const float* p) { return (gptr_f32)p; }

// Waves per workgroup of the body with CB 32-column blocks per wave: four
// for 32- and 64-chromosome tiles, eight for 128-chromosome tiles (waves 0-3
// take the even row tiles of the split and 4-7 the odd ones, two per SIMD).
__host__ __device__ constexpr int fit_waves(int cb) { return cb == 4 ? 8 : 4; }

// Tile range [split's tiles] x chromosome tile ctile (32*CB chromosomes,
// the first one ctile * 32*CB) of the launch described by a_in; writes
// a.partial[split * ld_partial + chromosome].  Each wave takes RB/2 consecutive 256-row tiles at a time
// (its 64-row slice of each: RB 32-row blocks).  genes: the chromosomes
// being scored; lds: the workgroup's dynamic LDS.  D is the degree.  BASIS
// is the expansion family (kTrigTable: the trigonometric one seeded from
// the stored (cos x, sin x) table a_in.cs instead of sincosf in every tile).
template <int BASIS, int D, int CB = 2, int RB = 2>
__device__ __forceinline__ void fitness_f32_block(const FitArgs& a_in, const float* __restrict__ genes,
                                                  int split, int ctile, float* lds) {
  // The parameters the body uses, read once into scalar registers (so that
  // no store in the loops can be taken to alias them and force reloads).
  FitArgs a;
  a.X = uniform(a_in.X);
  a.t = uniform(a_in.t);
  a.partial = uniform(a_in.partial);
  a.NP = uniform(a_in.NP);
  a.N = uniform(a_in.N);
  a.K = uniform(a_in.K);
  a.n_chrom = uniform(a_in.n_chrom);
  a.U = uniform(a_in.U);
  a.Q = uniform(a_in.Q);
  a.pairs_per_chunk = uniform(a_in.pairs_per_chunk);
  a.n_chunks = uniform(a_in.n_chunks);
  a.ld_partial = uniform(a_in.ld_partial);
  a.tiles_per_split = uniform(a_in.tiles_per_split);
  a.n_tiles = uniform(a_in.n_tiles);
  a.error_fn = uniform(a_in.error_fn);
  a.R = uniform(a_in.R);
  constexpr bool kTable = BASIS == kTrigTable;
  constexpr int FAM = kTable ? 3 : BASIS;   // expansion family
  static_assert(FAM >= 0 && FAM <= 3, "compile-time expansion family");
  a.cs = kTable ? uniform(a_in.cs) : nullptr;
  static_assert(D >= 1 && D <= kMaxDegree, "compile-time degree");
  constexpr int Dv = D;
  constexpr bool trig = FAM == 3;
  genes = uniform(genes);
  split = uniform(split);
  ctile = uniform(ctile);
  lds = uniform(lds);
  static_assert(CB == 1 || CB == 2 || CB == 4, "32-, 64- or 128-chromosome tiles");
  constexpr int NW = fit_waves(CB);   // waves per workgroup
  constexpr int TS = NW / 4;          // tile streams (wave groups)
  static_assert(RB == 2 || RB == 4, "one or two 256-row tiles per wave");
  constexpr int TPW = RB / 2;         // consecutive row tiles per wave
  constexpr int STEP = TS * TPW;      // row tiles per step of the workgroup
  constexpr int kCols = 32 * CB;      // chromosomes per tile
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wq = wave & 3;            // 64-row slice of a tile
  const int wg = TS == 1 ? 0 : wave >> 2;  // tile stream
  const int m = lane & 31;
  const int h = lane >> 5;
  const int c0 = ctile * kCols;

  const int ppc = a.pairs_per_chunk;
  const int SC = ppc * Dv;         // K-steps per chunk
  const int WS = 2 * SC + 1;       // LDS row stride in floats (odd)
  const int BUF = kCols * WS;      // floats per gene buffer
  const int nk = (2 * SC + 63) >> 6;  // 64-gene pieces of a row
  const int K = a.K;
  const int wave_u = __builtin_amdgcn_readfirstlane(wave);

  float w0[CB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    const int n = c0 + cb * 32 + m;
    w0[cb] = n < a.n_chrom ? global_f32(genes)[(int64_t)n * K] : 0.f;
  }

  // Issue the copy of the chunk's genes (sub-features [u0, u0 + 2 ppc)) into
  // buffer buf: row c = genes 1 + u0*D ... of chromosome c0 + c, canonical
  // order.  Rows past the population repeat the last chromosome (their sums
  // are never read).  Gene slots of a sub-feature past U (the odd half of the
  // last pair) are zeroed: that lane's expansion of x = 0 is not zero.  The
  // copy has landed once this wave's vmcnt reaches zero.
  auto stage_issue = [&](int chunk, int buf) {
    const int u0 = chunk * ppc * 2;
    const int rem = a.U - u0;
    const int valid = min(2 * SC, rem * Dv);
    float* dst0 = lds + buf * BUF;
    const float* src0 = genes + 1 + u0 * Dv + lane;
    for (int i = wave_u; i < kCols * nk; i += NW) {
      const int c = i / nk;
      const int k = i - c * nk;
      const int n = min(c0 + c, a.n_chrom - 1);
      if (k * 64 + lane < valid)
        __builtin_amdgcn_global_load_lds(
            (const void*)(src0 + (int64_t)n * K + k * 64),
            (__attribute__((address_space(3))) void*)(dst0 + c * WS + k * 64), 4, 0, 0);
    }
    if ((rem & 1) && rem < 2 * ppc) {
      for (int idx = threadIdx.x; idx < kCols * Dv; idx += 64 * NW) {
        const int c = idx / Dv;
        dst0[c * WS + rem * Dv + (idx - c * Dv)] = 0.f;
      }
    }
  };

  if (a.n_chunks == 1) {
    stage_issue(0, 0);
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's copies landed
    __syncthreads();
  }

  double acc64[CB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) acc64[cb] = 0.0;
  const int64_t NP = a.NP;
  const int N = a.N;
  const int tile_begin = split * a.tiles_per_split;
  const int tile_end = min(tile_begin + a.tiles_per_split, a.n_tiles);

  // x of sub-feature pair q for this lane's two rows (0 outside the data);
  // from the stored trig table, cos x into xo and sin x into so instead.
  // Row of block rb of the wave whose first tile is `tile`: blocks 2i and
  // 2i+1 are the wave's 64-row slice of tile + i.
  auto row_of = [&](int tile, int rb) -> int64_t {
    return (int64_t)(tile + rb / 2) * kTileRows + wq * 64 + (rb & 1) * 32 + m;
  };
  auto load_x = [&](int tile, int q, float (&xo)[RB], float (&so)[RB]) {
    if constexpr (kTable) {
      typedef float f32x2 __attribute__((ext_vector_type(2)));
      typedef const f32x2 __attribute__((address_space(1)))* gptr_f32x2;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        const int64_t r = row_of(tile, rb);
        f32x2 v = {0.f, 0.f};
        if (r < NP) v = ((gptr_f32x2)a.cs)[r * N + q];
        xo[rb] = v.x;
        so[rb] = v.y;
      }
      return;
    }
    const int u = 2 * q + h;
    const int f = trig ? q : u;
    const bool fvalid = trig ? true : (u < a.U);
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int64_t r = row_of(tile, rb);
      xo[rb] = (r < NP && fvalid) ? global_f32(a.X)[r * N + f] : 0.f;
    }
  };

  float xn[RB], sn[RB];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) xn[rb] = sn[rb] = 0.f;
  if (tile_begin + wg * TPW < tile_end) load_x(tile_begin + wg * TPW, 0, xn, sn);
  // Chunked genes: stage index st runs over (tile, chunk) in loop order and
  // uses buffer st & 1.
  int st = 0;
  if (a.n_chunks > 1 && tile_begin < tile_end) stage_issue(0, 0);

  // Every wave takes the same number of steps of STEP tiles.  A wave whose
  // stream has no tile left in the last step leaves at once when the genes
  // are staged once, and otherwise still joins the staging barriers of each
  // chunk but computes nothing.
  const int n_steps = (tile_end - tile_begin + STEP - 1) / STEP;
  for (int step = 0; step < n_steps; ++step) {
    const int tile = tile_begin + step * STEP + wg * TPW;   // the wave's first tile
    const bool active = TS == 1 || tile < tile_end;   // one stream: every step has its tile
    if (!active && a.n_chunks == 1) break;
    // Rows past the data take a zero A operand in every K-step (bias step
    // included), so their residuals are exactly zero and the epilogue needs
    // no row mask.
    bool row_ok[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
      row_ok[rb] = (RB == 2 || tile + rb / 2 < tile_end) && row_of(tile, rb) < NP;
    // Minus the targets of this lane's rows (0 past the data); they join
    // with the bias in a last K-step, so the load's latency hides behind the
    // K loop.
    float nt[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int64_t r = row_of(tile, rb);
      nt[rb] = active && row_ok[rb] ? -global_f32(a.t)[r] : 0.f;
    }
    // Accumulators start at zero (an inline constant, nothing to keep live
    // across tiles).
    f32x16 acc[RB][CB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) acc[rb][cb] = f32x16{};

    for (int chunk = 0; chunk < a.n_chunks; ++chunk) {
      const float* wbuf = lds;
      if (a.n_chunks > 1) {
        // Every wave's copy of this chunk has landed and every wave is done
        // with the other buffer: start the copy of the next stage into it.
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
        __syncthreads();
        if (chunk + 1 < a.n_chunks) stage_issue(chunk + 1, (st + 1) & 1);
        else if (step + 1 < n_steps) stage_issue(0, (st + 1) & 1);
        wbuf = lds + (st & 1) * BUF;
        ++st;
      }
      if (!active) continue;
      const int q_begin = chunk * ppc;
      const int q_end = min(q_begin + ppc, a.Q);
      for (int q = q_begin; q < q_end; ++q) {
        float x[RB], sx[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          x[rb] = xn[rb];
          sx[rb] = sn[rb];
        }
        // prefetch the next pair, or the first pair of the next tile
        if (q + 1 < a.Q) load_x(tile, q + 1, xn, sn);
        else if (tile + STEP < tile_end) load_x(tile + STEP, 0, xn, sn);
        Recur<FAM> rc[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          if constexpr (kTable) {
            rc[rb].seed_cs(x[rb], sx[rb], h);
          } else {
            rc[rb].seed(x[rb], h);
          }
          zero_chain(rc[rb], row_ok[rb]);
        }
        const float* wl = wbuf + m * WS + (2 * (q - q_begin) + h) * Dv;
        // One K-step per degree: CB MFMA columns x two row blocks, then the
        // recurrence moves every lane's A value to the next degree.
        auto kstep = [&](auto jc) {
          constexpr int j = decltype(jc)::value;
          float b[CB];
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) b[cb] = wl[cb * 32 * WS + j];
#pragma unroll
          for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int cb = 0; cb < CB; ++cb)
              acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(rc[rb].cur, b[cb], acc[rb][cb], 0, 0, 0);
          if constexpr (j + 1 < D) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
              rc[rb].template advance<j + 1>(x[rb]);
            }
          }
        };
        [&]<int... J>(std::integer_sequence<int, J...>) {
          (kstep(std::integral_constant<int, J>{}), ...);
        }(std::make_integer_sequence<int, D>{});
      }
    }

    if (!active) continue;
    // Bias and target K-step: lane half 0 multiplies 1 by a0 of its column,
    // half 1 multiplies -t of its row by 1, so the accumulators end at
    // Out - t (0 for rows past the data).
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const float ab = h ? nt[rb] : (row_ok[rb] ? 1.f : 0.f);
#pragma unroll
      for (int cb = 0; cb < CB; ++cb)
        acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x2f32(ab, h ? 1.f : w0[cb], acc[rb][cb], 0, 0, 0);
    }

    // Epilogue: residual Out - t, squared (or thresholded), summed over the
    // lane's 32 rows (register order; accumulator register i of row block rb
    // holds row rb*32 + 8*(i/4) + 4*h + i%4 of the wave's 64 rows).  Rows
    // past the data add exactly zero.
    // One float32 sum per row tile (its two row blocks), added to the
    // float64 running sum tile by tile, so that a tile's sum does not
    // depend on how many tiles a wave takes at once.
    float s[TPW][CB];
#pragma unroll
    for (int tp = 0; tp < TPW; ++tp)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) s[tp][cb] = 0.f;
    auto epilogue = [&](auto mode_c) {
      constexpr int mode = decltype(mode_c)::value;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int i = 0; i < 16; ++i)
#pragma unroll
          for (int cb = 0; cb < CB; ++cb)
            s[rb / 2][cb] = add_error_term<mode>(s[rb / 2][cb], acc[rb][cb][i], a.R);
    };
    if (a.error_fn == 2) epilogue(std::integral_constant<int, 2>{});
    else if (a.error_fn == 3) epilogue(std::integral_constant<int, 3>{});
    else epilogue(std::integral_constant<int, 0>{});
#pragma unroll
    for (int tp = 0; tp < TPW; ++tp)
#pragma unroll
      for (int cb = 0; cb < CB; ++cb) acc64[cb] += (double)s[tp][cb];
  }

  // Combine the two lane halves (same chromosome, different rows), then the
  // waves, in a fixed order.
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) acc64[cb] += __shfl_xor(acc64[cb], 32);
  __syncthreads();
  double* red = reinterpret_cast<double*>(lds);
  if (h == 0) {
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) red[wave * kCols + cb * 32 + m] = acc64[cb];
  }
  __syncthreads();
  if (threadIdx.x < kCols) {
    const int c = threadIdx.x;
    double v = red[c];
#pragma unroll
    for (int w = 1; w < NW; ++w) v += red[w * kCols + c];
    a.partial[(int64_t)split * a.ld_partial + c0 + c] = v;
  }
}


}  // namespace game
