// Fused GAME fitness with BF16 operands on MFMA (gfx950), FP32 accumulation.
//
// Same contraction as the float32 kernel (Eq. 2 over NP patterns, then the
// error of Eqs. 3-5/10), with the expansion values and the genes rounded to
// bfloat16 (round to nearest even) and fed to v_mfma_f32_32x32x16_bf16;
// products accumulate in float32.  The bias gene and the target stay exact:
// one extra K-step multiplies the three-part bfloat16 splits of a_0 and of
// -t_k (hi + mid + lo reproduces a float32 exactly) by ones, so the
// accumulator ends at Out - t and the epilogue only squares and sums.  Squared
// residuals are summed in float32 per tile and the tile sums are added with
// Neumaier compensation, so the reduction over a million patterns adds no
// error beyond the per-tile float32 sums.
//
// Operand layout: in a K-step each lane supplies 8 consecutive K values of
// its pattern row (A) and of its chromosome column (B).  The two lane halves
// carry different sub-features, so a lane's 8 values are consecutive members
// phi_j of its own recurrence chains: a group of G sub-features per lane
// half (a multiple of 8 / gcd(d, 8)) fills exactly G*d/8 K-steps and no
// chain is split between lanes.  Genes are staged in LDS in that order as
// bfloat16.
//
// Tiles: a workgroup covers 128 chromosomes; each wave takes 64 patterns (two
// 32-row blocks) of a 256-row tile x 128 chromosomes (four 32-column blocks):
// eight 32x32 accumulators, so each generated A fragment feeds four MFMAs.
// With eight waves (see bf16_waves) waves 0-3 take the even tiles of the
// split and waves 4-7 the odd ones, two waves per SIMD.
//
// Pipelining: within a group, the eight MFMAs of K-step k are issued in
// pairs, each pair followed by the B fragments of K-step k+1 for that column
// block and two of K-step k+1's A values (the last K-step generates the next
// group's first one), with scheduling barriers holding that order.
//
// Features and targets (XL variant, feature count a multiple of 4 and
// 16-byte aligned rows): each wave copies the 64 rows of its next tile from
// HBM straight into its own LDS buffer (global_load_lds_dwordx4, four
// features per lane and instruction; one dword per lane for the targets) as
// soon as it has read the current tile's last features, two groups before
// the tile ends; only the wave's own vmcnt wait guards the buffer.  Other
// shapes load features into registers one group ahead.
#include <utility>

#include "basis.h"
#include "common.h"

namespace game {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int gcd_int(int a, int b) { return b == 0 ? a : gcd_int(b, a % b); }

// Sub-features per lane half in one group: the smallest count whose d values
// fill whole K-steps of 8, repeated until a group spans at least 4 K-steps
// (so the next group's features load, and its first values are generated,
// while this group's MFMAs run), at most 16 - but at most 4 whenever whole
// K-steps allow it (even d), so that the group fits two waves per SIMD (see
// bf16_waves): a second wave per SIMD hides more than the deeper group
// pipeline does (d = 2, 4, 6 ran 1.6, 1.24 and 1.17 times faster so).
constexpr int group_size(int d) {
  const int g0 = 8 / gcd_int(d, 8);
  const int ks0 = g0 * d / 8;
  int r = ks0 >= 4 ? 1 : (4 + ks0 - 1) / ks0;
  while (g0 * r > 16) --r;
  if (g0 <= 4 && g0 * r > 4) r = 4 / g0;
  return g0 * r;
}

// x = p[0] + p[1] + p[2] exactly (three bfloat16 parts, round to nearest
// even, each taking the next 8 significant bits of the remainder).
__device__ __forceinline__ void split3(float x, bf16x8& p) {
  const __bf16 hi = (__bf16)x;
  const float r1 = x - (float)hi;
  const __bf16 mid = (__bf16)r1;
  const __bf16 lo = (__bf16)(r1 - (float)mid);
  p[0] = hi;
  p[1] = mid;
  p[2] = lo;
}

// LDS row stride for one chromosome: 32 bytes per K-step (two lane halves x
// 8 bf16) plus 16 bytes so that rows start 4 banks apart.
__host__ __device__ constexpr int bf16_row_bytes(int ksteps) { return ksteps * 32 + 16; }

// Per-wave LDS bytes of one XL buffer: features [N/4][64 rows][4 floats],
// then the 64 targets.
__host__ __device__ constexpr int xl_buffer_bytes(int n_features) {
  return (n_features / 4) * 64 * 16 + 64 * 4;
}

// Waves per workgroup.  Eight (two per SIMD, 256 registers each) when a
// group holds at most 4 sub-features per lane half (even degrees): waves 0-3
// take the even tiles of the split and waves 4-7 the odd ones, and one
// wave's vector work and memory waits run under the other wave's MFMAs (for
// d = 2, 4, 6 one 16-byte value that lives across the tile loop goes to
// scratch, reloaded once per tile).  Larger groups (odd degrees) need more
// registers than two waves per SIMD allow and run four waves over
// consecutive tiles.
__host__ __device__ constexpr int bf16_waves(int degree) { return group_size(degree) <= 4 ? 8 : 4; }

template <int BASIS, int D, bool XL>
__global__ __launch_bounds__(64 * bf16_waves(D), 1) void fitness_bf16_kernel(FitArgs a) {
  constexpr int G = group_size(D);         // sub-features per lane half per group
  constexpr int KS = G * D / 8;            // K-steps per group
  constexpr int NW = bf16_waves(D);        // waves per workgroup
  constexpr int NT = 64 * NW;              // threads per workgroup
  constexpr int TS = NW / 4;               // tiles in flight per workgroup (tile stride)
  extern __shared__ __attribute__((aligned(16))) unsigned char lds_raw[];
  if (a.stop) {
    const int32_t stopped = *a.stop;
    if (a.stop_seen && blockIdx.x == 0 && threadIdx.x == 0) *a.stop_seen = stopped;
    if (stopped) return;
  }
  const float* __restrict__ genes = a.genes;
  if (a.gen_sel && (*a.gen_sel & 1)) genes = a.genes_alt;

  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wq = wave & 3;                 // 64-row slice within a tile
  const int wg = wave >> 2;                // tile offset (0..TS-1) this wave takes
  const int m = lane & 31;
  const int h = lane >> 5;

  const int total = gridDim.x;
  const int b = blockIdx.x;
  const int L = a.xcd_remap ? (b & 7) * (total >> 3) + (b >> 3) : b;
  const int split = L / a.n_ctiles;
  const int ctile = L - split * a.n_ctiles;
  constexpr int kCols = 128;
  const int c0 = ctile * kCols;

  const int gpc = a.pairs_per_chunk;       // groups per chunk
  const int ks_chunk = gpc * KS;           // K-steps per chunk
  const int RS = bf16_row_bytes(ks_chunk); // LDS row stride in bytes
  const int K = a.K;

  // B fragments of the bias K-step: lane half 0 carries the split bias of
  // its chromosome, half 1 ones (they multiply the split targets).
  bf16x8 bbias[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    const int n = c0 + cb * 32 + m;
    const float w0 = n < a.n_chrom ? genes[(int64_t)n * K] : 0.f;
    bf16x8 v = {};
    if (h == 0) {
      split3(w0, v);
    } else {
      v[0] = (__bf16)1.f;
      v[1] = (__bf16)1.f;
      v[2] = (__bf16)1.f;
    }
    bbias[cb] = v;
  }

  // Stage groups [chunk*gpc, chunk*gpc + gpc): value p (0..G*D-1) of lane
  // half hh in group g is gene (sub-feature u = 2(g*G + p/D) + hh, degree
  // p%D + 1); it goes to byte (kstep*32 + hh*16 + (p%8)*2) of the row.
  auto stage = [&](int chunk) {
    const int per_row = gpc * 2 * G * D;   // values per chromosome row
    for (int idx = threadIdx.x; idx < kCols * per_row; idx += NT) {
      const int c = idx / per_row;
      const int r = idx - c * per_row;
      const int gl = r / (2 * G * D);      // group within the chunk
      const int r2 = r - gl * (2 * G * D);
      const int hh = r2 / (G * D);
      const int p = r2 - hh * (G * D);
      const int qi = (chunk * gpc + gl) * G + p / D;
      const int j = p % D;
      const int u = 2 * qi + hh;
      const int n = c0 + c;
      float v = 0.f;
      if (n < a.n_chrom && u < a.U) v = genes[(int64_t)n * K + 1 + u * D + j];
      const int ks = gl * KS + p / 8;
      __bf16* dst = reinterpret_cast<__bf16*>(lds_raw + c * RS + ks * 32 + hh * 16) + (p & 7);
      *dst = (__bf16)v;
    }
  };

  if (a.n_chunks == 1) {
    stage(0);
    __syncthreads();
  }

  // Neumaier-compensated running sums of the per-tile float32 sums.
  float sum[4] = {0.f, 0.f, 0.f, 0.f}, comp[4] = {0.f, 0.f, 0.f, 0.f};
  const int64_t NP = a.NP;
  const int N = a.N;
  const int tile_begin = split * a.tiles_per_split;
  const int tile_end = min(tile_begin + a.tiles_per_split, a.n_tiles);

  // x of the G sub-features of group g for this lane's two rows.
  auto load_x = [&](int64_t row0, int g, float (&xo)[2][G]) {
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const int qi = g * G + i;
      const int u = 2 * qi + h;
      const int f = BASIS == 3 ? qi : u;
      const bool fvalid = BASIS == 3 ? (qi < N) : (u < a.U);
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        const int64_t r = row0 + rb * 32 + m;
        xo[rb][i] = (r < NP && fvalid) ? a.X[r * N + f] : 0.f;
      }
    }
  };

  const bool key_sq = a.error_fn == 3;
  const bool tube = a.error_fn == 2 || a.error_fn == 3;
  const float thr = a.R;

  // XL: this wave's two buffers after the gene rows.
  const int XB = xl_buffer_bytes(N);
  unsigned char* xl_base = lds_raw + kCols * RS + wave * XB;
  auto xl_issue = [&](int tile) {
    const int64_t r = min((int64_t)tile * kTileRows + wq * 64 + lane, NP - 1);
    const float* src = a.X + r * N;
    unsigned char* dst = xl_base;
    for (int q = 0; q < N / 4; ++q)
      __builtin_amdgcn_global_load_lds((const void*)(src + 4 * q),
                                       (__attribute__((address_space(3))) void*)(dst + q * 1024),
                                       16, 0, 0);
    __builtin_amdgcn_global_load_lds((const void*)(a.t + r),
                                     (__attribute__((address_space(3))) void*)(dst + (N / 4) * 1024),
                                     4, 0, 0);
  };
  // Every group holds whole sub-features (no ragged last group): then the
  // features of group g sit at fixed offsets from one per-lane address.
  // Feature f of row r is at byte (f >> 2) * 1024 + r * 16 + (f & 3) * 4;
  // with G even, f = 2(gG + i) + h gives g * G * 512 + (i >> 1) * 1024 +
  // (i & 1) * 8 + h * 4 (trig, G a multiple of 4: f = gG + i gives
  // g * G * 256 + (i >> 2) * 1024 + (i & 3) * 4).
  constexpr bool kFixedOffsets = BASIS != 3 || G % 4 == 0;
  const bool whole_groups =
      kFixedOffsets && (BASIS == 3 ? G * a.Q == N : 2 * G * a.Q == a.U);
  const unsigned char* xl_lane = xl_base + m * 16 + (BASIS == 3 ? 0 : h * 4);
  // x of group g from this wave's XL buffer (rows rb*32 + m of the slice).
  auto xl_read = [&](int g, float (&xo)[2][G]) {
    if (whole_groups) {
      const unsigned char* src = xl_lane + g * (BASIS == 3 ? G * 256 : G * 512);
#pragma unroll
      for (int i = 0; i < G; ++i) {
        const int off = BASIS == 3 ? (i >> 2) * 1024 + (i & 3) * 4 : (i >> 1) * 1024 + (i & 1) * 8;
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
          xo[rb][i] = *reinterpret_cast<const float*>(src + off + rb * 512);
      }
      return;
    }
    const unsigned char* src = xl_base;
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const int qi = g * G + i;
      const int u = 2 * qi + h;
      const bool fvalid = BASIS == 3 ? (qi < N) : (u < a.U);
      const int f = fvalid ? (BASIS == 3 ? qi : u) : 0;
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        const float* p = reinterpret_cast<const float*>(src + (f >> 2) * 1024 + (rb * 32 + m) * 16) + (f & 3);
        const float v = *p;                  // f is clamped: always in the buffer
        xo[rb][i] = fvalid ? v : 0.f;
      }
    }
  };

  float xt[2][G];                          // next tile's first group (register path)
  if constexpr (XL) {
    if (tile_begin + wg < tile_end) xl_issue(tile_begin + wg);
  } else {
    if (tile_begin + wg < tile_end) load_x((int64_t)(tile_begin + wg) * kTileRows + wq * 64, 0, xt);
  }
  const int n_groups = a.Q;

  // B fragments of this lane for the four column blocks at a K-step's byte
  // offset within the chunk.
  const unsigned char* wrow = lds_raw + m * RS + h * 16;
  const int chunk_bytes = ks_chunk * 32;
  auto load_b = [&](int kbyte, bf16x8 (&bo)[4]) {
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
      bo[cb] = *reinterpret_cast<const bf16x8*>(wrow + cb * 32 * RS + kbyte);
  };
  // bq[k & 1]: B fragments of K-step k of the group; av[k & 1][rb]: A
  // fragments likewise (with an odd number of K-steps per group, the next
  // group's first fragments are moved to index 0 at the group's end).
  bf16x8 bq[2][4];
  if (a.n_chunks == 1) load_b(0, bq[0]);
  bf16x8 av[2][2];

  // Value p of a group (sub-feature p / D, degree p % D + 1) from features xs
  // and recurrence rs, into A buffer buf.
  auto gen = [&](auto pc, Recur<BASIS> (&rs)[2], const float (&xs)[2][G], bf16x8 (&dst)[2]) {
    constexpr int p = decltype(pc)::value;
    constexpr int i = p / D;
    constexpr int j = p % D;
    if constexpr (j == 0) {
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) rs[rb].seed(xs[rb][i], h);
    }
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) dst[rb][p & 7] = (__bf16)rs[rb].cur;
    if constexpr (j + 1 < D) {
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) rs[rb].template advance<j + 1>(xs[rb][i]);
    }
  };

  // Every wave runs the same number of iterations (the chunked path has
  // barriers inside); a wave without a tile of its own in the last round
  // recomputes the split's last tile and discards the result.
  for (int tp = tile_begin; tp < tile_end; tp += TS) {
    const bool active = tp + wg < tile_end;
    const int tile = active ? tp + wg : tile_end - 1;
    const int64_t row0 = (int64_t)tile * kTileRows + wq * 64;
    // Once the last features and the targets of this tile have been read
    // from the wave's buffer, the buffer takes the copy of the wave's next
    // tile (two groups and the epilogue ahead of its use for 4+ groups).
    auto xl_release = [&]() {
      __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0): the reads returned
      __asm__ __volatile__("" ::: "memory");
      if (tile + TS < tile_end) xl_issue(tile + TS);
    };
    // Features and recurrences of two consecutive groups: groups alternate
    // between the A and B sets, so nothing is copied from one group to the
    // next.
    float xA[2][G], xB[2][G];
    if constexpr (XL) {
      // This tile's copy (issued after the previous tile's last read) has
      // landed.
      __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
      __asm__ __volatile__("" ::: "memory");
      xl_read(0, xA);
      xl_read(n_groups > 1 ? 1 : 0, xB);
    } else {
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int i = 0; i < G; ++i) xA[rb][i] = xt[rb][i];
      load_x(row0, n_groups > 1 ? 1 : 0, xB);
    }
    // Bias K-step: accumulators start at a_0 - t_k, exactly.  The first
    // K-step's A values are generated meanwhile.
    Recur<BASIS> rcA[2], rcB[2];
    [&]<int... P>(std::integer_sequence<int, P...>) {
      (gen(std::integral_constant<int, P>{}, rcA, xA, av[0]), ...);
    }(std::make_integer_sequence<int, 8>{});
    f32x16 acc[2][4];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb) {
      bf16x8 abias = {};
      if (h == 0) {
        abias[0] = (__bf16)1.f;
        abias[1] = (__bf16)1.f;
        abias[2] = (__bf16)1.f;
      } else if constexpr (XL) {
        const float* tl = reinterpret_cast<const float*>(xl_base + (N / 4) * 1024);
        split3(-tl[rb * 32 + m], abias);
      } else {
        const int64_t r = row0 + rb * 32 + m;
        split3(-a.t[r < NP ? r : NP - 1], abias);
      }
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
        acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(abias, bbias[cb], f32x16{}, 0, 0, 0);
    }
    if constexpr (XL) {
      if (n_groups <= 2) xl_release();
    }

    for (int chunk = 0; chunk < a.n_chunks; ++chunk) {
      if (a.n_chunks > 1) {
        __syncthreads();
        stage(chunk);
        __syncthreads();
        load_b(0, bq[0]);
      }
      const int g_begin = chunk * gpc;
      const int g_end = min(g_begin + gpc, n_groups);
      // Group g with the current set (rc_c, x_c) and the next group's set
      // (rc_n, x_n); K-step k uses fragment buffer (k + PAR) & 1.
      auto group = [&](int g, auto par_c, Recur<BASIS> (&rc_c)[2], float (&x_c)[2][G],
                       Recur<BASIS> (&rc_n)[2], float (&x_n)[2][G]) {
        constexpr int PAR = decltype(par_c)::value;
        if constexpr (!XL) {
          // The next tile's first features, one group ahead of their use.
          if (g + 1 == n_groups && tile + TS < tile_end) load_x(row0 + TS * kTileRows, 0, xt);
        }
        const int kbase = (g - g_begin) * KS * 32;
        // K-step k: its eight MFMAs, each pair followed by the B fragment of
        // K-step k+1 for that column block and two of K-step k+1's A values
        // (for the last K-step: the next group's first K-step), so the vector
        // work issues while the matrix core runs.  The scheduling barriers
        // keep that order.
        auto kstep = [&](auto kc) {
          constexpr int k = decltype(kc)::value;
          constexpr int cur = (k + PAR) & 1, nxt = cur ^ 1;
          int nb = kbase + (k + 1) * 32;
          nb = nb == chunk_bytes ? 0 : nb;
          auto pair = [&](auto cc) {
            constexpr int cb = decltype(cc)::value;
            acc[0][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[cur][0], bq[cur][cb], acc[0][cb], 0, 0, 0);
            acc[1][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[cur][1], bq[cur][cb], acc[1][cb], 0, 0, 0);
            bq[nxt][cb] = *reinterpret_cast<const bf16x8*>(wrow + cb * 32 * RS + nb);
            if constexpr (k + 1 < KS) {
              gen(std::integral_constant<int, 8 * (k + 1) + 2 * cb>{}, rc_c, x_c, av[nxt]);
              gen(std::integral_constant<int, 8 * (k + 1) + 2 * cb + 1>{}, rc_c, x_c, av[nxt]);
            } else {
              gen(std::integral_constant<int, 2 * cb>{}, rc_n, x_n, av[nxt]);
              gen(std::integral_constant<int, 2 * cb + 1>{}, rc_n, x_n, av[nxt]);
            }
            __builtin_amdgcn_sched_barrier(0);
          };
          pair(std::integral_constant<int, 0>{});
          pair(std::integral_constant<int, 1>{});
          pair(std::integral_constant<int, 2>{});
          pair(std::integral_constant<int, 3>{});
        };
        [&]<int... Ks>(std::integer_sequence<int, Ks...>) {
          (kstep(std::integral_constant<int, Ks>{}), ...);
        }(std::make_integer_sequence<int, KS>{});
        // The current set is done: group g + 2's features go into it.
        if constexpr (XL) {
          if (g + 2 < n_groups) xl_read(g + 2, x_c);
          if (g + 3 == n_groups) xl_release();
        } else {
          load_x(row0, g + 2 < n_groups ? g + 2 : n_groups - 1, x_c);
        }
      };
      int g = g_begin;
      for (; g + 1 < g_end; g += 2) {
        group(g, std::integral_constant<int, 0>{}, rcA, xA, rcB, xB);
        group(g + 1, std::integral_constant<int, KS & 1>{}, rcB, xB, rcA, xA);
      }
      if (g < g_end) {
        // A last unpaired group: its successor's set (B) becomes A, group
        // g + 2's features (now in A) go to B, and fragments to parity 0.
        group(g, std::integral_constant<int, 0>{}, rcA, xA, rcB, xB);
        if constexpr (KS % 2 == 1) {
#pragma unroll
          for (int rb = 0; rb < 2; ++rb) av[0][rb] = av[1][rb];
#pragma unroll
          for (int cb = 0; cb < 4; ++cb) bq[0][cb] = bq[1][cb];
        }
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
          rcA[rb] = rcB[rb];
#pragma unroll
          for (int i = 0; i < G; ++i) {
            const float t2 = xA[rb][i];
            xA[rb][i] = xB[rb][i];
            xB[rb][i] = t2;
          }
        }
      }
    }

    // Epilogue: the accumulators hold Out - t.  MSE/RMSE sum the squares
    // (a NaN propagates); the convergence tube keeps a square when its key
    // exceeds R (|r| for TMSE, r^2 for the printed form of Eq. 10).  Rows
    // past the data count only in the ragged last tile.
    const bool full = row0 + 64 <= NP;
    float s[4] = {0.f, 0.f, 0.f, 0.f};
    if (!tube && full) {
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int i = 0; i < 16; ++i)
#pragma unroll
          for (int cb = 0; cb < 4; ++cb) s[cb] = fmaf(acc[rb][cb][i], acc[rb][cb][i], s[cb]);
    } else {
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int rl = rb * 32 + 8 * (i >> 2) + 4 * h + (i & 3);
          const bool ok = full || (row0 + rl < NP);
#pragma unroll
          for (int cb = 0; cb < 4; ++cb) {
            const float v = acc[rb][cb][i];
            const float e = v * v;
            const float key = key_sq ? e : fabsf(v);
            const float kept = tube ? (key > thr ? e : 0.f) : e;
            s[cb] += ok ? kept : 0.f;
          }
        }
      }
    }
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const float sc = active ? s[cb] : 0.f;
      const float t2 = sum[cb] + sc;
      comp[cb] += fabsf(sum[cb]) >= fabsf(sc) ? (sum[cb] - t2) + sc : (sc - t2) + sum[cb];
      sum[cb] = t2;
    }
  }

  double acc64[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    acc64[cb] = (double)sum[cb] + (double)comp[cb];
    acc64[cb] += __shfl_xor(acc64[cb], 32);
  }
  __syncthreads();
  double* red = reinterpret_cast<double*>(lds_raw);
  if (h == 0) {
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) red[wave * kCols + cb * 32 + m] = acc64[cb];
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

size_t fitness_bf16_lds_bytes(const FitArgs& a, int degree, bool xl) {
  const int G = group_size(degree);
  const int KS = G * degree / 8;
  const size_t w = (size_t)128 * bf16_row_bytes(a.pairs_per_chunk * KS) +
                   (xl ? (size_t)bf16_waves(degree) * xl_buffer_bytes(a.N) : 0);
  const size_t red = (size_t)bf16_waves(degree) * 128 * sizeof(double);
  return w > red ? w : red;
}

// The LDS copy path needs whole 16-byte feature quads per row, 16-byte
// aligned rows and room for the buffers next to the genes.
static bool use_xl(const FitArgs& a, int degree) {
  constexpr size_t kLdsPerCu = 160 * 1024;
  return a.N % 4 == 0 && ((uintptr_t)a.X & 15) == 0 && ((uintptr_t)a.t & 3) == 0 &&
         fitness_bf16_lds_bytes(a, degree, true) <= kLdsPerCu;
}

// Plan: Q = number of groups of 2G sub-features; pairs_per_chunk = groups
// staged in LDS at once: all of them when their BF16 genes fit a CU's LDS
// (staged once per workgroup; the feature copy buffers then come only if
// they fit beside them, see use_xl), otherwise 16 K-steps' worth per chunk,
// restaged for every pattern tile; 128-chromosome tiles.
void plan_fitness_bf16(FitArgs& a, int degree, int basis) {
  constexpr size_t kLdsPerCu = 160 * 1024;
  const int G = group_size(degree);
  const int KS = G * degree / 8;
  a.U = (basis == 3 ? 2 : 1) * a.N;
  a.Q = (a.U + 2 * G - 1) / (2 * G);
  int gpc = (size_t)128 * bf16_row_bytes(a.Q * KS) <= kLdsPerCu ? a.Q : 16 / KS;
  if (gpc < 1) gpc = 1;
  if (gpc > a.Q) gpc = a.Q;
  a.pairs_per_chunk = gpc;
  a.n_chunks = (a.Q + gpc - 1) / gpc;
  a.n_ctiles = (a.n_chrom + 127) / 128;
  a.tile_cols = 128;
  a.ld_partial = a.n_ctiles * 128;
  a.n_tiles = (int32_t)((a.NP + kTileRows - 1) / kTileRows);
  const int target = 512;
  int splits = (target + a.n_ctiles - 1) / a.n_ctiles;
  if (splits > max_splits(a.ld_partial)) splits = max_splits(a.ld_partial);
  if (splits > a.n_tiles) splits = a.n_tiles;
  if (splits < 1) splits = 1;
  a.tiles_per_split = (a.n_tiles + splits - 1) / splits;
  a.n_splits = (a.n_tiles + a.tiles_per_split - 1) / a.tiles_per_split;
  a.xcd_remap = ((a.n_ctiles * a.n_splits) % 8) == 0 ? 1 : 0;
}

template <int BASIS, int D, bool XL>
static hipError_t launch_variant(const FitArgs& a, hipStream_t s) {
  const size_t lds = fitness_bf16_lds_bytes(a, D, XL);
  const int grid = a.n_ctiles * a.n_splits;
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute((const void*)fitness_bf16_kernel<BASIS, D, XL>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((fitness_bf16_kernel<BASIS, D, XL>), dim3(grid), dim3(64 * bf16_waves(D)), lds, s,
                     a);
  return hipGetLastError();
}

template <int BASIS, int D>
static hipError_t launch_one(const FitArgs& a, hipStream_t s) {
  return use_xl(a, D) ? launch_variant<BASIS, D, true>(a, s) : launch_variant<BASIS, D, false>(a, s);
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

hipError_t launch_fitness_bf16(const FitArgs& a, int basis, int degree, hipStream_t s) {
  switch (basis) {
    case 0: return launch_basis<0>(a, degree, s);
    case 1: return launch_basis<1>(a, degree, s);
    case 2: return launch_basis<2>(a, degree, s);
    case 3: return launch_basis<3>(a, degree, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace game
