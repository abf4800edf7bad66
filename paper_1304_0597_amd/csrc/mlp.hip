// Fitness-surrogate network kernels: a multilayer perceptron with GELU
// hidden layers (genes -> standardised log error), trained on the GPU.
//
// Products C[m][n] = sum_k A(m,k) B(n,k) with arbitrary element strides for
// A and B (so forward products, weight gradients dZ^T X and input gradients
// dZ W all use one argument block), on MFMA: BF16 operands with FP32
// accumulation (v_mfma_f32_32x32x16_bf16), or FP32 operands
// (v_mfma_f32_32x32x2_f32) for a full-precision mode.  Epilogues: + bias[n],
// then identity, GELU (optionally storing the pre-activation), or
// multiplication by GELU'(aux[m][n]) (the backward of a GELU layer).
//
// Two kernels serve them.  Minibatch-sized products (M <= 4096 rows, and
// every split product) are latency-bound: gemm_small_kernel gives each
// workgroup a 32x32 tile of C and cuts K across its 8 waves; each wave
// loads its operand values straight from global memory into registers (all
// loads of a round in flight at once), runs its MFMAs, and the 8 partial
// tiles are added in a fixed order through LDS.  Weight gradients (K = the
// minibatch) also split K over blockIdx.z into ranges whose raw sums the
// Adam launch adds in order, and the bias gradient (the row sum of the
// product's A operand) comes from the same registers.  Larger products (the
// forward pass over all oversampled candidates) use gemm_kernel: 64x64
// tiles from 64x128 slices of A and B staged in LDS.  Out-of-range rows,
// columns and k read as zero in both.  Results never depend on scheduling.
#include <math.h>

#include <algorithm>

#include "common.h"

namespace game {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kGemmTile = 64;
constexpr int kGemmK = 128;           // K values staged per pass (all loads in flight at once)
constexpr int kGemmLd = kGemmK + 1;   // LDS row stride in floats (odd: conflict-free columns)
constexpr size_t kGemmLds = 2 * kGemmTile * kGemmLd * sizeof(float);
constexpr float kSqrtHalf = 0.70710678118654752440f;
constexpr float kInvSqrt2Pi = 0.39894228040143267794f;

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.f + erff(z * kSqrtHalf)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.f + erff(z * kSqrtHalf)) + z * kInvSqrt2Pi * expf(-0.5f * z * z);
}

// Keeps x when ok, else +0 (a mask, not a select: a select of a loaded
// value may be turned into a branch around the load).
__device__ __forceinline__ float keep_if(float x, bool ok) {
  return __uint_as_float(__float_as_uint(x) & (ok ? 0xFFFFFFFFu : 0u));
}

// Stages a 64 x 128 slice X(r0 + r, k0 + c) into S[r * kGemmLd + c]; rows
// >= R or k >= K read as zero.  Threads run along c when the k stride is 1
// (thread t holds c = t % 128 of rows t / 128 + 2u), else along r (thread t
// holds r = t % 64 of columns t / 64 + 4u), so each load instruction of a
// workgroup reads consecutive addresses.  A slice inside the matrix loads
// with linear addresses; an edge slice clamps them into the matrix and masks
// the values, so in both cases all 32 loads of a thread issue back to back.
__device__ __forceinline__ void stage_slice(float* S, const float* X, int64_t ld_r, int64_t ld_k,
                                            int r0, int R, int k0, int K) {
  constexpr int kPer = kGemmTile * kGemmK / 256;
  float v[kPer];
  const int t = threadIdx.x;
  if (ld_k == 1) {
    const int c = t & (kGemmK - 1), gk = k0 + c;
    const int rt = t >> 7;
    const float* col = X + min(gk, K - 1);
    if (r0 + kGemmTile <= R) {
      const float* p = col + (int64_t)(r0 + rt) * ld_r;
#pragma unroll
      for (int u = 0; u < kPer; ++u) v[u] = keep_if(p[2 * u * ld_r], gk < K);
    } else {
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int gr = r0 + rt + 2 * u;
        v[u] = keep_if(col[(int64_t)min(gr, R - 1) * ld_r], gr < R && gk < K);
      }
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) S[(rt + 2 * u) * kGemmLd + c] = v[u];
  } else {
    const int r = t & (kGemmTile - 1), gr = r0 + r;
    const int ct = t >> 6;
    const float* row = X + (int64_t)min(gr, R - 1) * ld_r;
    if (k0 + kGemmK <= K) {
      const float* p = row + (int64_t)(k0 + ct) * ld_k;
#pragma unroll
      for (int u = 0; u < kPer; ++u) v[u] = keep_if(p[4 * u * ld_k], gr < R);
    } else {
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int gk = k0 + ct + 4 * u;
        v[u] = keep_if(row[(int64_t)min(gk, K - 1) * ld_k], gr < R && gk < K);
      }
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) S[r * kGemmLd + ct + 4 * u] = v[u];
  }
}

// The arithmetic of a product, whichever kernel runs it: K is cut into
// 16-value steps, the steps into kSmallWaves ranges of ceil(steps /
// kSmallWaves); each range is accumulated from zero by MFMAs in step order
// (a bf16 step is one 32x32x16 MFMA over k = 16 s + 8 h + v; an FP32 step is
// eight 32x32x2 MFMAs, MFMA v pairing k = 16 s + v and 16 s + 8 + v), and
// the range sums are added in range order.  So a row's output does not
// depend on how many rows the product has (the network's predictions for a
// chromosome are the same in any batch).
constexpr int kSmallWaves = 8;
constexpr int kSmallSteps = 4;
constexpr int kSmallMaxM = 4096;

// Epilogue of output (m, n) with the product value z.
__device__ __forceinline__ void gemm_store(const GemmArgs& g, int m, int n, float z) {
  if (g.bias) z += g.bias[n];
  const int64_t off = (int64_t)m * g.ldc + n;
  if (g.act == 1) {
    if (g.Z) g.Z[off] = z;
    z = gelu_f(z);
  } else if (g.act == 2) {
    z *= gelu_grad_f(g.aux[(int64_t)m * g.ld_aux + n]);
  }
  g.C[off] = z;
}

template <bool BF16>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
  extern __shared__ float gemm_lds[];
  float* As = gemm_lds;
  float* Bs = gemm_lds + kGemmTile * kGemmLd;
  if (g.skip && *g.skip) return;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;       // 2 x 2 waves of 32 x 32
  const int m0 = blockIdx.y * kGemmTile, n0 = blockIdx.x * kGemmTile;
  const int l32 = lane & 31, h = lane >> 5;
  // Range sums in range order (see the arithmetic of a product above).
  const int per_w = (((g.K + 15) >> 4) + kSmallWaves - 1) / kSmallWaves;
  f32x16 total = f32x16{}, acc = f32x16{};
  int w = 0, next = per_w;                        // acc holds range w; range w + 1 starts at next
  auto fold = [&]() {
    total = w == 0 ? acc : total + acc;
    acc = f32x16{};
    ++w;
    next += per_w;
  };
  for (int k0 = 0; k0 < g.K; k0 += kGemmK) {
    stage_slice(As, g.A, g.lda_m, g.lda_k, m0, g.M, k0, g.K);
    stage_slice(Bs, g.B, g.ldb_n, g.ldb_k, n0, g.N, k0, g.K);
    __syncthreads();
    const int kn = min(kGemmK, g.K - k0);          // steps past kn read zeros: skip them
    const float* ar = As + (wm * 32 + l32) * kGemmLd;
    const float* br = Bs + (wn * 32 + l32) * kGemmLd;
    for (int kk = 0; kk < kn; kk += 16) {
      while (((k0 + kk) >> 4) >= next) fold();
      if constexpr (BF16) {
        bf16x8 a, b;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          a[v] = (__bf16)ar[kk + 8 * h + v];
          b[v] = (__bf16)br[kk + 8 * h + v];
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
      } else {
#pragma unroll
        for (int v = 0; v < 8; ++v)
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[kk + 8 * h + v], br[kk + 8 * h + v], acc,
                                                     0, 0, 0);
      }
    }
    __syncthreads();
  }
  while (w < kSmallWaves) fold();
  const int n = n0 + wn * 32 + l32;
  if (n >= g.N) return;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int m = m0 + wm * 32 + 8 * (i >> 2) + 4 * h + (i & 3);
    if (m < g.M) gemm_store(g, m, n, total[i]);
  }
}

// Small products: a 32x32 tile of C per workgroup of kSmallWaves waves.
// The K range of the workgroup (all of K, or range blockIdx.z of a split
// product) is cut into 16-value steps, wave w taking range w of them.  In
// step s, lane (r, h) of a wave needs X(row0 + r, 16 s + 8 h + v), v = 0..7,
// of each operand X.  When the row index is the unit stride (or the operand
// has one row) each lane loads its own values: a load instruction reads
// consecutive addresses.  When k is the unit stride, the wave instead loads
// its 32 rows x 64 k block along k (one row per instruction), writes it to
// its own LDS area and reads its values back.  A wave loads up to
// kSmallSteps steps per round, every load of the round issued before the
// first wait.  The waves' partial tiles (and row sums) are added in wave
// order through LDS (over the staging areas, after a barrier).
constexpr int kStageLd = 68;                    // staged row: 64 k values + 4 (16-byte rows)
constexpr int kStageFloats = 32 * kStageLd;     // one operand of one wave

template <bool STAGED>
struct SmallOperand {
  const float* X;
  int64_t ld_r, ld_k;
  int row0, R;
  float* stage;                                 // this wave's LDS area (staged only)
};

__host__ __device__ inline bool small_staged(int64_t ld_r, int64_t ld_k, int R) {
  return ld_k == 1 && ld_r != 1 && R > 1;
}

// Issues the loads of a round (steps s0 ..) into raw[32], branch-free so
// that both operands' loads are in flight together: load j reads row
// row0 + j at k = 16 s0 + lane (staged), or row row0 + r at
// k = 16 (s0 + j / 8) + 8 h + j % 8 (direct); clamped into the operand.
// Offsets are 32-bit byte offsets from the operand's base (the launch
// checks that every operand spans less than 4 GiB), so each load needs one
// address register.
template <bool STAGED>
__device__ __forceinline__ void small_issue(const SmallOperand<STAGED>& o, int s0, int K, int lane,
                                            float (&raw)[32]) {
  const int r = lane & 31, h = lane >> 5;
  const uint32_t ldr = (uint32_t)o.ld_r * 4u, ldk = (uint32_t)o.ld_k * 4u;
  const char* base = reinterpret_cast<const char*>(o.X);
#pragma unroll
  for (int j = 0; j < 32; ++j) {
    const int row = o.row0 + (STAGED ? j : r);
    const int k = STAGED ? s0 * 16 + lane : (s0 + (j >> 3)) * 16 + 8 * h + (j & 7);
    const uint32_t off = (uint32_t)min(row, o.R - 1) * ldr + (uint32_t)min(k, K - 1) * ldk;
    raw[j] = *reinterpret_cast<const float*>(base + off);
  }
}

// The round's values of lane (r, h), zero outside rows < R, k < K and
// steps < se.
template <bool STAGED>
__device__ __forceinline__ void small_finish(const SmallOperand<STAGED>& o, int s0, int se, int K,
                                             int lane, const float (&raw)[32],
                                             float (&val)[kSmallSteps][8]) {
  const int r = lane & 31, h = lane >> 5;
  if constexpr (STAGED) {
    const int k = s0 * 16 + lane;
    const bool kok = k < K && (k >> 4) < se;
#pragma unroll
    for (int j = 0; j < 32; ++j) o.stage[j * kStageLd + lane] = keep_if(raw[j], kok && o.row0 + j < o.R);
#pragma unroll
    for (int i = 0; i < kSmallSteps; ++i)
#pragma unroll
      for (int v = 0; v < 8; ++v) val[i][v] = o.stage[r * kStageLd + i * 16 + 8 * h + v];
  } else {
    const bool rok = o.row0 + r < o.R;
#pragma unroll
    for (int i = 0; i < kSmallSteps; ++i)
#pragma unroll
      for (int v = 0; v < 8; ++v) {
        const int k = (s0 + i) * 16 + 8 * h + v;
        val[i][v] = keep_if(raw[i * 8 + v], rok && k < K && s0 + i < se);
      }
  }
}

size_t small_lds_bytes(const GemmArgs& g) {
  const int st = (small_staged(g.lda_m, g.lda_k, g.M) ? 1 : 0) +
                 (small_staged(g.ldb_n, g.ldb_k, g.N) ? 1 : 0);
  const size_t stage = (size_t)kSmallWaves * st * kStageFloats;
  const size_t red = (size_t)kSmallWaves * 32 * 32;
  return ((size_t)kSmallWaves * 64 + (stage > red ? stage : red)) * sizeof(float);
}

// One launch may carry up to kMaxProducts independent products (row tiles
// [ty_end[p-1], ty_end[p]) serve product p); each product's workgroups take
// the operand-layout variant of its own operands.
constexpr int kMaxProducts = 3;
struct GemmMulti {
  GemmArgs g[kMaxProducts];
  int32_t ty_end[kMaxProducts];
  int32_t n;
};

template <bool BF16, bool SA, bool SB>
__device__ __forceinline__ void small_body(const GemmArgs& g, int by, float* small_lds) {
  float* red_rs = small_lds;                            // [waves][64]
  float* red = small_lds + kSmallWaves * 64;            // [waves][32 * 32], over the staging areas
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int r = lane & 31, h = lane >> 5;
  const int m0 = by * 32, n0 = blockIdx.x * 32;
  const int steps = (g.K + 15) >> 4;
  const int per_z = (steps + g.k_split - 1) / g.k_split;
  const int zb = min(steps, (int)blockIdx.z * per_z), ze = min(steps, zb + per_z);
  const int per_w = (ze - zb + kSmallWaves - 1) / kSmallWaves;
  const int wb = min(ze, zb + wave * per_w), we = min(ze, wb + per_w);
  float* area = red + wave * ((SA ? 1 : 0) + (SB ? 1 : 0)) * kStageFloats;
  const SmallOperand<SA> oa{g.A, g.lda_m, g.lda_k, m0, g.M, area};
  const SmallOperand<SB> ob{g.B, g.ldb_n, g.ldb_k, n0, g.N, area + (SA ? kStageFloats : 0)};
  f32x16 acc = f32x16{};
  float rs = 0.f;
  for (int s0 = wb; s0 < we; s0 += kSmallSteps) {
    float ra[32], rb[32];
    small_issue(oa, s0, g.K, lane, ra);
    small_issue(ob, s0, g.K, lane, rb);
    __builtin_amdgcn_sched_barrier(0);   // keep every load ahead of the first use
    float av[kSmallSteps][8], bv[kSmallSteps][8];
    small_finish(oa, s0, we, g.K, lane, ra, av);
    small_finish(ob, s0, we, g.K, lane, rb, bv);
    // Steps past the wave's range hold zeros: running their MFMAs keeps the
    // code free of branches.
#pragma unroll
    for (int i = 0; i < kSmallSteps; ++i) {
#pragma unroll
      for (int v = 0; v < 8; ++v) rs += av[i][v];
      if constexpr (BF16) {
        bf16x8 a, b;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          a[v] = (__bf16)av[i][v];
          b[v] = (__bf16)bv[i][v];
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
      } else {
#pragma unroll
        for (int v = 0; v < 8; ++v)
          acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i][v], bv[i][v], acc, 0, 0, 0);
      }
    }
  }
  __syncthreads();   // every wave is done with its staging area
  // Accumulator register i of lane (r, h) is C row 8 (i / 4) + 4 h + i % 4,
  // column r.
  float* rw = red + wave * 32 * 32;
#pragma unroll
  for (int i = 0; i < 16; ++i) rw[(8 * (i >> 2) + 4 * h + (i & 3)) * 32 + r] = acc[i];
  red_rs[wave * 64 + lane] = rs;
  __syncthreads();
  const bool split = g.part != nullptr;
  for (int o = threadIdx.x; o < 32 * 32; o += 64 * kSmallWaves) {
    const int mm = m0 + (o >> 5), nn = n0 + (o & 31);
    if (mm >= g.M || nn >= g.N) continue;
    float z = red[o];
#pragma unroll
    for (int w = 1; w < kSmallWaves; ++w) z += red[w * 32 * 32 + o];
    if (split) g.part[(int64_t)blockIdx.z * g.part_ld + (int64_t)mm * g.ldc + nn] = z;
    else gemm_store(g, mm, nn, z);
  }
  // Row sums of A over the range (the first column tile computes them):
  // the two lane halves of each wave, waves in order.
  if (g.rowsum_part && blockIdx.x == 0 && threadIdx.x < 32 && m0 + (int)threadIdx.x < g.M) {
    const int t = threadIdx.x;
    float v = 0.f;
#pragma unroll
    for (int w = 0; w < kSmallWaves; ++w) v += red_rs[w * 64 + t] + red_rs[w * 64 + t + 32];
    g.rowsum_part[(int64_t)blockIdx.z * g.part_ld + m0 + t] = v;
  }
}

template <bool BF16>
__global__ __launch_bounds__(64 * kSmallWaves) __attribute__((amdgpu_waves_per_eu(1, 2)))
void gemm_small_kernel(GemmMulti gm) {
  extern __shared__ float small_lds[];
  int pi = 0;
  while (pi + 1 < gm.n && (int)blockIdx.y >= gm.ty_end[pi]) ++pi;
  const GemmArgs& g = gm.g[pi];
  const int by = (int)blockIdx.y - (pi ? gm.ty_end[pi - 1] : 0);
  if (g.skip && *g.skip) return;
  if ((int)blockIdx.x * 32 >= g.N || by * 32 >= g.M || (int)blockIdx.z >= g.k_split) return;
  const bool sa = small_staged(g.lda_m, g.lda_k, g.M), sb = small_staged(g.ldb_n, g.ldb_k, g.N);
  if (sa) {
    if (sb) small_body<BF16, true, true>(g, by, small_lds);
    else small_body<BF16, true, false>(g, by, small_lds);
  } else {
    if (sb) small_body<BF16, false, true>(g, by, small_lds);
    else small_body<BF16, false, false>(g, by, small_lds);
  }
}

template <bool BF16>
static hipError_t launch_gemm_t(const GemmArgs& g, const dim3& grid, hipStream_t s) {
  static bool lds_set = false;   // one attribute call per instantiation
  if (!lds_set) {
    const hipError_t e = hipFuncSetAttribute((const void*)gemm_kernel<BF16>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)kGemmLds);
    if (e != hipSuccess) return e;
    lds_set = true;
  }
  hipLaunchKernelGGL(gemm_kernel<BF16>, grid, dim3(256), kGemmLds, s, g);
  return hipGetLastError();
}

template <bool BF16>
static hipError_t launch_small_t(const GemmMulti& gm, const dim3& grid, size_t lds, hipStream_t s) {
  static bool lds_set = false;   // one attribute call per instantiation
  if (!lds_set) {
    const int most = (int)((kSmallWaves * 64 + kSmallWaves * 2 * kStageFloats) * sizeof(float));
    const hipError_t e = hipFuncSetAttribute((const void*)gemm_small_kernel<BF16>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, most);
    if (e != hipSuccess) return e;
    lds_set = true;
  }
  hipLaunchKernelGGL(gemm_small_kernel<BF16>, grid, dim3(64 * kSmallWaves), lds, s, gm);
  return hipGetLastError();
}

// Checks a product's arguments; small: it runs on gemm_small_kernel.
static hipError_t check_gemm(GemmArgs& g, bool* small) {
  if (g.k_split < 1) g.k_split = 1;
  if (g.k_split > 1 && !g.part) return hipErrorInvalidValue;
  if (g.rowsum_part && !g.part) return hipErrorInvalidValue;
  // Operand spans in bytes (the small-product kernel uses 32-bit offsets).
  const auto span = [](int64_t rows, int64_t ld_r, int64_t K, int64_t ld_k) {
    return ((rows - 1) * ld_r + (K - 1) * ld_k + 1) * (int64_t)sizeof(float);
  };
  const bool fits = g.lda_m >= 0 && g.lda_k >= 0 && g.ldb_n >= 0 && g.ldb_k >= 0 &&
                    span(g.M, g.lda_m, g.K, g.lda_k) < (int64_t)UINT32_MAX &&
                    span(g.N, g.ldb_n, g.K, g.ldb_k) < (int64_t)UINT32_MAX;
  if (g.part && !fits) return hipErrorInvalidValue;
  *small = g.part || (g.M <= kSmallMaxM && fits);
  return hipSuccess;
}

hipError_t launch_gemm_multi(const GemmArgs* gs, int n, bool bf16, hipStream_t s) {
  if (n < 1 || n > kMaxProducts) return hipErrorInvalidValue;
  GemmMulti gm{};
  gm.n = n;
  int tx = 0, ty = 0, tz = 1;
  size_t lds = 0;
  for (int p = 0; p < n; ++p) {
    GemmArgs g = gs[p];
    bool small = false;
    const hipError_t e = check_gemm(g, &small);
    if (e != hipSuccess) return e;
    if (!small) return hipErrorInvalidValue;
    gm.g[p] = g;
    tx = std::max(tx, (g.N + 31) / 32);
    ty += (g.M + 31) / 32;
    gm.ty_end[p] = ty;
    tz = std::max(tz, g.k_split);
    lds = std::max(lds, small_lds_bytes(g));
  }
  const dim3 grid(tx, ty, tz);
  return bf16 ? launch_small_t<true>(gm, grid, lds, s) : launch_small_t<false>(gm, grid, lds, s);
}

hipError_t launch_gemm(const GemmArgs& g0, bool bf16, hipStream_t s) {
  GemmArgs g = g0;
  bool small = false;
  const hipError_t e = check_gemm(g, &small);
  if (e != hipSuccess) return e;
  if (small) return launch_gemm_multi(&g, 1, bf16, s);
  const dim3 grid((g.N + kGemmTile - 1) / kGemmTile, (g.M + kGemmTile - 1) / kGemmTile, 1);
  return bf16 ? launch_gemm_t<true>(g, grid, s) : launch_gemm_t<false>(g, grid, s);
}

// Output layer, one wave per row b: y_b = b3 + sum_j H2[b][j] w3[j] in
// float32 (lane l adds j = l, l+64, ... in order, then a butterfly), and,
// when t is set, the backward of loss = mean((y - t)^2) over the B rows:
// dy_b = 2 (y_b - t_b) / B, dZ2[b][j] = dy_b w3[j] gelu'(Z2[b][j]).  A
// training step also advances the Adam step counter here (step, when set),
// so the Adam launch that follows reads the new count.
__global__ __launch_bounds__(256) void out_layer_kernel(const float* H2, const float* w3,
                                                        const float* b3, int B, int H, float* y,
                                                        const float* t, const float* Z2, float* dy,
                                                        float* dZ2, int32_t* step,
                                                        const int32_t* skip) {
  if (skip && *skip) return;
  if (step && blockIdx.x == 0 && threadIdx.x == 0) *step += 1;
  const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (b >= B) return;
  const float* h = H2 + (int64_t)b * H;
  constexpr int kRow = 8;   // up to 512 units: the row's values stay in registers
  if (H <= 64 * kRow) {
    // Every load (H2, w3, Z2, t) issued before the first use: one memory
    // round trip; the sums keep the order of the general path below.
    float hv[kRow], wv[kRow], zv[kRow];
#pragma unroll
    for (int u = 0; u < kRow; ++u) {
      const int j = min(lane + 64 * u, H - 1);
      hv[u] = h[j];
      wv[u] = w3[j];
      zv[u] = t ? Z2[(int64_t)b * H + j] : 0.f;
    }
    const float tb = t ? t[b] : 0.f;
    float acc = 0.f;
#pragma unroll
    for (int u = 0; u < kRow; ++u)
      if (lane + 64 * u < H) acc = fmaf(hv[u], wv[u], acc);
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    const float yb = acc + b3[0];
    if (lane == 0) y[b] = yb;
    if (!t) return;
    const float d = 2.f * (yb - tb) / (float)B;
    if (lane == 0) dy[b] = d;
#pragma unroll
    for (int u = 0; u < kRow; ++u)
      if (lane + 64 * u < H) dZ2[(int64_t)b * H + lane + 64 * u] = d * wv[u] * gelu_grad_f(zv[u]);
    return;
  }
  float acc = 0.f;
  for (int j = lane; j < H; j += 64) acc = fmaf(h[j], w3[j], acc);
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  const float yb = acc + b3[0];
  if (lane == 0) y[b] = yb;
  if (!t) return;
  const float d = 2.f * (yb - t[b]) / (float)B;
  if (lane == 0) dy[b] = d;
  for (int j = lane; j < H; j += 64)
    dZ2[(int64_t)b * H + j] = d * w3[j] * gelu_grad_f(Z2[(int64_t)b * H + j]);
}

hipError_t launch_out_layer(const float* H2, const float* w3, const float* b3, int B, int H,
                            float* y, const float* t, const float* Z2, float* dy, float* dZ2,
                            int32_t* step, const int32_t* skip, hipStream_t s) {
  hipLaunchKernelGGL(out_layer_kernel, dim3((unsigned)((B + 3) / 4)), dim3(256), 0, s, H2, w3, b3,
                     B, H, y, t, Z2, dy, dZ2, step, skip);
  return hipGetLastError();
}

// Adam (Kingma & Ba) with bias correction on float32 parameters.  The
// gradient of parameter i is the sum of the ks split ranges part[z * n + i]
// in order z = 0, 1, ... (the weight-gradient products write them).  The
// step counter lives on the device (so a captured graph advances it on
// every replay); the training step's output-layer launch has already
// advanced it.
__global__ void adam_kernel(float* p, const float* part, int ks, float* m, float* v, int64_t n,
                            float lr, const SurrogateState* st, const int32_t* skip) {
  if (skip && *skip) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) adam_update(p, part, ks, m, v, n, lr, st->step, i);
}

hipError_t launch_adam(float* p, const float* part, int ks, float* m, float* v, int64_t n,
                       float lr, SurrogateState* st, const int32_t* skip, hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, part, ks,
                     m, v, n, lr, (const SurrogateState*)st, skip);
  return hipGetLastError();
}

__global__ void sum_ranges_kernel(float* g, const float* part, int ks, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) g[i] = sum_ranges(part, ks, n, i);
}

hipError_t launch_sum_ranges(float* g, const float* part, int ks, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(sum_ranges_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g,
                     part, ks, n);
  return hipGetLastError();
}

// Fills n floats with zero (used instead of a memset so the work can sit in
// a captured graph).
__global__ void fill_kernel(float* p, int64_t n, float value) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

hipError_t launch_fill(float* p, int64_t n, float value, hipStream_t s) {
  int blocks = (int)((n + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(fill_kernel, dim3(blocks), dim3(256), 0, s, p, n, value);
  return hipGetLastError();
}

hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s) { return launch_fill(p, n, 0.f, s); }

}  // namespace game
