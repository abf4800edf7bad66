// Fitness-surrogate network kernels: a multilayer perceptron with GELU
// hidden layers (genes -> standardised log error), trained on the GPU.
//
// gemm_kernel computes C[m][n] = sum_k A(m,k) B(n,k) with arbitrary element
// strides for A and B (so forward products, weight gradients dZ^T X and
// input gradients dZ W all use one kernel), on MFMA: BF16 operands with FP32
// accumulation (v_mfma_f32_32x32x16_bf16), or FP32 operands
// (v_mfma_f32_32x32x2_f32) for a full-precision mode.  Epilogues: + bias[n],
// then identity, GELU (optionally storing the pre-activation), or
// multiplication by GELU'(aux[m][n]) (the backward of a GELU layer).
// A workgroup of 4 waves computes a 64x64 tile of C from 64x32 slices of A
// and B staged in LDS; out-of-range rows, columns and k read as zero.  Each
// operand is staged with consecutive threads along its unit-stride index,
// so the global reads are coalesced whichever way the operand is laid out.
// Optionally the workgroups of the first column tile also sum the rows of
// A over k (the bias gradient of a layer comes with its weight gradient).
// Long-K products with a small M x N (weight gradients over a minibatch)
// split K over blockIdx.z; the ranges' partial results are added in a fixed
// order by gemm_reduce_kernel, so results do not depend on scheduling.
#include <math.h>

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
  // K range of this split (whole 32-value steps; the last range may be short).
  const int kc = ((g.K + g.k_split - 1) / g.k_split + 31) / 32 * 32;
  const int kb = blockIdx.z * kc, ke = min(g.K, kb + kc);
  const bool do_rs = g.rowsum && blockIdx.x == 0;
  const int rs_r = threadIdx.x >> 2, rs_q = threadIdx.x & 3;   // 4 threads per row
  float rs = 0.f;
  f32x16 acc = f32x16{};
  for (int k0 = kb; k0 < ke; k0 += kGemmK) {
    stage_slice(As, g.A, g.lda_m, g.lda_k, m0, g.M, k0, ke);
    stage_slice(Bs, g.B, g.ldb_n, g.ldb_k, n0, g.N, k0, ke);
    __syncthreads();
    if (do_rs) {
#pragma unroll
      for (int c = 0; c < kGemmK / 4; ++c) rs += As[rs_r * kGemmLd + rs_q * (kGemmK / 4) + c];
      static_assert(kGemmK == 128, "staging maps assume 128 K values per pass");
    }
    const int kn = min(kGemmK, ke - k0);           // MFMA steps past kn read zeros: skip them
    const float* ar = As + (wm * 32 + l32) * kGemmLd;
    const float* br = Bs + (wn * 32 + l32) * kGemmLd;
    if constexpr (BF16) {
      for (int kk = 0; kk < kn; kk += 16) {
        bf16x8 a, b;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          a[v] = (__bf16)ar[kk + 8 * h + v];
          b[v] = (__bf16)br[kk + 8 * h + v];
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
      }
    } else {
      for (int kk = 0; kk < kn; kk += 2)
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(ar[kk + h], br[kk + h], acc, 0, 0, 0);
    }
    __syncthreads();
  }
  if (do_rs) {
    // The row's 4 partial sums sit in 4 consecutive lanes: fixed-order pairs.
    rs += __shfl_xor(rs, 1);
    rs += __shfl_xor(rs, 2);
    const int m = m0 + rs_r;
    if (rs_q == 0 && m < g.M) {
      if (g.k_split > 1) g.part_rs[(int64_t)blockIdx.z * g.M + m] = rs;
      else g.rowsum[m] = rs;
    }
  }
  const int n = n0 + wn * 32 + l32;
  if (n >= g.N) return;
  if (g.k_split > 1) {
    float* P = g.part + (int64_t)blockIdx.z * g.M * g.N;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int m = m0 + wm * 32 + 8 * (i >> 2) + 4 * h + (i & 3);
      if (m < g.M) P[(int64_t)m * g.N + n] = acc[i];
    }
    return;
  }
  const float bias = g.bias ? g.bias[n] : 0.f;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int m = m0 + wm * 32 + 8 * (i >> 2) + 4 * h + (i & 3);
    if (m >= g.M) continue;
    float z = acc[i] + bias;
    const int64_t off = (int64_t)m * g.ldc + n;
    if (g.act == 1) {
      if (g.Z) g.Z[off] = z;
      z = gelu_f(z);
    } else if (g.act == 2) {
      z *= gelu_grad_f(g.aux[(int64_t)m * g.ld_aux + n]);
    }
    g.C[off] = z;
  }
}

// Split-K results: C[m][n] = epilogue(sum over ranges in order); row sums
// likewise (no epilogue).
__global__ void gemm_reduce_kernel(GemmArgs g) {
  if (g.skip && *g.skip) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t MN = (int64_t)g.M * g.N;
  if (i < MN) {
    float z = 0.f;
    for (int k = 0; k < g.k_split; ++k) z += g.part[(int64_t)k * MN + i];
    const int m = (int)(i / g.N), n = (int)(i - (int64_t)m * g.N);
    if (g.bias) z += g.bias[n];
    const int64_t off = (int64_t)m * g.ldc + n;
    if (g.act == 1) {
      if (g.Z) g.Z[off] = z;
      z = gelu_f(z);
    } else if (g.act == 2) {
      z *= gelu_grad_f(g.aux[(int64_t)m * g.ld_aux + n]);
    }
    g.C[off] = z;
  } else if (g.rowsum && i < MN + g.M) {
    const int m = (int)(i - MN);
    float s = 0.f;
    for (int k = 0; k < g.k_split; ++k) s += g.part_rs[(int64_t)k * g.M + m];
    g.rowsum[m] = s;
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

hipError_t launch_gemm(const GemmArgs& g0, bool bf16, hipStream_t s) {
  GemmArgs g = g0;
  if (g.k_split < 1) g.k_split = 1;
  if (g.k_split > 1 && (!g.part || (g.rowsum && !g.part_rs))) return hipErrorInvalidValue;
  const dim3 grid((g.N + kGemmTile - 1) / kGemmTile, (g.M + kGemmTile - 1) / kGemmTile,
                  g.k_split);
  hipError_t e = bf16 ? launch_gemm_t<true>(g, grid, s) : launch_gemm_t<false>(g, grid, s);
  if (e != hipSuccess || g.k_split == 1) return e;
  const int64_t n = (int64_t)g.M * g.N + (g.rowsum ? g.M : 0);
  hipLaunchKernelGGL(gemm_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g);
  return hipGetLastError();
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

// Adam (Kingma & Ba) with bias correction on float32 parameters.  The step
// counter lives on the device (so a captured graph advances it on every
// replay); the training step's output-layer launch has already advanced it.
__global__ void adam_kernel(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                            const SurrogateState* st, const int32_t* skip) {
  if (skip && *skip) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int step = st->step;
  const float c1 = 1.f - powf(0.9f, (float)step);
  const float c2 = 1.f - powf(0.999f, (float)step);
  const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
  const float gi = g[i];
  const float mi = beta1 * m[i] + (1.f - beta1) * gi;
  const float vi = beta2 * v[i] + (1.f - beta2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                       SurrogateState* st, const int32_t* skip, hipStream_t s) {
  hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m, v,
                     n, lr, (const SurrogateState*)st, skip);
  return hipGetLastError();
}

// Fills n floats with zero (used instead of a memset so the work can sit in
// a captured graph).
__global__ void fill_zero_kernel(float* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.f;
}

hipError_t launch_fill_zero(float* p, int64_t n, hipStream_t s) {
  int blocks = (int)((n + 255) / 256);
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(blocks), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace game
