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
constexpr int kGemmK = 32;
constexpr float kSqrtHalf = 0.70710678118654752440f;
constexpr float kInvSqrt2Pi = 0.39894228040143267794f;

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.f + erff(z * kSqrtHalf)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.f + erff(z * kSqrtHalf)) + z * kInvSqrt2Pi * expf(-0.5f * z * z);
}

// Stages a 64 x 32 slice X(r0 + r, k0 + c) into S[r][c]; rows >= R or
// k >= K read as zero.  Threads run along c when the k stride is 1, else
// along r.
__device__ __forceinline__ void stage_slice(float (*S)[kGemmK + 1], const float* X, int64_t ld_r,
                                            int64_t ld_k, int r0, int R, int k0, int K) {
  if (ld_k == 1) {
    for (int i = threadIdx.x; i < kGemmTile * kGemmK; i += 256) {
      const int r = i / kGemmK, c = i % kGemmK;
      const int gr = r0 + r, gk = k0 + c;
      S[r][c] = (gr < R && gk < K) ? X[(int64_t)gr * ld_r + gk] : 0.f;
    }
  } else {
    for (int i = threadIdx.x; i < kGemmTile * kGemmK; i += 256) {
      const int r = i % kGemmTile, c = i / kGemmTile;
      const int gr = r0 + r, gk = k0 + c;
      S[r][c] = (gr < R && gk < K) ? X[(int64_t)gr * ld_r + (int64_t)gk * ld_k] : 0.f;
    }
  }
}

template <bool BF16>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
  __shared__ float As[kGemmTile][kGemmK + 1];
  __shared__ float Bs[kGemmTile][kGemmK + 1];
  if (g.skip && *g.skip) return;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;       // 2 x 2 waves of 32 x 32
  const int m0 = blockIdx.y * kGemmTile, n0 = blockIdx.x * kGemmTile;
  const int l32 = lane & 31, h = lane >> 5;
  // K range of this split (whole slices; the last range may be short).
  const int kc = ((g.K + g.k_split - 1) / g.k_split + kGemmK - 1) / kGemmK * kGemmK;
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
      for (int c = 0; c < 8; ++c) rs += As[rs_r][rs_q * 8 + c];
    }
    const int am = wm * 32 + l32, bn = wn * 32 + l32;
    if constexpr (BF16) {
#pragma unroll
      for (int kk = 0; kk < kGemmK; kk += 16) {
        bf16x8 a, b;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          a[v] = (__bf16)As[am][kk + 8 * h + v];
          b[v] = (__bf16)Bs[bn][kk + 8 * h + v];
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < kGemmK; kk += 2)
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(As[am][kk + h], Bs[bn][kk + h], acc, 0, 0, 0);
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

// Split-K results: C[m][n] = sum over ranges in order; row sums likewise.
__global__ void gemm_reduce_kernel(GemmArgs g) {
  if (g.skip && *g.skip) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t MN = (int64_t)g.M * g.N;
  if (i < MN) {
    float s = 0.f;
    for (int z = 0; z < g.k_split; ++z) s += g.part[(int64_t)z * MN + i];
    const int m = (int)(i / g.N), n = (int)(i - (int64_t)m * g.N);
    g.C[(int64_t)m * g.ldc + n] = s;
  } else if (g.rowsum && i < MN + g.M) {
    const int m = (int)(i - MN);
    float s = 0.f;
    for (int z = 0; z < g.k_split; ++z) s += g.part_rs[(int64_t)z * g.M + m];
    g.rowsum[m] = s;
  }
}

hipError_t launch_gemm(const GemmArgs& g0, bool bf16, hipStream_t s) {
  GemmArgs g = g0;
  if (g.k_split < 1) g.k_split = 1;
  if (g.k_split > 1 && (g.bias || g.act || !g.part || (g.rowsum && !g.part_rs)))
    return hipErrorInvalidValue;   // split-K products carry no epilogue
  const dim3 grid((g.N + kGemmTile - 1) / kGemmTile, (g.M + kGemmTile - 1) / kGemmTile,
                  g.k_split);
  if (bf16) hipLaunchKernelGGL(gemm_kernel<true>, grid, dim3(256), 0, s, g);
  else hipLaunchKernelGGL(gemm_kernel<false>, grid, dim3(256), 0, s, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || g.k_split == 1) return e;
  const int64_t n = (int64_t)g.M * g.N + (g.rowsum ? g.M : 0);
  hipLaunchKernelGGL(gemm_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g);
  return hipGetLastError();
}

// Output layer backward for loss = mean((y - t)^2) over B rows:
// dy = 2 (y - t) / B; dZ2[b][j] = dy[b] w3[j] gelu'(Z2[b][j]).
__global__ void out_grad_kernel(const float* y, const float* t, int B, const float* w3,
                                const float* Z2, int H, float* dy, float* dZ2, const int32_t* skip) {
  if (skip && *skip) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * H) return;
  const int b = (int)(i / H), j = (int)(i - (int64_t)b * H);
  const float d = 2.f * (y[b] - t[b]) / (float)B;
  if (j == 0) dy[b] = d;
  dZ2[i] = d * w3[j] * gelu_grad_f(Z2[i]);
}

hipError_t launch_out_grad(const float* y, const float* t, int B, const float* w3, const float* Z2,
                           int H, float* dy, float* dZ2, const int32_t* skip, hipStream_t s) {
  const int64_t n = (int64_t)B * H;
  hipLaunchKernelGGL(out_grad_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, y, t,
                     B, w3, Z2, H, dy, dZ2, skip);
  return hipGetLastError();
}

// Adam (Kingma & Ba) with bias correction on float32 parameters.  The step
// counter lives on the device (so a captured graph advances it on every
// replay): adam_tick_kernel increments it and stores the two bias
// corrections, adam_kernel applies the update.
__global__ void adam_tick_kernel(SurrogateState* st, const int32_t* skip) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (skip && *skip) return;
  const int step = st->step + 1;
  st->step = step;
  st->c1 = 1.f - powf(0.9f, (float)step);
  st->c2 = 1.f - powf(0.999f, (float)step);
}

__global__ void adam_kernel(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                            const SurrogateState* st, const int32_t* skip) {
  if (skip && *skip) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
  const float gi = g[i];
  const float mi = beta1 * m[i] + (1.f - beta1) * gi;
  const float vi = beta2 * v[i] + (1.f - beta2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / st->c1) / (sqrtf(vi / st->c2) + eps);
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                       SurrogateState* st, const int32_t* skip, hipStream_t s) {
  hipLaunchKernelGGL(adam_tick_kernel, dim3(1), dim3(64), 0, s, st, skip);
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
