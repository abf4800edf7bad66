// Fitness-surrogate network kernels: a multilayer perceptron with GELU
// hidden layers (genes -> standardised log error), trained on the GPU.
//
// gemm_kernel computes C[m][n] = sum_k A(m,k) B(n,k) with arbitrary element
// strides for A and B (so forward products, weight gradients X^T dZ and
// input gradients dZ W all use one kernel), on MFMA: BF16 operands with FP32
// accumulation (v_mfma_f32_32x32x16_bf16), or FP32 operands
// (v_mfma_f32_32x32x2_f32) for a full-precision mode.  Epilogues: + bias[n],
// then identity, GELU (optionally storing the pre-activation), or
// multiplication by GELU'(aux[m][n]) (the backward of a GELU layer).
// A workgroup of 4 waves computes a 64x64 tile of C from 64x32 slices of A
// and B staged in LDS; out-of-range rows, columns and k read as zero.
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
  f32x16 acc = f32x16{};
  for (int k0 = 0; k0 < g.K; k0 += kGemmK) {
    for (int i = threadIdx.x; i < kGemmTile * kGemmK; i += 256) {
      const int r = i / kGemmK, c = i % kGemmK;
      const int m = m0 + r, n = n0 + r, k = k0 + c;
      As[r][c] = (m < g.M && k < g.K) ? g.A[(int64_t)m * g.lda_m + (int64_t)k * g.lda_k] : 0.f;
      Bs[r][c] = (n < g.N && k < g.K) ? g.B[(int64_t)n * g.ldb_n + (int64_t)k * g.ldb_k] : 0.f;
    }
    __syncthreads();
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
  const int n = n0 + wn * 32 + l32;
  if (n >= g.N) return;
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

hipError_t launch_gemm(const GemmArgs& g, bool bf16, hipStream_t s) {
  const dim3 grid((g.N + kGemmTile - 1) / kGemmTile, (g.M + kGemmTile - 1) / kGemmTile);
  if (bf16) hipLaunchKernelGGL(gemm_kernel<true>, grid, dim3(256), 0, s, g);
  else hipLaunchKernelGGL(gemm_kernel<false>, grid, dim3(256), 0, s, g);
  return hipGetLastError();
}

// out[n] = sum_m A[m * ld + n] in a fixed order (column sums: bias gradients).
__global__ void colsum_kernel(const float* A, int M, int N, int ld, float* out,
                              const int32_t* skip) {
  if (skip && *skip) return;
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float s = 0.f;
  for (int m = 0; m < M; ++m) s += A[(int64_t)m * ld + n];
  out[n] = s;
}

hipError_t launch_colsum(const float* A, int M, int N, int ld, float* out, const int32_t* skip,
                         hipStream_t s) {
  hipLaunchKernelGGL(colsum_kernel, dim3((N + 255) / 256), dim3(256), 0, s, A, M, N, ld, out, skip);
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
