// Per-pattern sums of the paper's own model (Eq. 9), in which every feature
// shares the genes a_j, b_j: Out = a_0 + sum_j a_j C_j + sum_j b_j S_j with
// C_j = sum_i cos(j f_i) and S_j = sum_i sin(j f_i).  The sums do not depend
// on the genes, so they are computed once per data set (the parallel version
// of Sec. 4.1 does the same) and the training loop then runs the degree-1
// power model over the 2d sums as features.
//
// One thread per pattern: cos/sin(j x) by the recurrence of Eq. 8 seeded
// with sincos(x), everything in float64, rounded to float32 once.  The
// per-degree sums live in registers (degree is a template argument).
//
// Also here: the per-feature trigonometric expansion's seeds (cos x, sin x of
// every pattern and feature), stored once per data set for the float32
// fitness kernel, which would otherwise evaluate them in every chromosome
// tile (Sec. 4.1: trigonometric terms computed once, not every iteration).
#include <hip/hip_runtime.h>

#include "common.h"

namespace game {

namespace {

template <int D>
__global__ __launch_bounds__(256) void trig_sums_kernel(const float* X, int64_t NP, int N,
                                                        float* Z) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= NP) return;
  double c[D], s[D];
#pragma unroll
  for (int j = 0; j < D; ++j) c[j] = s[j] = 0.0;
  const float* x = X + k * N;
  for (int i = 0; i < N; ++i) {
    double sn, cs;
    sincos((double)x[i], &sn, &cs);
    const double m2 = 2.0 * cs;
    double cp = 1.0, cc = cs, sp = 0.0, sc = sn;     // j-1 and j terms
#pragma unroll
    for (int j = 0; j < D; ++j) {
      c[j] += cc;
      s[j] += sc;
      const double cn = fma(m2, cc, -cp), sn2 = fma(m2, sc, -sp);
      cp = cc;
      cc = cn;
      sp = sc;
      sc = sn2;
    }
  }
  float* z = Z + k * (2 * D);
#pragma unroll
  for (int j = 0; j < D; ++j) {
    z[j] = (float)c[j];
    z[D + j] = (float)s[j];
  }
}

template <int D>
hipError_t launch_d(const float* X, int64_t NP, int N, float* Z, hipStream_t s) {
  hipLaunchKernelGGL(trig_sums_kernel<D>, dim3((unsigned)((NP + 255) / 256)), dim3(256), 0, s, X,
                     NP, N, Z);
  return hipGetLastError();
}

template <int... Ds>
hipError_t dispatch(int d, const float* X, int64_t NP, int N, float* Z, hipStream_t s,
                    std::integer_sequence<int, Ds...>) {
  hipError_t e = hipErrorInvalidValue;
  ((d == Ds + 1 ? (e = launch_d<Ds + 1>(X, NP, N, Z, s), 0) : 0), ...);
  return e;
}

__global__ __launch_bounds__(256) void trig_cs_kernel(const float* X, int64_t n, float* cs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float sn, c;
  sincosf(X[i], &sn, &c);
  cs[2 * i] = c;
  cs[2 * i + 1] = sn;
}

}  // namespace

hipError_t launch_trig_cs(const float* X, int64_t NP, int N, float* cs, hipStream_t s) {
  const int64_t n = NP * N;
  hipLaunchKernelGGL(trig_cs_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, X, n, cs);
  return hipGetLastError();
}

hipError_t launch_trig_sums(const float* X, int64_t NP, int N, int d, float* Z, hipStream_t s) {
  return dispatch(d, X, NP, N, Z, s, std::make_integer_sequence<int, kMaxDegree>{});
}

}  // namespace game
