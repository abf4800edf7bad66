// Float64 re-score: the error of a few chromosomes (the elite at the end of
// a reduced-precision run, or an audit sample) computed in double precision
// on the vector ALUs, from the same X, t and genes (Eqs. 2-5, 10).
//
// Grid (blocks_per_chromosome, n): the chromosome's genes are widened to
// double in LDS; each thread accumulates the squared residuals of a strided
// set of patterns, the block reduces them in a fixed tree order, and a
// finish pass sums the blocks in order, so the result is deterministic.
#include <utility>

#include "basis.h"
#include "common.h"

namespace game {

constexpr int kRescoreThreads = 256;

template <int BASIS, int D>
__global__ __launch_bounds__(kRescoreThreads) void rescore64_kernel(Rescore64Args a) {
  extern __shared__ double genes_lds[];
  __shared__ double red[kRescoreThreads];
  const int c = blockIdx.y;
  const float* g = a.genes + (int64_t)c * a.K;
  for (int i = threadIdx.x; i < a.K; i += blockDim.x) genes_lds[i] = (double)g[i];
  __syncthreads();
  const int B = BASIS == 3 ? 2 : 1;
  double acc = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < a.NP;
       k += (int64_t)gridDim.x * blockDim.x) {
    double out = genes_lds[0];
    for (int f = 0; f < a.N; ++f) {
      const double x = (double)a.X[k * a.N + f];
      for (int bb = 0; bb < B; ++bb) {
        Recur<BASIS, double> rc;
        rc.seed(x, bb);
        const double* w = genes_lds + 1 + (f * B + bb) * D;
        auto term = [&](auto jc) {
          constexpr int j = decltype(jc)::value;
          out = fma(w[j], rc.cur, out);
          if constexpr (j + 1 < D) rc.template advance<j + 1>(x);
        };
        [&]<int... J>(std::integer_sequence<int, J...>) {
          (term(std::integral_constant<int, J>{}), ...);
        }(std::make_integer_sequence<int, D>{});
      }
    }
    const double r = (double)a.t[k] - out;
    double e = r * r;
    if (a.error_fn == 2) e = fabs(r) > a.R ? e : 0.0;
    else if (a.error_fn == 3) e = e > a.R ? e : 0.0;
    acc += e;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kRescoreThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.partial[(int64_t)blockIdx.x * a.n + c] = red[0];
}

__global__ void rescore64_finish(const double* partial, int32_t blocks, int32_t n, int64_t NP,
                                 int32_t error_fn, double* out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  double s = 0.0;
  for (int b = 0; b < blocks; ++b) s += partial[(int64_t)b * n + c];
  double v = s / (double)NP;
  if (error_fn == 1) v = sqrt(v);
  if (isnan(v)) v = INFINITY;
  out[c] = v;
}

template <int BASIS, int D>
static hipError_t launch_one(const Rescore64Args& a, hipStream_t s) {
  hipLaunchKernelGGL((rescore64_kernel<BASIS, D>), dim3(a.blocks, a.n), dim3(kRescoreThreads),
                     (size_t)a.K * sizeof(double), s, a);
  return hipGetLastError();
}

template <int BASIS>
static hipError_t launch_basis(const Rescore64Args& a, int degree, hipStream_t s) {
  switch (degree) {
#define GAME_CASE(D) case D: return launch_one<BASIS, D>(a, s);
    GAME_CASE(1) GAME_CASE(2) GAME_CASE(3) GAME_CASE(4) GAME_CASE(5) GAME_CASE(6)
    GAME_CASE(7) GAME_CASE(8) GAME_CASE(9) GAME_CASE(10) GAME_CASE(11) GAME_CASE(12)
    GAME_CASE(13) GAME_CASE(14) GAME_CASE(15) GAME_CASE(16)
#undef GAME_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_rescore64(const Rescore64Args& a, int basis, int degree, double* out,
                            hipStream_t s) {
  hipError_t e;
  switch (basis) {
    case 0: e = launch_basis<0>(a, degree, s); break;
    case 1: e = launch_basis<1>(a, degree, s); break;
    case 2: e = launch_basis<2>(a, degree, s); break;
    case 3: e = launch_basis<3>(a, degree, s); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(rescore64_finish, dim3((a.n + 255) / 256), dim3(256), 0, s, a.partial,
                     a.blocks, a.n, a.NP, a.error_fn, out);
  return hipGetLastError();
}

}  // namespace game
