// The "run" and classification use cases (Sec. 2 use cases; Sec. 5 figures
// of merit): the model output Out (Eq. 2) of given chromosomes on a set of
// patterns, stored, or turned into class decisions and counted.
//
// These are not on the training loop's hot path, so one thread computes one
// (pattern, chromosome) output on the vector ALUs in float32, in the
// canonical gene order (feature, block, degree) with fused multiply-adds;
// the chromosome's genes sit in LDS.  Prediction and classification share
// the same output routine, so a class decision equals the stored output
// compared with the threshold.
#include "basis.h"
#include "common.h"

namespace game {

namespace {

// Out for one pattern row x[0..N) of a chromosome w[0..K) (runtime degree).
template <int BASIS>
__device__ float model_output(const float* x, int N, int d, const float* w) {
  constexpr int B = BASIS == 3 ? 2 : 1;
  float out = w[0];
  for (int f = 0; f < N; ++f) {
    const float xv = x[f];
    for (int b = 0; b < B; ++b) {
      const float* wf = w + 1 + (f * B + b) * d;
      float prev, cur, m2 = 2.f * xv;
      if constexpr (BASIS == 3) {
        float s, c;
        sincosf(xv, &s, &c);
        prev = b ? 0.f : 1.f;
        cur = b ? s : c;
        m2 = 2.f * c;
      } else {
        prev = 1.f;
        cur = xv;
      }
      for (int j = 1; j <= d; ++j) {
        out = fmaf(wf[j - 1], cur, out);
        if (j == d) break;
        float nx;
        if constexpr (BASIS == 0 || BASIS == 3) {
          nx = fmaf(m2, cur, -prev);
        } else if constexpr (BASIS == 1) {
          // (j+1) P_{j+1} = (2j+1) x P_j - j P_{j-1}
          const float a = (float)(2 * j + 1) / (float)(j + 1), c = (float)j / (float)(j + 1);
          nx = fmaf(a * xv, cur, -c * prev);
        } else {
          nx = cur * xv;
        }
        prev = cur;
        cur = nx;
      }
    }
  }
  return out;
}

template <int BASIS, bool CLASSIFY>
__global__ __launch_bounds__(256) void predict_kernel(PredictArgs a) {
  extern __shared__ float w[];
  __shared__ unsigned long long tally[4];
  const int c = blockIdx.y;
  const float* g = a.genes + (int64_t)c * a.K;
  for (int i = threadIdx.x; i < a.K; i += blockDim.x) w[i] = g[i];
  if (CLASSIFY && threadIdx.x < 4) tally[threadIdx.x] = 0;
  __syncthreads();
  uint32_t tp = 0, fp = 0, tn = 0, fn = 0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < a.NP;
       k += (int64_t)gridDim.x * blockDim.x) {
    const float out = model_output<BASIS>(a.X + k * a.N, a.N, a.degree, w);
    if constexpr (CLASSIFY) {
      const bool pred = out >= a.threshold;
      const bool pos = a.t[k] > 0.5f;
      tp += pred && pos;
      fp += pred && !pos;
      tn += !pred && !pos;
      fn += !pred && pos;
    } else {
      a.out[(int64_t)c * a.NP + k] = out;
    }
  }
  if constexpr (CLASSIFY) {
    // Integer sums: exact in any order.
    for (int o = 32; o > 0; o >>= 1) {
      tp += __shfl_xor(tp, o);
      fp += __shfl_xor(fp, o);
      tn += __shfl_xor(tn, o);
      fn += __shfl_xor(fn, o);
    }
    if ((threadIdx.x & 63) == 0) {
      atomicAdd(&tally[0], (unsigned long long)tp);
      atomicAdd(&tally[1], (unsigned long long)fp);
      atomicAdd(&tally[2], (unsigned long long)tn);
      atomicAdd(&tally[3], (unsigned long long)fn);
    }
    __syncthreads();
    if (threadIdx.x < 4)
      atomicAdd((unsigned long long*)a.counts + (int64_t)c * 4 + threadIdx.x, tally[threadIdx.x]);
  }
}

__global__ void zero_counts_kernel(int64_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

template <bool CLASSIFY>
hipError_t launch_mode(const PredictArgs& a, int basis, hipStream_t s) {
  const int64_t want = (a.NP + 255) / 256;
  const dim3 grid((unsigned)(want < 1024 ? want : 1024), (unsigned)a.n);
  const size_t lds = (size_t)a.K * sizeof(float);
  switch (basis) {
    case 0: hipLaunchKernelGGL((predict_kernel<0, CLASSIFY>), grid, dim3(256), lds, s, a); break;
    case 1: hipLaunchKernelGGL((predict_kernel<1, CLASSIFY>), grid, dim3(256), lds, s, a); break;
    case 2: hipLaunchKernelGGL((predict_kernel<2, CLASSIFY>), grid, dim3(256), lds, s, a); break;
    case 3: hipLaunchKernelGGL((predict_kernel<3, CLASSIFY>), grid, dim3(256), lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_predict(const PredictArgs& a, int basis, hipStream_t s) {
  if (!a.counts) return launch_mode<false>(a, basis, s);
  const int64_t n = (int64_t)a.n * 4;
  hipLaunchKernelGGL(zero_counts_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     a.counts, n);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_mode<true>(a, basis, s);
}

}  // namespace game
