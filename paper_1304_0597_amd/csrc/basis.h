// Three-term recurrences of the expansion families (Eq. 1 leaves g free;
// Eq. 8 is the trigonometric one).  A lane seeds the recurrence with its
// feature value and advances it one degree per K-step; `cur` holds phi_j.
// T is float for the MFMA paths and double for the float64 re-score.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace game {

template <int BASIS, typename T = float>
struct Recur;

// Chebyshev: T_{j+1} = 2x T_j - T_{j-1}
template <typename T>
struct Recur<0, T> {
  T prev, cur, m2;
  __device__ void seed(T x, int) { prev = T(1); cur = x; m2 = T(2) * x; }
  template <int J>
  __device__ void advance(T) { T n = fma(m2, cur, -prev); prev = cur; cur = n; }
};
// Legendre: (j+1) P_{j+1} = (2j+1) x P_j - j P_{j-1}
template <typename T>
constexpr T legendre_a(int J) { return T(2 * J + 1) / T(J + 1); }
template <typename T>
constexpr T legendre_b(int J) { return T(J) / T(J + 1); }

template <typename T>
struct Recur<1, T> {
  T prev, cur;
  __device__ void seed(T x, int) { prev = T(1); cur = x; }
  template <int J>
  __device__ void advance(T x) {
    constexpr T a = legendre_a<T>(J);
    constexpr T b = legendre_b<T>(J);
    T n = fma(a * x, cur, -b * prev);
    prev = cur; cur = n;
  }
};
// Powers: x^{j+1} = x * x^j
template <typename T>
struct Recur<2, T> {
  T cur;
  __device__ void seed(T x, int) { cur = x; }
  template <int J>
  __device__ void advance(T x) { cur *= x; }
};
// Trigonometric (Eq. 8): cos/sin((j+1)x) = 2 cos x * cos/sin(jx) - cos/sin((j-1)x).
// Lane half 0 runs the cos chain, half 1 the sin chain of the same feature.
template <typename T>
struct Recur<3, T> {
  T prev, cur, m2;
  __device__ void seed(T x, int half) {
    T s, c;
    if constexpr (std::is_same_v<T, float>) sincosf(x, &s, &c);
    else sincos(x, &s, &c);
    prev = half ? T(0) : T(1);
    cur = half ? s : c;
    m2 = T(2) * c;
  }
  // The same seed from a stored (cos x, sin x) pair.
  __device__ void seed_cs(T c, T s, int half) {
    prev = half ? T(0) : T(1);
    cur = half ? s : c;
    m2 = T(2) * c;
  }
  template <int J>
  __device__ void advance(T) { T n = fma(m2, cur, -prev); prev = cur; cur = n; }
};

}  // namespace game
