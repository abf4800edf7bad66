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
  __device__ void advance_rt(int, T) { T n = fma(m2, cur, -prev); prev = cur; cur = n; }
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
  // The same step at a run-time J (1..16): the coefficients come from a
  // table of the same compile-time values, so both forms give the same bits.
  __device__ void advance_rt(int J, T x) {
    constexpr T ta[17] = {T(0), legendre_a<T>(1), legendre_a<T>(2), legendre_a<T>(3),
                          legendre_a<T>(4), legendre_a<T>(5), legendre_a<T>(6),
                          legendre_a<T>(7), legendre_a<T>(8), legendre_a<T>(9),
                          legendre_a<T>(10), legendre_a<T>(11), legendre_a<T>(12),
                          legendre_a<T>(13), legendre_a<T>(14), legendre_a<T>(15),
                          legendre_a<T>(16)};
    constexpr T tb[17] = {T(0), legendre_b<T>(1), legendre_b<T>(2), legendre_b<T>(3),
                          legendre_b<T>(4), legendre_b<T>(5), legendre_b<T>(6),
                          legendre_b<T>(7), legendre_b<T>(8), legendre_b<T>(9),
                          legendre_b<T>(10), legendre_b<T>(11), legendre_b<T>(12),
                          legendre_b<T>(13), legendre_b<T>(14), legendre_b<T>(15),
                          legendre_b<T>(16)};
    T n = fma(ta[J] * x, cur, -tb[J] * prev);
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
  __device__ void advance_rt(int, T x) { cur *= x; }
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
  template <int J>
  __device__ void advance(T) { T n = fma(m2, cur, -prev); prev = cur; cur = n; }
  __device__ void advance_rt(int, T) { T n = fma(m2, cur, -prev); prev = cur; cur = n; }
};

// Any family, chosen at run time (fam = 0..3 as above): the same seeds and
// the same arithmetic per step as the fixed-family recurrences, so it gives
// the same bits; the choice is a uniform branch.  One body then serves every
// family (the batched kernel), with the register allocation of one.
template <typename T>
struct Recur<-1, T> {
  T prev, cur, m2;
  int fam;
  __device__ void seed(T x, int half) {
    if (fam == 3) {
      T s, c;
      if constexpr (std::is_same_v<T, float>) sincosf(x, &s, &c);
      else sincos(x, &s, &c);
      prev = half ? T(0) : T(1);
      cur = half ? s : c;
      m2 = T(2) * c;
    } else {
      prev = T(1);
      cur = x;
      m2 = T(2) * x;
    }
  }
  __device__ void advance_rt(int J, T x) {
    T n;
    if (fam == 1) {
      Recur<1, T> l;
      l.prev = prev;
      l.cur = cur;
      l.advance_rt(J, x);
      n = l.cur;
    } else if (fam == 2) {
      n = cur * x;
    } else {
      n = fma(m2, cur, -prev);
    }
    prev = cur;
    cur = n;
  }
};

}  // namespace game
