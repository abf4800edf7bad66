// Three-term recurrences of the expansion families (Eq. 1 leaves g free;
// Eq. 8 is the trigonometric one).  A lane seeds the recurrence with its
// feature value and advances it one degree per K-step; `cur` holds phi_j.
// T is float for the MFMA paths and double for the float64 re-score.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

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

// Any family, chosen at run time (fam = 0..3 as above), with one
// branch-free step for every family: n = fma(A_J * xs, cur, -(B_J * prev)).
// Chebyshev and trig take A = B = 1 and xs = 2x (2 cos x), Legendre the
// coefficients above with xs = x, powers A = 1, B = 0 with xs = x.  Each
// family's step gives the bits of its fixed-family form: multiplying by 1 is
// exact, -(b * prev) equals (-b) * prev, and for powers fma(x, cur, -0)
// rounds x * cur once like the product itself (only the sign of an exact
// zero can differ, which no sum of squares can see).  Only the seed
// branches (uniformly, once per chain), and the (A_J, B_J) pair of a degree
// is one scalar load (recur_coef), so the degree loop carries no branch.
template <typename T>
struct Recur<-1, T> {
  T prev, cur, xs;
  __device__ void seed(int fam, T x, int half) {
    if (fam == 3) {
      T s, c;
      if constexpr (std::is_same_v<T, float>) sincosf(x, &s, &c);
      else sincos(x, &s, &c);
      prev = half ? T(0) : T(1);
      cur = half ? s : c;
      xs = T(2) * c;
    } else {
      prev = T(1);
      cur = x;
      xs = fam == 0 ? T(2) * x : x;
    }
  }
  // Degree J's step for the family `fam` given to seed (its coefficients
  // from recur_coef, defined below).
  template <int J>
  __device__ void advance_fam(int fam);
  __device__ void advance_ab(T A, T B) {
    const T n = fma(A * xs, cur, -(B * prev));
    prev = cur;
    cur = n;
  }
};

// (A_J, B_J) of the run-time step for family f at degree J (J = 1..16).
struct RecurCoef {
  float a, b;
};
constexpr RecurCoef recur_coef_of(int f, int J) {
  return f == 1 ? RecurCoef{legendre_a<float>(J), legendre_b<float>(J)}
                : RecurCoef{1.f, f == 2 ? 0.f : 1.f};
}
template <int... I>
constexpr auto recur_coef_table(std::integer_sequence<int, I...>) {
  struct Table {
    RecurCoef v[sizeof...(I)];
  };
  return Table{{recur_coef_of(I / 17, I % 17)...}};
}
static __constant__ const auto recur_coef = recur_coef_table(std::make_integer_sequence<int, 4 * 17>{});

template <typename T>
template <int J>
__device__ void Recur<-1, T>::advance_fam(int fam) {
  const RecurCoef ab = recur_coef.v[fam * 17 + J];
  advance_ab(T(ab.a), T(ab.b));
}

}  // namespace game
