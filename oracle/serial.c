/* Plain serial float64 GAME fitness: test infrastructure, and the
 * single-thread CPU baseline of the benchmark (the counterpart of the
 * paper's serial version, Sec. 5).  One chromosome, one pattern, one term at
 * a time, straight from the definitions:
 *
 *   Out(pat_k) = a_0 + sum_i sum_b sum_j gene(i,b,j) phi_{b,j}(f_i)   (Eq. 2)
 *   E_k = (t_k - Out(pat_k))^2                                         (Eq. 3)
 *   MSE = sum_k E_k / NP (Eq. 4), RMSE its root (Eq. 5), TMSE keeps E_k
 *   only where |t_k - Out| > R (Eq. 10; error_fn 3: where E_k > R).
 *
 * phi_{0,j} is T_j (Chebyshev), P_j (Legendre) or x^j (power), each from
 * its textbook three-term recurrence (Eq. 1 leaves the function g free; the
 * paper gives no recurrence); for the trigonometric expansion (Eq. 8)
 * phi_{0,j} = cos(j x) and phi_{1,j} = sin(j x).  Gene layout: gene 0 is a_0,
 * gene 1 + i*B*d + b*d + (j-1) multiplies phi_{b,j} of feature i.
 * Built with -ffp-contract=off: every product and sum is rounded on its own.
 */
#include <math.h>
#include <stdint.h>

static double member(int basis, int j, double x) {
  if (basis == 2) { /* power */
    double v = 1.0;
    for (int q = 0; q < j; ++q) v = v * x;
    return v;
  }
  double prev = 1.0, cur = x; /* members 0 and 1 */
  for (int q = 1; q < j; ++q) {
    double nxt;
    if (basis == 0)
      nxt = 2.0 * x * cur - prev;
    else
      nxt = ((2.0 * q + 1.0) * x * cur - q * prev) / (q + 1.0);
    prev = cur;
    cur = nxt;
  }
  return cur;
}

/* fitness[p] for the n chromosomes genes[p * K ...]; returns 0, or -1 on a
 * bad argument.  X [NP x N] and t [NP] are float32, as the GPU path takes
 * them. */
int oracle_fitness_serial(const float* X, const float* t, int64_t NP, int N, const float* genes,
                          int n, int basis, int degree, int error_fn, double R, double* fitness) {
  if (!X || !t || !genes || !fitness || NP < 1 || N < 1 || n < 0 || degree < 1 ||
      basis < 0 || basis > 3)
    return -1;
  const int B = basis == 3 ? 2 : 1;
  const int64_t K = 1 + (int64_t)B * N * degree;
  for (int p = 0; p < n; ++p) {
    const float* g = genes + (int64_t)p * K;
    double sum = 0.0;
    for (int64_t k = 0; k < NP; ++k) {
      double out = g[0];
      for (int i = 0; i < N; ++i) {
        const double x = X[k * N + i];
        for (int b = 0; b < B; ++b)
          for (int j = 1; j <= degree; ++j) {
            double phi;
            if (basis == 3)
              phi = b == 0 ? cos(j * x) : sin(j * x);
            else
              phi = member(basis, j, x);
            out += (double)g[1 + (int64_t)i * B * degree + b * degree + (j - 1)] * phi;
          }
      }
      const double r = (double)t[k] - out;
      double e = r * r;
      if (error_fn == 2 && !(fabs(r) > R)) e = 0.0;
      if (error_fn == 3 && !(e > R)) e = 0.0;
      sum += e;
    }
    const double m = sum / (double)NP;
    fitness[p] = error_fn == 1 ? sqrt(m) : m;
  }
  return 0;
}
