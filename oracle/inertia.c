/* Eigenvalue counts of the pencil (S, M) by Sylvester's law of inertia.
 * TEST INFRASTRUCTURE (part of the CPU oracle; never linked into the library).
 *
 * The pencil of Section 2 (eq. def:basisMatrixEVP) has S symmetric positive
 * semi-definite and M diagonal positive (Remark 2.1), so the number of
 * eigenvalues omega^2 < sigma equals the number of negative pivots of
 * A = S - sigma M = L D L^T (A congruent to D).  The factorisation here is
 * the plain one without pivoting on the lower band of A, of half-bandwidth
 * bw (every stored entry has |row - col| <= bw): O(n bw^2) work, n (bw + 1)
 * doubles of memory.
 *
 * band[j * (bw + 1) + t] holds A(j + t, j), t = 0..bw.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Returns the number of negative pivots, or -1 when an entry lies outside
 * the band, -2 when a pivot vanishes (|d| <= 1e-300: sigma is, to working
 * accuracy, an eigenvalue of a leading block; retry with a nearby sigma),
 * -3 when memory runs out. */
int64_t kf_oracle_inertia(int32_t n, const int32_t* rowptr, const int32_t* col, const double* val, const double* m,
                          double sigma, int32_t bw) {
  const int64_t w = (int64_t)bw + 1;
  double* band = (double*)calloc((size_t)n * (size_t)w, sizeof(double));
  if (!band) return -3;
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
      const int32_t c = col[q];
      if (c > i) continue; /* lower triangle only (S is symmetric) */
      if (i - c > bw) {
        free(band);
        return -1;
      }
      band[(int64_t)c * w + (i - c)] += val[q];
    }
    band[(int64_t)i * w] -= sigma * m[i];
  }
  int64_t neg = 0;
  for (int32_t j = 0; j < n; ++j) {
    double* cj = band + (int64_t)j * w;
    const double d = cj[0];
    if (!(fabs(d) > 1e-300)) {
      free(band);
      return -2;
    }
    if (d < 0.0) ++neg;
    const int32_t tmax = (n - 1 - j) < bw ? (n - 1 - j) : bw;
    /* trailing update: A(j+t, j+s) -= A(j+t, j) A(j+s, j) / d, s <= t */
    for (int32_t s = 1; s <= tmax; ++s) {
      const double ls = cj[s] / d;
      if (ls == 0.0) continue;
      double* cs = band + (int64_t)(j + s) * w;
      for (int32_t t = s; t <= tmax; ++t) cs[t - s] -= cj[t] * ls;
    }
  }
  free(band);
  return neg;
}
