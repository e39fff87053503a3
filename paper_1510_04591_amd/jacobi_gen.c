/* Jacobi matrix with a prescribed spectrum (test input generator).
 *
 * Given nodes lam[0..n) and a unit weight vector w, builds the symmetric
 * tridiagonal T = Q^T diag(lam) Q with Q e_1 = w, i.e. the matrix Lanczos on
 * diag(lam) produces from the start vector w, in O(n^2) operations and with
 * orthogonal transformations only (the reconstruction of Gragg and Harrod,
 * 1984).  The arrow matrix [[0, w^T], [w, diag(lam)]] is reduced to
 * tridiagonal form while its first row and column keep one coupling: nodes
 * are added one at a time; a Givens rotation folds the new node's weight
 * into the coupling of the anchor row, and the bulge this leaves in the new
 * row is chased down the diagonal until the new row couples only to the last
 * index.  Off-diagonals come out as absolute values.
 *
 * Holds none of the eigensolver's arithmetic; used to make matrices with a
 * known spectrum for tests and benchmarks. */
#include <math.h>
#include <stdlib.h>

int adc_gen_jacobi(int n, const double* lam, const double* w, double* diag, double* off) {
  if (n <= 0) return 0;
  /* d[0] is the anchor (0); d[1..n] the matrix; e[i] couples i and i+1 */
  double* d = (double*)calloc((size_t)n + 1, sizeof(double));
  double* e = (double*)calloc((size_t)n + 1, sizeof(double));
  if (!d || !e) {
    free(d);
    free(e);
    return -1;
  }
  d[1] = lam[0];
  e[0] = w[0];
  for (int k = 1; k < n; ++k) {
    const int p = k + 1; /* the new index */
    double dp = lam[k];
    double x = w[k]; /* entry (p, j-1), to be eliminated */
    double y = 0.0;  /* entry (p, j), the coupling with row j */
    for (int j = 1; j <= k; ++j) {
      const double a = e[j - 1]; /* entry (j, j-1) */
      const double r = sqrt(a * a + x * x); /* entries are bounded by the spectral radius */
      double c = 1.0, s = 0.0;
      if (r > 0.0) {
        c = a / r;
        s = x / r;
      }
      e[j - 1] = r;
      const double dj = d[j];
      const double cs = c * s;
      d[j] = c * c * dj + 2.0 * cs * y + s * s * dp;
      const double dpn = s * s * dj - 2.0 * cs * y + c * c * dp;
      const double yn = (c * c - s * s) * y + cs * (dp - dj);
      dp = dpn;
      if (j < k) {
        /* row j's coupling to j+1 mixes into row p: bulge at (p, j+1) */
        const double ej = e[j];
        e[j] = c * ej;
        x = yn;
        y = -s * ej;
      } else {
        e[k] = yn; /* row p now couples to k only */
      }
    }
    d[p] = dp;
  }
  for (int i = 0; i < n; ++i) diag[i] = d[i + 1];
  for (int i = 0; i + 1 < n; ++i) off[i] = fabs(e[i + 1]);
  free(d);
  free(e);
  return 0;
}
