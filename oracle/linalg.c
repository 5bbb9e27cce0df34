/* Dense Gaussian elimination with partial pivoting for the small systems the
 * oracle solves (n <= 8).  Test infrastructure only (see cgks_oracle.h). */
#include <math.h>
#include "oracle_internal.h"

/* Solve A x = b in place: A is n*n row-major (destroyed), b becomes x.
 * Returns 0, or -1 for a singular matrix. */
int orc_solve(int n, double *A, double *b) {
  for (int k = 0; k < n; ++k) {
    int piv = k;
    double best = fabs(A[k * n + k]);
    for (int r = k + 1; r < n; ++r) {
      double v = fabs(A[r * n + k]);
      if (v > best) { best = v; piv = r; }
    }
    if (best == 0.0) return -1;
    if (piv != k) {
      for (int c = 0; c < n; ++c) { double t = A[k * n + c]; A[k * n + c] = A[piv * n + c]; A[piv * n + c] = t; }
      double t = b[k]; b[k] = b[piv]; b[piv] = t;
    }
    for (int r = k + 1; r < n; ++r) {
      double f = A[r * n + k] / A[k * n + k];
      if (f == 0.0) continue;
      for (int c = k; c < n; ++c) A[r * n + c] -= f * A[k * n + c];
      b[r] -= f * b[k];
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    double s = b[k];
    for (int c = k + 1; c < n; ++c) s -= A[k * n + c] * b[c];
    b[k] = s / A[k * n + k];
  }
  return 0;
}

/* Inverse of an n*n matrix by solving against the unit vectors. */
int orc_invert(int n, const double *A, double *Ainv) {
  double work[64], col[8];
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i < n * n; ++i) work[i] = A[i];
    for (int i = 0; i < n; ++i) col[i] = (i == j) ? 1.0 : 0.0;
    if (orc_solve(n, work, col)) return -1;
    for (int i = 0; i < n; ++i) Ainv[i * n + j] = col[i];
  }
  return 0;
}
