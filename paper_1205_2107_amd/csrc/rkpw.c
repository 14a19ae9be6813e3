/*
 * Jacobi matrix with a prescribed spectrum (input generation only; none of the
 * eigensolver's arithmetic).
 *
 * Given nodes t[0..n-1] and a vector om[0..n-1], build the symmetric tridiagonal
 * T (diagonal d, off-diagonal e) that the Lanczos process produces from
 * diag(t) and the start vector om / ||om||: T = U^T diag(t) U with U orthogonal
 * and U^T om = ||om|| e_1.  When om is a uniformly random unit vector this has
 * the distribution of the Householder tridiagonal form of Q diag(t) Q^T with Q
 * Haar-distributed.
 *
 * Method (Rutishauser / Gragg-Harrod style, O(n^2), backward stable): keep the
 * bordered tridiagonal J = [[0, b0 e1^T], [b0 e1, T_k]] and add one node at a
 * time as a new last row/column coupled only to the border; a Givens rotation
 * in plane (1, q) removes that coupling and the bulge it creates is chased down
 * the band by rotations in planes (p, q), p = 2..k.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

int workload_rkpw(int64_t n, const double* t, const double* om, double* d, double* e) {
  if (n < 1) return 0;
  double* a = (double*)malloc((size_t)(n + 2) * sizeof(double));
  double* b = (double*)malloc((size_t)(n + 2) * sizeof(double));
  if (!a || !b) { free(a); free(b); return -1; }
  a[0] = 0.0;
  b[0] = om[0];
  a[1] = t[0];
  for (int64_t k = 1; k < n; k++) {
    /* J has indices 0..k; the new index q = k + 1 carries t[k] and couples to 0 */
    double x = om[k]; /* entry (p-1, q) to annihilate */
    double B = 0.0;   /* entry (p, q) */
    double C = t[k];  /* entry (q, q) */
    for (int64_t p = 1; p <= k; p++) {
      double y = b[p - 1];
      double r = sqrt(y * y + x * x);
      double c = 1.0, s = 0.0;
      if (r > 0.0) { c = y / r; s = x / r; }
      b[p - 1] = r;
      double A = a[p];
      a[p] = c * c * A + 2.0 * c * s * B + s * s * C;
      double Cn = s * s * A - 2.0 * c * s * B + c * c * C;
      double Bn = c * s * (C - A) + (c * c - s * s) * B;
      C = Cn;
      if (p < k) {
        x = Bn;
        B = -s * b[p];
        b[p] = c * b[p];
      } else {
        b[k] = Bn;
      }
    }
    a[k + 1] = C;
  }
  for (int64_t i = 0; i < n; i++) d[i] = a[i + 1];
  for (int64_t i = 0; i + 1 < n; i++) e[i] = b[i + 1];
  free(a);
  free(b);
  return 0;
}
