/* One-sided (Hestenes) Jacobi SVD in float64, for the oracle's singular value
 * soft-threshold (eq:svt).  TEST INFRASTRUCTURE ONLY: loaded by oracle/msld_oracle.py,
 * never by the product library, with which it shares no code.
 *
 * For a block B (m x n) the columns are rotated pairwise until every pair is
 * orthogonal to working precision: with alpha = ||b_p||^2, beta = ||b_q||^2 and
 * gamma = b_p . b_q, the plane rotation
 *     zeta = (beta - alpha) / (2 gamma),  t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),
 *     c = 1 / sqrt(1 + t^2),  s = c t,
 *     b_p <- c b_p - s b_q,  b_q <- s b_p + c b_q
 * zeroes gamma (the textbook Jacobi rotation; Golub & Van Loan, Matrix Computations,
 * Sec. 8.6; Demmel & Veselic 1992).  The same rotations applied to the identity give
 * V, so that B V has orthogonal columns a_j = sigma_j u_j: sigma_j = ||a_j||,
 * u_j = a_j / sigma_j, and B = U diag(sigma) V^T.  A pair is rotated while
 * |gamma| > tol sqrt(alpha beta) with tol = max(m, 32) 2^-52: a dot product of
 * length m carries a relative error up to about m 2^-53 and the rotation a few units
 * more, so a tighter test could keep rotating rounding noise.  A column whose norm is
 * at most delta = 2^-52 ||B||_F is numerically zero (a pair of parallel columns
 * rotates one of them down to such rounding noise, which stays parallel to the
 * other): it is not rotated, and at the end it gives sigma = 0 with a zero left
 * vector, an error of at most delta per column.  Sweeps run until one rotates
 * nothing, at most max_sweeps.
 *
 * Pair order: the round-robin (tournament) ordering, n - 1 rounds of n / 2 disjoint
 * pairs per sweep (one column idles per round when n is odd), a cyclic ordering for
 * which one-sided Jacobi converges (Brent & Luk 1985).  Each block is decomposed by one
 * thread; a batch of blocks is spread over OpenMP threads (the result does not depend
 * on the thread count).  Blocks with m < n are handled by the caller through B^T.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Pair k of round r for an even column count n2 (n2 - 1 rounds): column 0 stays put,
 * the other n2 - 1 columns rotate around it. */
static void rr_pair(int r, int k, int n2, int *a, int *b) {
  const int n1 = n2 - 1;
  *a = (k == 0) ? 0 : 1 + (k - 1 + r) % n1;
  *b = 1 + (n2 - 2 - k + r) % n1;
}

/* One pair: returns 1 if it rotated. A and V are column-major (A: n columns of length
 * m, V: n columns of length n). Columns >= n (the phantom column of an odd n) idle. */
static int jacobi_pair(double *A, double *V, int m, int n, int p, int q, double tol,
                       double delta2) {
  if (p >= n || q >= n) return 0;
  if (p > q) { const int t = p; p = q; q = t; }
  double *ap = A + (size_t)p * m, *aq = A + (size_t)q * m;
  double al = 0.0, be = 0.0, ga = 0.0;
#pragma omp simd reduction(+ : al, be, ga)
  for (int i = 0; i < m; ++i) {
    al += ap[i] * ap[i];
    be += aq[i] * aq[i];
    ga += ap[i] * aq[i];
  }
  if (al <= delta2 || be <= delta2 || !(fabs(ga) > tol * sqrt(al) * sqrt(be))) return 0;
  const double zeta = (be - al) / (2.0 * ga);
  const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double c = 1.0 / sqrt(1.0 + t * t);
  const double s = c * t;
#pragma omp simd
  for (int i = 0; i < m; ++i) {
    const double x = ap[i], y = aq[i];
    ap[i] = c * x - s * y;
    aq[i] = s * x + c * y;
  }
  double *vp = V + (size_t)p * n, *vq = V + (size_t)q * n;
#pragma omp simd
  for (int i = 0; i < n; ++i) {
    const double x = vp[i], y = vq[i];
    vp[i] = c * x - s * y;
    vq[i] = s * x + c * y;
  }
  return 1;
}

/* SVD of one block given column-major in A (m x n, m >= n; overwritten by U diag(s)).
 * V (n x n column-major) receives the right vectors, s the singular values (unsorted).
 * Returns the sweeps run. */
static int jacobi_one(double *A, double *V, double *s, int m, int n, int max_sweeps) {
  const double tol = (double)(m > 32 ? m : 32) * ldexp(1.0, -52);
  double f2 = 0.0;
  for (size_t e = 0; e < (size_t)m * n; ++e) f2 += A[e] * A[e];
  const double delta = ldexp(sqrt(f2), -52), delta2 = delta * delta;
  memset(V, 0, sizeof(double) * (size_t)n * n);
  for (int j = 0; j < n; ++j) V[(size_t)j * n + j] = 1.0;
  const int n2 = n + (n & 1);
  int sweeps = 0;
  if (n > 1) {
    for (; sweeps < max_sweeps;) {
      int rotated = 0;
      for (int r = 0; r < n2 - 1; ++r)
        for (int k = 0; k < n2 / 2; ++k) {
          int a, b;
          rr_pair(r, k, n2, &a, &b);
          rotated |= jacobi_pair(A, V, m, n, a, b, tol, delta2);
        }
      ++sweeps;
      if (!rotated) break;
    }
  }
  for (int j = 0; j < n; ++j) {
    const double *a = A + (size_t)j * m;
    double nn = 0.0;
    for (int i = 0; i < m; ++i) nn += a[i] * a[i];
    s[j] = nn > delta2 ? sqrt(nn) : 0.0;
  }
  return sweeps;
}

/* Batched SVD: B holds nb blocks, each m x n row-major (m >= n). Outputs per block:
 * U (m x n row-major, columns u_j; a column with sigma_j = 0 is zero), s (n), V (n x n
 * row-major, columns v_j), sweeps. Returns the largest sweep count, or -1 if a block
 * did not converge within max_sweeps. */
int msld_oracle_jacobi_svd(int nb, int m, int n, const double *B, double *U, double *s,
                           double *V, int *sweeps, int max_sweeps) {
  if (nb <= 0 || m <= 0 || n <= 0 || m < n) return nb == 0 ? 0 : -2;
  int worst = 0, fail = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(max : worst) reduction(| : fail)
  for (int b = 0; b < nb; ++b) {
    double *A = (double *)malloc(sizeof(double) * (size_t)m * n);
    double *W = (double *)malloc(sizeof(double) * (size_t)n * n);
    const double *src = B + (size_t)b * m * n;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < n; ++j) A[(size_t)j * m + i] = src[(size_t)i * n + j];
    double *sb = s + (size_t)b * n;
    const int sw = jacobi_one(A, W, sb, m, n, max_sweeps);
    if (sw >= max_sweeps && max_sweeps > 0) {
      /* the last sweep may still have rotated: check orthogonality once more */
      const double tol = (double)(m > 32 ? m : 32) * ldexp(1.0, -52);
      for (int p = 0; p < n && !fail; ++p)
        for (int q = p + 1; q < n; ++q) {
          const double *ap = A + (size_t)p * m, *aq = A + (size_t)q * m;
          double al = 0.0, be = 0.0, ga = 0.0;
          for (int i = 0; i < m; ++i) {
            al += ap[i] * ap[i];
            be += aq[i] * aq[i];
            ga += ap[i] * aq[i];
          }
          if (sb[p] > 0.0 && sb[q] > 0.0 && fabs(ga) > tol * sqrt(al) * sqrt(be)) {
            fail = 1;
            break;
          }
        }
    }
    sweeps[b] = sw;
    if (sw > worst) worst = sw;
    double *ub = U + (size_t)b * m * n;
    for (int j = 0; j < n; ++j) {
      const double inv = sb[j] > 0.0 ? 1.0 / sb[j] : 0.0;
      for (int i = 0; i < m; ++i) ub[(size_t)i * n + j] = A[(size_t)j * m + i] * inv;
    }
    double *vb = V + (size_t)b * n * n;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) vb[(size_t)i * n + j] = W[(size_t)j * n + i];
    free(A);
    free(W);
  }
  return fail ? -1 : worst;
}
