/*
 * FP64 CPU oracle for blockwise matrix inversion.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no code with the HIP path.
 *
 * Every routine is the plain, slow, obviously-correct form of what it computes:
 * row-major n x n double matrices, naive loops, OpenMP only across independent
 * output rows (which leaves the per-element arithmetic unchanged).
 *
 *   orc_gj_inverse         Gauss-Jordan with partial pivoting: the plain
 *                          definition of X = A^-1 (the standard method the
 *                          paper names as the usual alternative, §5.7).
 *   orc_blockwise_inverse  The out-of-place recursive blockwise inversion of
 *                          Eq. (a) (§3), in the product order of the
 *                          invertor_by_a procedure (§4.1), with closed-form
 *                          leaves of order <= 4 (§5.1).  Independent of
 *                          orc_gj_inverse: no code in common.
 *   orc_partial_sweep      The state after eliminating the leading h x h block:
 *                          [[A11^-1, A11^-1 A12], [-A21 A11^-1, A22 - A21 A11^-1 A12]],
 *                          i.e. Eq. (a)'s first half; built from orc_gj_inverse.
 *   orc_residual_rows      Selected rows of R = A X - I with compensated (Dot2,
 *                          Ogita-Rump-Oishi 2005) dot products, so the residual
 *                          is measured at about twice working precision.
 *   orc_ns_step            One Newton-Schulz step X + X (I - A X), plain FP64.
 *   orc_matmul             C = A B, plain i-k-j loop (for pins and tests).
 *
 * Singularity convention: a pivot (or a leaf determinant) that is exactly 0.0
 * makes the routine return the 1-based global row concerned; 0 means success.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define IDX(i, j, ld) ((size_t)(i) * (size_t)(ld) + (size_t)(j))

/* ------------------------------------------------------------------------ */
/* O1: Gauss-Jordan with partial pivoting (first maximum wins).              */
/* ------------------------------------------------------------------------ */
int64_t orc_gj_inverse(int64_t n, const double* A, double* X) {
  if (n <= 0) return 0;
  memcpy(X, A, sizeof(double) * (size_t)n * (size_t)n);
  int64_t* swap_r = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  if (!swap_r) return -1;
  for (int64_t c = 0; c < n; ++c) {
    /* pivot search in column c, rows c..n-1; the lowest row index wins ties */
    int64_t r = c;
    double best = fabs(X[IDX(c, c, n)]);
    for (int64_t i = c + 1; i < n; ++i) {
      double v = fabs(X[IDX(i, c, n)]);
      if (v > best) { best = v; r = i; }
    }
    if (X[IDX(r, c, n)] == 0.0) { free(swap_r); return c + 1; }
    swap_r[c] = r;
    if (r != c) {
      for (int64_t j = 0; j < n; ++j) {
        double t = X[IDX(c, j, n)];
        X[IDX(c, j, n)] = X[IDX(r, j, n)];
        X[IDX(r, j, n)] = t;
      }
    }
    /* scale the pivot row by q = 1/pivot; the pivot position becomes q */
    double q = 1.0 / X[IDX(c, c, n)];
    X[IDX(c, c, n)] = 1.0;
    for (int64_t j = 0; j < n; ++j) X[IDX(c, j, n)] *= q;
    /* eliminate column c from every other row; column c receives -f*q */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      if (i == c) continue;
      double f = X[IDX(i, c, n)];
      X[IDX(i, c, n)] = 0.0;
      if (f == 0.0) continue;
      for (int64_t j = 0; j < n; ++j) X[IDX(i, j, n)] -= f * X[IDX(c, j, n)];
    }
  }
  /* undo the row interchanges as column interchanges, in reverse order */
  for (int64_t c = n - 1; c >= 0; --c) {
    int64_t r = swap_r[c];
    if (r == c) continue;
    for (int64_t i = 0; i < n; ++i) {
      double t = X[IDX(i, c, n)];
      X[IDX(i, c, n)] = X[IDX(i, r, n)];
      X[IDX(i, r, n)] = t;
    }
  }
  free(swap_r);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Plain products on strided sub-blocks.                                     */
/* ------------------------------------------------------------------------ */

/* C (m x p, ldc) = alpha * A (m x q, lda) * B (q x p, ldb) + beta * Cin (ldci)
 * Cin may alias C (elementwise read then write) or be NULL (beta ignored). */
static void mm(int64_t m, int64_t q, int64_t p, double alpha,
               const double* A, int64_t lda, const double* B, int64_t ldb,
               const double* Cin, int64_t ldci, double* C, int64_t ldc) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    double* row = (double*)malloc(sizeof(double) * (size_t)(p > 0 ? p : 1));
    for (int64_t j = 0; j < p; ++j) row[j] = 0.0;
    for (int64_t t = 0; t < q; ++t) {
      double a = A[IDX(i, t, lda)];
      for (int64_t j = 0; j < p; ++j) row[j] += a * B[IDX(t, j, ldb)];
    }
    for (int64_t j = 0; j < p; ++j) {
      double v = alpha * row[j];
      if (Cin) v += Cin[IDX(i, j, ldci)];
      C[IDX(i, j, ldc)] = v;
    }
    free(row);
  }
}

void orc_matmul(int64_t m, int64_t q, int64_t p, const double* A, const double* B, double* C) {
  mm(m, q, p, 1.0, A, q, B, p, NULL, 0, C, p);
}

/* ------------------------------------------------------------------------ */
/* O2: recursive blockwise inversion by Eq. (a), invertor_by_a order.        */
/* ------------------------------------------------------------------------ */

/* Closed-form inverse of an order-m block (m <= 4) by adjugate / determinant
 * (§5.1 inverts the small diagonal blocks with algebraic expressions).
 * Returns 0, or 1 if the determinant is exactly zero. */
static int leaf_inverse(int64_t m, const double* a, int64_t lda, double* x, int64_t ldx) {
#define a_(i, j) a[IDX(i, j, lda)]
#define x_(i, j) x[IDX(i, j, ldx)]
  if (m == 1) {
    if (a_(0, 0) == 0.0) return 1;
    x_(0, 0) = 1.0 / a_(0, 0);
    return 0;
  }
  if (m == 2) {
    double det = a_(0, 0) * a_(1, 1) - a_(0, 1) * a_(1, 0);
    if (det == 0.0) return 1;
    double id = 1.0 / det;
    double a00 = a_(0, 0), a01 = a_(0, 1), a10 = a_(1, 0), a11 = a_(1, 1);
    x_(0, 0) = a11 * id;  x_(0, 1) = -a01 * id;
    x_(1, 0) = -a10 * id; x_(1, 1) = a00 * id;
    return 0;
  }
  if (m == 3) {
    /* cofactors C_ij; inverse = C^T / det */
    double c[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        int r0 = (i + 1) % 3, r1 = (i + 2) % 3, s0 = (j + 1) % 3, s1 = (j + 2) % 3;
        /* cyclic index order gives the cofactor sign automatically */
        c[i][j] = a_(r0, s0) * a_(r1, s1) - a_(r0, s1) * a_(r1, s0);
      }
    double det = a_(0, 0) * c[0][0] + a_(0, 1) * c[0][1] + a_(0, 2) * c[0][2];
    if (det == 0.0) return 1;
    double id = 1.0 / det;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) x_(i, j) = c[j][i] * id;
    return 0;
  }
  if (m == 4) {
    /* Laplace expansion by complementary 2x2 minors of rows {0,1} and {2,3}. */
    double b[4][4];
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) b[i][j] = a_(i, j);
    double s0 = b[0][0] * b[1][1] - b[1][0] * b[0][1];
    double s1 = b[0][0] * b[1][2] - b[1][0] * b[0][2];
    double s2 = b[0][0] * b[1][3] - b[1][0] * b[0][3];
    double s3 = b[0][1] * b[1][2] - b[1][1] * b[0][2];
    double s4 = b[0][1] * b[1][3] - b[1][1] * b[0][3];
    double s5 = b[0][2] * b[1][3] - b[1][2] * b[0][3];
    double c5 = b[2][2] * b[3][3] - b[3][2] * b[2][3];
    double c4 = b[2][1] * b[3][3] - b[3][1] * b[2][3];
    double c3 = b[2][1] * b[3][2] - b[3][1] * b[2][2];
    double c2 = b[2][0] * b[3][3] - b[3][0] * b[2][3];
    double c1 = b[2][0] * b[3][2] - b[3][0] * b[2][2];
    double c0 = b[2][0] * b[3][1] - b[3][0] * b[2][1];
    double det = s0 * c5 - s1 * c4 + s2 * c3 + s3 * c2 - s4 * c1 + s5 * c0;
    if (det == 0.0) return 1;
    double id = 1.0 / det;
    x_(0, 0) = ( b[1][1] * c5 - b[1][2] * c4 + b[1][3] * c3) * id;
    x_(0, 1) = (-b[0][1] * c5 + b[0][2] * c4 - b[0][3] * c3) * id;
    x_(0, 2) = ( b[3][1] * s5 - b[3][2] * s4 + b[3][3] * s3) * id;
    x_(0, 3) = (-b[2][1] * s5 + b[2][2] * s4 - b[2][3] * s3) * id;
    x_(1, 0) = (-b[1][0] * c5 + b[1][2] * c2 - b[1][3] * c1) * id;
    x_(1, 1) = ( b[0][0] * c5 - b[0][2] * c2 + b[0][3] * c1) * id;
    x_(1, 2) = (-b[3][0] * s5 + b[3][2] * s2 - b[3][3] * s1) * id;
    x_(1, 3) = ( b[2][0] * s5 - b[2][2] * s2 + b[2][3] * s1) * id;
    x_(2, 0) = ( b[1][0] * c4 - b[1][1] * c2 + b[1][3] * c0) * id;
    x_(2, 1) = (-b[0][0] * c4 + b[0][1] * c2 - b[0][3] * c0) * id;
    x_(2, 2) = ( b[3][0] * s4 - b[3][1] * s2 + b[3][3] * s0) * id;
    x_(2, 3) = (-b[2][0] * s4 + b[2][1] * s2 - b[2][3] * s0) * id;
    x_(3, 0) = (-b[1][0] * c3 + b[1][1] * c1 - b[1][2] * c0) * id;
    x_(3, 1) = ( b[0][0] * c3 - b[0][1] * c1 + b[0][2] * c0) * id;
    x_(3, 2) = (-b[3][0] * s3 + b[3][1] * s1 - b[3][2] * s0) * id;
    x_(3, 3) = ( b[2][0] * s3 - b[2][1] * s1 + b[2][2] * s0) * id;
    return 0;
  }
#undef a_
#undef x_
  return 1;
}

/* Invert the m x m block a (lda) into x (ldx) whose diagonal blocks have the
 * orders part[0..k).  row0 is the block's first global row (for error
 * reporting).  Eq. (a) with A the leading floor(k/2) blocks:
 *   nAiB = -A^-1 B,  CAi = C A^-1            (the two products computed first)
 *   S    = D + C nAiB                        (Schur complement, reduction 1)
 *   Si   = S^-1                              (recursive)
 *   X12  = nAiB Si,  X21 = -Si CAi           (= -A^-1 B S^-1, -S^-1 C A^-1)
 *   X11  = A^-1 + nAiB X21                   (reduction 2), X22 = Si.
 * A single block larger than 4 is split into halves of its order, so every
 * leaf is a closed-form inverse of order <= 4. */
static int64_t by_a(int64_t m, const double* a, int64_t lda, int32_t k, const int32_t* part,
                    double* x, int64_t ldx, int64_t row0) {
  if (m == 0) return 0;
  int32_t split_part[2];
  if (k == 1) {
    if (m <= 4) return leaf_inverse(m, a, lda, x, ldx) ? row0 + 1 : 0;
    split_part[0] = (int32_t)(m / 2);
    split_part[1] = (int32_t)(m - m / 2);
    part = split_part;
    k = 2;
  }
  int32_t h = k / 2;
  int64_t ma = 0;
  for (int32_t i = 0; i < h; ++i) ma += part[i];
  int64_t md = m - ma;
  const double* A = a;
  const double* B = a + ma;
  const double* C = a + (size_t)ma * lda;
  const double* D = a + (size_t)ma * lda + ma;
  double* X11 = x;
  double* X12 = x + ma;
  double* X21 = x + (size_t)ma * ldx;
  double* X22 = x + (size_t)ma * ldx + ma;

  double* Ai = (double*)malloc(sizeof(double) * (size_t)(ma * ma));
  double* nAiB = (double*)malloc(sizeof(double) * (size_t)(ma * md));
  double* CAi = (double*)malloc(sizeof(double) * (size_t)(md * ma));
  double* S = (double*)malloc(sizeof(double) * (size_t)(md * md));
  int64_t info = -1;
  if (!Ai || !nAiB || !CAi || !S) goto done;

  info = by_a(ma, A, lda, h, part, Ai, ma, row0);
  if (info) goto done;
  mm(ma, ma, md, -1.0, Ai, ma, B, lda, NULL, 0, nAiB, md);   /* -A^-1 B */
  mm(md, ma, ma, 1.0, C, lda, Ai, ma, NULL, 0, CAi, ma);     /* C A^-1  */
  mm(md, ma, md, 1.0, C, lda, nAiB, md, D, lda, S, md);      /* D - C A^-1 B */
  info = by_a(md, S, md, k - h, part + h, X22, ldx, row0 + ma); /* S^-1 into X22 */
  if (info) goto done;
  mm(ma, md, md, 1.0, nAiB, md, X22, ldx, NULL, 0, X12, ldx);     /* -A^-1 B S^-1 */
  mm(md, md, ma, -1.0, X22, ldx, CAi, ma, NULL, 0, X21, ldx);     /* -S^-1 C A^-1 */
  mm(ma, md, ma, 1.0, nAiB, md, X21, ldx, Ai, ma, X11, ldx);      /* A^-1 + A^-1 B S^-1 C A^-1 */
done:
  free(Ai); free(nAiB); free(CAi); free(S);
  return info;
}

/* part == NULL or k <= 0: a single block of order n (recursive halving). */
int64_t orc_blockwise_inverse(int64_t n, const double* A, int32_t k, const int32_t* part, double* X) {
  if (n <= 0) return 0;
  int32_t one = (int32_t)n;
  if (!part || k <= 0) { part = &one; k = 1; }
  int64_t s = 0;
  for (int32_t i = 0; i < k; ++i) { if (part[i] <= 0) return -2; s += part[i]; }
  if (s != n) return -2;
  return by_a(n, A, n, k, part, X, n, 0);
}

/* ------------------------------------------------------------------------ */
/* Partial sweep after eliminating the leading h x h block.                  */
/* ------------------------------------------------------------------------ */
int64_t orc_partial_sweep(int64_t n, const double* A, int64_t h, double* W) {
  if (h <= 0) { memcpy(W, A, sizeof(double) * (size_t)(n * n)); return 0; }
  int64_t r = n - h;
  double* A11 = (double*)malloc(sizeof(double) * (size_t)(h * h));
  double* Ai = (double*)malloc(sizeof(double) * (size_t)(h * h));
  int64_t info = -1;
  if (!A11 || !Ai) goto done;
  for (int64_t i = 0; i < h; ++i) memcpy(A11 + i * h, A + i * n, sizeof(double) * (size_t)h);
  info = orc_gj_inverse(h, A11, Ai);
  if (info) goto done;
  for (int64_t i = 0; i < h; ++i) memcpy(W + i * n, Ai + i * h, sizeof(double) * (size_t)h);
  if (r > 0) {
    mm(h, h, r, 1.0, Ai, h, A + h, n, NULL, 0, W + h, n);                       /* A11^-1 A12 */
    mm(r, h, h, -1.0, A + (size_t)h * n, n, Ai, h, NULL, 0, W + (size_t)h * n, n); /* -A21 A11^-1 */
    /* A22 - A21 (A11^-1 A12), using the row panel just formed */
    mm(r, h, r, -1.0, A + (size_t)h * n, n, W + h, n, A + (size_t)h * n + h, n, W + (size_t)h * n + h, n);
  }
done:
  free(A11); free(Ai);
  return info;
}

/* ------------------------------------------------------------------------ */
/* O3: compensated residual rows of R = A X - I.                             */
/* ------------------------------------------------------------------------ */
static inline void two_sum(double a, double b, double* s, double* e) {
  double x = a + b;
  double z = x - a;
  *e = (a - (x - z)) + (b - z);
  *s = x;
}

/* rows[0..nr) are the row indices of R to produce, written row by row to R
 * (nr x n).  Dot2: products split exactly by fma, sums by TwoSum. */
void orc_residual_rows(int64_t n, const double* A, const double* X, int64_t nr,
                       const int64_t* rows, double* R) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t t = 0; t < nr; ++t) {
    int64_t i = rows[t];
    double* s = (double*)malloc(sizeof(double) * (size_t)n);
    double* c = (double*)malloc(sizeof(double) * (size_t)n);
    for (int64_t j = 0; j < n; ++j) { s[j] = (i == j) ? -1.0 : 0.0; c[j] = 0.0; }
    for (int64_t q = 0; q < n; ++q) {
      double a = A[IDX(i, q, n)];
      if (a == 0.0) continue;
      const double* xr = X + (size_t)q * n;
      for (int64_t j = 0; j < n; ++j) {
        double p = a * xr[j];
        double pe = fma(a, xr[j], -p);
        double ss, se;
        two_sum(s[j], p, &ss, &se);
        s[j] = ss;
        c[j] += se + pe;
      }
    }
    for (int64_t j = 0; j < n; ++j) R[IDX(t, j, n)] = s[j] + c[j];
    free(s); free(c);
  }
}

/* ------------------------------------------------------------------------ */
/* O4: one Newton-Schulz step X_next = X + X (I - A X), plain FP64.          */
/* ------------------------------------------------------------------------ */
int64_t orc_ns_step(int64_t n, const double* A, const double* X, double* Xnext) {
  double* R = (double*)malloc(sizeof(double) * (size_t)(n * n));
  if (!R) return -1;
  /* R = I - A X */
  mm(n, n, n, -1.0, A, n, X, n, NULL, 0, R, n);
  for (int64_t i = 0; i < n; ++i) R[IDX(i, i, n)] += 1.0;
  /* X_next = X + X R */
  mm(n, n, n, 1.0, X, n, R, n, X, n, Xnext, n);
  free(R);
  return 0;
}
