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
 *   orc_block_gj           Block Gauss-Jordan over a partition (Eq. (a)
 *                          unrolled one diagonal block at a time, §4.2),
 *                          without pivoting across blocks or with block-row
 *                          pivoting by tournament selection: the two readings
 *                          the GPU path implements (see its comment).
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

/* ------------------------------------------------------------------------ */
/* O6: block Gauss-Jordan over a partition, in the two readings the GPU      */
/* path implements.  Test infrastructure: it follows the steps of the        */
/* unrolled in-place Eq. (a) (§3, §4.2) one diagonal block at a time, in     */
/* plain loops, and shares nothing with the HIP code.                        */
/*                                                                           */
/* pivot = 0  (the paper's method: no pivoting across blocks, §3)            */
/*   P = W_pp^-1: Gauss-Jordan with partial pivoting inside the block when   */
/*       b <= 128, else block Gauss-Jordan on the block with `sub`-wide      */
/*       sub-blocks, each sub-block's leaf inverted by Gauss-Jordan with     */
/*       partial pivoting inside that leaf;                                  */
/*   R = P W[p, :] with R[:, p] = P (row panel);                             */
/*   W[i, j] -= W[i, p] R[:, j] (j outside p), W[i, p] = -W[i, p] P          */
/*       for every row i outside p, then W[p, :] = R.                        */
/*                                                                           */
/* pivot = 1  (block-row pivoting, the re-blocking remedy of §3 taken to     */
/*   rows: the counter-diagonal Eqs. (b)/(c) are Eq. (a) on a block-row      */
/*   permuted matrix; here the rows that form the pivot block are chosen):   */
/*   - the b pivot rows come from rows o..n-1 by tournament selection over   */
/*     `sub`-wide column strips of the block's current columns: leaves are   */
/*     chunks of `leaf_rows` consecutive rows (rows already chosen left      */
/*     out), each node keeps the rows Gauss elimination with partial         */
/*     pivoting picks among its candidates (the lowest candidate position    */
/*     wins ties), `arity` consecutive nodes merge into one, and the root's  */
/*     picks in pick order are the strip's pivot rows; the strip is then     */
/*     eliminated from the block's later columns of every row (through the   */
/*     inverse of the picked rows' strip block, Gauss-Jordan with partial    */
/*     pivoting);                                                            */
/*   - the picked rows move to positions o..o+b-1 in pick order, the rows    */
/*     they displace take the vacated positions in ascending order;          */
/*   - R = the pivot rows after block Gauss-Jordan with `sub`-wide           */
/*     sub-blocks on their b x b block, applied to all n columns (so R's     */
/*     p columns hold P and the others P W[p, :] formed by the same          */
/*     sub-block row operations);                                            */
/*   - the update of the other rows as above;                                */
/*   - at the end, column perm[c] of X is column c of W (perm[c] = the       */
/*     original row at position c), which undoes the row moves.              */
/* Returns 0, the 1-based row (pivot position) of an exactly-zero pivot, or  */
/* < 0 on bad arguments.  perm_out (may be NULL): the final row order.       */
/* ------------------------------------------------------------------------ */

/* Gauss elimination with partial pivoting on the nc candidate rows cand[] of
 * the panel T (rows indexed from o, ld ldt) over columns [c0, c0 + w).
 * Writes up to w picked rows (in pick order) to win[] and returns how many;
 * *zero (if not NULL) becomes the first column index whose pick had a zero
 * value, else -1. */
static int64_t gepp_pick(int64_t nc, const int64_t* cand, const double* T, int64_t ldt, int64_t o, int64_t c0,
                         int64_t w, int64_t* win, int64_t* zero) {
  double* V = (double*)malloc(sizeof(double) * (size_t)(nc * w + 1));
  char* used = (char*)calloc((size_t)nc + 1, 1);
  int64_t got = 0;
  if (zero) *zero = -1;
  for (int64_t i = 0; i < nc; ++i)
    for (int64_t j = 0; j < w; ++j) V[i * w + j] = T[IDX(cand[i] - o, c0 + j, ldt)];
  for (int64_t c = 0; c < w && got < nc; ++c) {
    int64_t r = -1;
    double best = -1.0;
    for (int64_t i = 0; i < nc; ++i) {
      if (used[i]) continue;
      double v = fabs(V[i * w + c]);
      if (v > best) { best = v; r = i; }
    }
    if (r < 0) break;
    used[r] = 1;
    win[got++] = cand[r];
    double pv = V[r * w + c];
    if (pv == 0.0) {
      if (zero && *zero < 0) *zero = c;
      continue;
    }
    double q = 1.0 / pv;
    for (int64_t i = 0; i < nc; ++i) {
      if (used[i]) continue;
      double l = V[i * w + c] * q;
      for (int64_t j = c + 1; j < w; ++j) V[i * w + j] -= l * V[r * w + j];
    }
  }
  free(V); free(used);
  return got;
}

/* Tournament over rows [o, n) not yet chosen (chosen_flag[row - o] != 0),
 * strip [c0, c0 + w) of the panel T.  Writes the w root picks to out[] and
 * returns the root's first zero-pivot column (or -1). */
static int64_t tournament(const double* T, int64_t ldt, int64_t o, int64_t n, const char* chosen_flag, int64_t c0,
                          int64_t w, int64_t leaf_rows, int64_t arity, int64_t* out) {
  int64_t nleaf = (n - o + leaf_rows - 1) / leaf_rows;
  int64_t* nodes = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nleaf * w + 1));
  int64_t* ncount = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nleaf + 1));
  int64_t* cand = (int64_t*)malloc(sizeof(int64_t) * (size_t)((leaf_rows > arity * w ? leaf_rows : arity * w) + 1));
  int64_t zero = -1;
  for (int64_t l = 0; l < nleaf; ++l) {
    int64_t nc = 0;
    for (int64_t r = o + l * leaf_rows; r < o + (l + 1) * leaf_rows && r < n; ++r)
      if (!chosen_flag[r - o]) cand[nc++] = r;
    ncount[l] = gepp_pick(nc, cand, T, ldt, o, c0, w, nodes + l * w, &zero);
  }
  int64_t nn = nleaf;
  while (nn > 1) {
    int64_t m = (nn + arity - 1) / arity;
    for (int64_t g = 0; g < m; ++g) {
      int64_t nc = 0;
      for (int64_t ch = g * arity; ch < (g + 1) * arity && ch < nn; ++ch)
        for (int64_t t = 0; t < ncount[ch]; ++t) cand[nc++] = nodes[ch * w + t];
      /* node g's picks overwrite slot g, which no later group reads */
      ncount[g] = gepp_pick(nc, cand, T, ldt, o, c0, w, nodes + g * w, &zero);
    }
    nn = m;
  }
  for (int64_t t = 0; t < w; ++t) out[t] = nodes[t];
  free(nodes); free(ncount); free(cand);
  return zero;
}

/* Block Gauss-Jordan on the b pivot rows M (b x ncols, ld ldm) with their
 * b x b block at columns [co, co + b): sub-block s (rows and columns
 * [s0, s0 + sb) of the block) in turn: Q = GJ-PP inverse of its current
 * leaf, its rows become Q times themselves (their leaf columns Q), every
 * other row i subtracts (its leaf-column values) times those new rows (its
 * leaf columns becoming -(values) Q).  Afterwards M[:, co:co+b] = block^-1
 * and the other columns hold block^-1 times their original values.
 * Returns 0 or the 1-based row (within the block) of a zero leaf pivot. */
static int64_t rows_block_gj(int64_t b, double* M, int64_t ldm, int64_t ncols, int64_t co, int64_t sub) {
  double* leaf = (double*)malloc(sizeof(double) * (size_t)(sub * sub));
  double* Q = (double*)malloc(sizeof(double) * (size_t)(sub * sub));
  double* Rj = (double*)malloc(sizeof(double) * (size_t)(sub * ncols));
  double* c = (double*)malloc(sizeof(double) * (size_t)sub);
  int64_t info = 0;
  for (int64_t s0 = 0; s0 < b; s0 += sub) {
    int64_t sb = b - s0 < sub ? b - s0 : sub;
    for (int64_t i = 0; i < sb; ++i)
      for (int64_t j = 0; j < sb; ++j) leaf[i * sb + j] = M[IDX(s0 + i, co + s0 + j, ldm)];
    int64_t e = orc_gj_inverse(sb, leaf, Q);
    if (e) { info = s0 + e; break; }
    /* Rj = Q * M[s0 rows, :], with Q in the leaf columns */
    for (int64_t i = 0; i < sb; ++i)
      for (int64_t j = 0; j < ncols; ++j) {
        double acc = 0.0;
        for (int64_t t = 0; t < sb; ++t) acc += Q[i * sb + t] * M[IDX(s0 + t, j, ldm)];
        Rj[i * ncols + j] = acc;
      }
    for (int64_t i = 0; i < sb; ++i)
      for (int64_t j = 0; j < sb; ++j) Rj[i * ncols + co + s0 + j] = Q[i * sb + j];
    for (int64_t i = 0; i < b; ++i) {
      if (i >= s0 && i < s0 + sb) continue;
      for (int64_t t = 0; t < sb; ++t) c[t] = M[IDX(i, co + s0 + t, ldm)];
      for (int64_t j = 0; j < ncols; ++j) {
        int in_leaf = (j >= co + s0 && j < co + s0 + sb);
        double acc = 0.0;
        for (int64_t t = 0; t < sb; ++t) acc += c[t] * Rj[t * ncols + j];
        M[IDX(i, j, ldm)] = (in_leaf ? 0.0 : M[IDX(i, j, ldm)]) - acc;
      }
    }
    for (int64_t i = 0; i < sb; ++i)
      for (int64_t j = 0; j < ncols; ++j) M[IDX(s0 + i, j, ldm)] = Rj[i * ncols + j];
  }
  free(leaf); free(Q); free(Rj); free(c);
  return info;
}

int64_t orc_block_gj(int64_t n, const double* A, int32_t k, const int32_t* part, int32_t pivot, int32_t sub,
                     int32_t leaf_rows, int32_t arity, double* X, int64_t* perm_out) {
  if (n < 0 || sub <= 0 || leaf_rows <= 0 || arity < 2) return -2;
  if (n == 0) return 0;
  int32_t one = (int32_t)n;
  if (!part || k <= 0) { part = &one; k = 1; }
  int64_t s = 0;
  for (int32_t i = 0; i < k; ++i) { if (part[i] <= 0) return -2; s += part[i]; }
  if (s != n) return -2;
  int64_t bmax = 0;
  for (int32_t i = 0; i < k; ++i) if (part[i] > bmax) bmax = part[i];

  double* W = (double*)malloc(sizeof(double) * (size_t)(n * n));
  double* Wn = (double*)malloc(sizeof(double) * (size_t)(n * n));
  int64_t* perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  int64_t* src = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
  double* R = (double*)malloc(sizeof(double) * (size_t)(bmax * n));
  double* P = (double*)malloc(sizeof(double) * (size_t)(bmax * bmax));
  double* blk = (double*)malloc(sizeof(double) * (size_t)(bmax * bmax));
  double* T = (double*)malloc(sizeof(double) * (size_t)(n * bmax));
  double* Q = (double*)malloc(sizeof(double) * (size_t)(sub * sub));
  double* G = (double*)malloc(sizeof(double) * (size_t)(sub * bmax));
  int64_t* chosen = (int64_t*)malloc(sizeof(int64_t) * (size_t)bmax);
  char* flag = (char*)malloc((size_t)n);
  int64_t info = -1;
  if (!W || !Wn || !perm || !src || !R || !P || !blk || !T || !Q || !G || !chosen || !flag) goto done;
  info = 0;
  memcpy(W, A, sizeof(double) * (size_t)(n * n));
  for (int64_t i = 0; i < n; ++i) perm[i] = i;

  int64_t o = 0;
  for (int32_t p = 0; p < k; o += part[p], ++p) {
    const int64_t b = part[p];
    if (pivot) {
      /* --- choose the b pivot rows among rows o..n-1 --- */
      const int64_t nr = n - o;
      for (int64_t i = 0; i < nr; ++i)
        for (int64_t t = 0; t < b; ++t) T[IDX(i, t, b)] = W[IDX(o + i, o + t, n)];
      memset(flag, 0, (size_t)nr);
      for (int64_t c0 = 0; c0 < b; c0 += sub) {
        const int64_t w = b - c0 < sub ? b - c0 : sub;
        int64_t z = tournament(T, b, o, n, flag, c0, w, leaf_rows, arity, chosen + c0);
        if (z >= 0) { info = o + c0 + z + 1; goto done; }
        for (int64_t t = 0; t < w; ++t) flag[chosen[c0 + t] - o] = 1;
        const int64_t rest = b - c0 - w;
        if (rest <= 0) continue;
        /* eliminate the strip from the block's later columns of every row */
        for (int64_t i = 0; i < w; ++i)
          for (int64_t j = 0; j < w; ++j) blk[i * w + j] = T[IDX(chosen[c0 + i] - o, c0 + j, b)];
        if (orc_gj_inverse(w, blk, Q)) { info = o + c0 + 1; goto done; }
        for (int64_t i = 0; i < w; ++i)
          for (int64_t j = 0; j < rest; ++j) {
            double acc = 0.0;
            for (int64_t t = 0; t < w; ++t) acc += Q[i * w + t] * T[IDX(chosen[c0 + t] - o, c0 + w + j, b)];
            G[i * rest + j] = acc;
          }
        for (int64_t i = 0; i < nr; ++i)
          for (int64_t j = 0; j < rest; ++j) {
            double acc = 0.0;
            for (int64_t t = 0; t < w; ++t) acc += T[IDX(i, c0 + t, b)] * G[t * rest + j];
            T[IDX(i, c0 + w + j, b)] -= acc;
          }
      }
      /* --- move: picked rows to o..o+b-1, displaced rows to the vacated slots --- */
      for (int64_t i = 0; i < n; ++i) src[i] = i;
      for (int64_t t = 0; t < b; ++t) src[o + t] = chosen[t];
      {
        int64_t dpos = o, vrow = o + b;
        for (;;) {
          while (dpos < o + b && flag[dpos - o]) ++dpos;   /* next displaced row */
          while (vrow < n && !flag[vrow - o]) ++vrow;      /* next vacated slot */
          if (dpos >= o + b || vrow >= n) break;
          src[vrow] = dpos;
          ++dpos; ++vrow;
        }
      }
      for (int64_t i = 0; i < n; ++i) memcpy(Wn + i * n, W + src[i] * n, sizeof(double) * (size_t)n);
      { double* t = W; W = Wn; Wn = t; }
      for (int64_t i = 0; i < n; ++i) src[i] = perm[src[i]];
      memcpy(perm, src, sizeof(int64_t) * (size_t)n);
      /* --- R by block Gauss-Jordan on the pivot rows --- */
      for (int64_t i = 0; i < b; ++i) memcpy(R + i * n, W + (o + i) * n, sizeof(double) * (size_t)n);
      int64_t e = rows_block_gj(b, R, n, n, o, sub);
      if (e) { info = o + e; goto done; }
      for (int64_t i = 0; i < b; ++i)
        for (int64_t j = 0; j < b; ++j) P[i * b + j] = R[IDX(i, o + j, n)];
    } else {
      for (int64_t i = 0; i < b; ++i)
        for (int64_t j = 0; j < b; ++j) blk[i * b + j] = W[IDX(o + i, o + j, n)];
      int64_t e;
      if (b <= 128) {
        e = orc_gj_inverse(b, blk, P);
      } else {
        e = rows_block_gj(b, blk, b, b, 0, sub);
        memcpy(P, blk, sizeof(double) * (size_t)(b * b));
      }
      if (e) { info = o + e; goto done; }
      /* R = P W[p, :], R[:, p] = P */
      for (int64_t i = 0; i < b; ++i)
        for (int64_t j = 0; j < n; ++j) {
          double acc = 0.0;
          for (int64_t t = 0; t < b; ++t) acc += P[i * b + t] * W[IDX(o + t, j, n)];
          R[i * n + j] = acc;
        }
      for (int64_t i = 0; i < b; ++i)
        for (int64_t j = 0; j < b; ++j) R[i * n + o + j] = P[i * b + j];
    }
    /* --- update every row outside block p, then the pivot rows --- */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      if (i >= o && i < o + b) continue;
      double* c = (double*)malloc(sizeof(double) * (size_t)b);
      for (int64_t t = 0; t < b; ++t) c[t] = W[IDX(i, o + t, n)];
      for (int64_t j = 0; j < n; ++j) {
        int jp = (j >= o && j < o + b);
        double acc = 0.0;
        for (int64_t t = 0; t < b; ++t) acc += c[t] * R[t * n + j];
        W[IDX(i, j, n)] = (jp ? 0.0 : W[IDX(i, j, n)]) - acc;
      }
      free(c);
    }
    for (int64_t i = 0; i < b; ++i) memcpy(W + (o + i) * n, R + i * n, sizeof(double) * (size_t)n);
  }
  /* undo the row moves: column perm[c] of X is column c of W */
  for (int64_t i = 0; i < n; ++i)
    for (int64_t c = 0; c < n; ++c) X[IDX(i, perm[c], n)] = W[IDX(i, c, n)];
  if (perm_out) memcpy(perm_out, perm, sizeof(int64_t) * (size_t)n);
done:
  free(W); free(Wn); free(perm); free(src); free(R); free(P); free(blk); free(T); free(Q); free(G);
  free(chosen); free(flag);
  return info;
}
