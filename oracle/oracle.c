/*
 * Plain CPU oracle for the panel-major dense linear algebra routines of
 * "BLASFEO: basic linear algebra subroutines for embedded optimization"
 * (Frison, Kouzoupis, Sartor, Zanelli, Diehl, arXiv 1704.02457).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library links, loads or calls
 * this file: only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header, table or helper with the HIP path.
 *
 * Storage: every matrix here is plain column-major FP64 (element (i,j) at
 * A[i + j*lda]), the format of the paper's reference implementation (§3.2),
 * not the panel-major format of the high-performance implementation.  All
 * loops are the textbook triple loops with the reduction index ascending;
 * there is no blocking, fusion or reordering.  Build with
 * `gcc -O2 -ffp-contract=off` so that no multiply-add is contracted.
 *
 * Each function states the passage of the paper it follows.  Readings of
 * passages that are silent or ambiguous are listed in the design notes.
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

#define EL(A, lda, i, j) (A)[(size_t)(i) + (size_t)(j) * (size_t)(lda)]

/* gemm_nt, Appendix A.2 (interface example): D <- alpha*A*B^T + beta*C with
 * A m-by-k, B n-by-k, C and D m-by-n; C and D may be the same array. */
void orc_dgemm_nt(int m, int n, int k, double alpha, const double *A, int lda,
                  const double *B, int ldb, double beta, const double *C,
                  int ldc, double *D, int ldd) {
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < m; ++i) {
      double s = 0.0;
      for (int l = 0; l < k; ++l) s += EL(A, lda, i, l) * EL(B, ldb, j, l);
      EL(D, ldd, i, j) = beta * EL(C, ldc, i, j) + alpha * s;
    }
}

/* gemm_nn, §4.4 (the NN variant of the gemm kernel: B read across panels)
 * and §5.2.2: D <- alpha*A*B + beta*C with A m-by-k, B k-by-n, C and D
 * m-by-n; C and D may be the same array. */
void orc_dgemm_nn(int m, int n, int k, double alpha, const double *A, int lda,
                  const double *B, int ldb, double beta, const double *C,
                  int ldc, double *D, int ldd) {
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < m; ++i) {
      double s = 0.0;
      for (int l = 0; l < k; ++l) s += EL(A, lda, i, l) * EL(B, ldb, l, j);
      EL(D, ldd, i, j) = beta * EL(C, ldc, i, j) + alpha * s;
    }
}

/* syrk_ln, §5.2.2 (syrk_ln paragraph): the lower triangle of
 * alpha*A*B^T + beta*C, where the two factors A and B (both m-by-k) may
 * differ.  The strictly upper part of D is neither read nor written. */
void orc_dsyrk_ln(int m, int k, double alpha, const double *A, int lda,
                  const double *B, int ldb, double beta, const double *C,
                  int ldc, double *D, int ldd) {
  for (int j = 0; j < m; ++j)
    for (int i = j; i < m; ++i) {
      double s = 0.0;
      for (int l = 0; l < k; ++l) s += EL(A, lda, i, l) * EL(B, ldb, j, l);
      EL(D, ldd, i, j) = beta * EL(C, ldc, i, j) + alpha * s;
    }
}

/* potrf_l, §5.2.2 (potrf_l paragraph) and §4.7.1 (inverse of the diagonal):
 * the lower Cholesky factor L of the symmetric matrix whose lower triangle
 * is C, so that L*L^T = C.  Column j of L follows from the definition
 *   L[j][j] = sqrt(C[j][j] - sum_{k<j} L[j][k]^2),
 *   L[i][j] = (C[i][j] - sum_{k<j} L[i][k]*L[j][k]) / L[j][j],  i > j,
 * where the division is a multiplication by the reciprocal 1/L[j][j], which
 * is also saved in dA[j] for later solves (§4.7.1).  Only the lower triangle
 * of C is read; C and D may be the same array.  Returns 0, or j+1 for the
 * first column whose pivot is not positive (LAPACK's info convention); the
 * columns before it are complete. */
int orc_dpotrf_l(int m, const double *C, int ldc, double *D, int ldd,
                 double *dA) {
  for (int j = 0; j < m; ++j) {
    double d = EL(C, ldc, j, j);
    for (int k = 0; k < j; ++k) d -= EL(D, ldd, j, k) * EL(D, ldd, j, k);
    if (!(d > 0.0)) return j + 1;
    double ljj = sqrt(d);
    double inv = 1.0 / ljj;
    EL(D, ldd, j, j) = ljj;
    if (dA) dA[j] = inv;
    for (int i = j + 1; i < m; ++i) {
      double s = EL(C, ldc, i, j);
      for (int k = 0; k < j; ++k) s -= EL(D, ldd, i, k) * EL(D, ldd, j, k);
      EL(D, ldd, i, j) = s * inv;
    }
  }
  return 0;
}

/* potrf_l_mn, §4.7.2 (stacking matrices): the non-square Cholesky
 * factorization of the stacked m-by-n matrix C = [H; A] (m >= n, H n-by-n
 * SPD): D = [L; A L^{-T}] with L L^T = H, i.e. potrf_l on the top block and
 * trsm_rltn on the rows below in one left-looking sweep over the n columns
 * (the rows run to m instead of n).  Only the lower triangle of the top
 * block and all of the bottom block are read.  dA[j] = 1/L[j][j] (n
 * entries).  Returns 0 or the 1-based index of the first pivot that is not
 * positive. */
int orc_dpotrf_l_mn(int m, int n, const double *C, int ldc, double *D,
                    int ldd, double *dA) {
  for (int j = 0; j < n; ++j) {
    double d = EL(C, ldc, j, j);
    for (int k = 0; k < j; ++k) d -= EL(D, ldd, j, k) * EL(D, ldd, j, k);
    if (!(d > 0.0)) return j + 1;
    double ljj = sqrt(d);
    double inv = 1.0 / ljj;
    EL(D, ldd, j, j) = ljj;
    if (dA) dA[j] = inv;
    for (int i = j + 1; i < m; ++i) {
      double s = EL(C, ldc, i, j);
      for (int k = 0; k < j; ++k) s -= EL(D, ldd, i, k) * EL(D, ldd, j, k);
      EL(D, ldd, i, j) = s * inv;
    }
  }
  return 0;
}

/* getrf, §5.2.2 (getrf paragraph: LU factorization with partial pivoting;
 * the routine list of the API names the pivot and nopivot variants): the
 * right-looking unblocked LU of the m-by-n matrix C into D.  For
 * k = 0..min(m,n)-1: with pivoting, p = the first row i >= k of largest
 * |D[i][k]| and rows k and p of D are swapped (ipiv[k] = p, 0-based);
 * without, ipiv[k] = k.  Then inv = 1/D[k][k], dA[k] = inv, the multipliers
 * D[i][k] *= inv (i > k) and the trailing update D[i][j] -= D[i][k]*D[k][j]
 * (i, j > k).  D holds L (unit lower, below the diagonal) and U (upper).
 * Returns 0, or k+1 for the first k with D[k][k] == 0 after the pivoting
 * (the factorization is still completed, as in LAPACK). */
int orc_dgetrf(int m, int n, const double *C, int ldc, double *D, int ldd,
               int *ipiv, double *dA, int pivot) {
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < m; ++i) EL(D, ldd, i, j) = EL(C, ldc, i, j);
  int info = 0;
  int mn = m < n ? m : n;
  for (int k = 0; k < mn; ++k) {
    int p = k;
    if (pivot) {
      double best = fabs(EL(D, ldd, k, k));
      for (int i = k + 1; i < m; ++i)
        if (fabs(EL(D, ldd, i, k)) > best) {
          best = fabs(EL(D, ldd, i, k));
          p = i;
        }
      if (p != k)
        for (int j = 0; j < n; ++j) {
          double t = EL(D, ldd, k, j);
          EL(D, ldd, k, j) = EL(D, ldd, p, j);
          EL(D, ldd, p, j) = t;
        }
    }
    ipiv[k] = p;
    double piv = EL(D, ldd, k, k);
    if (piv == 0.0 && info == 0) info = k + 1;
    double inv = 1.0 / piv;
    if (dA) dA[k] = inv;
    for (int i = k + 1; i < m; ++i) EL(D, ldd, i, k) *= inv;
    for (int j = k + 1; j < n; ++j)
      for (int i = k + 1; i < m; ++i) EL(D, ldd, i, j) -= EL(D, ldd, i, k) * EL(D, ldd, k, j);
  }
  return info;
}

/* gelqf, §5.2.2 (gelqf paragraph: the LQ factorization by Householder
 * reflectors, unblocked here): A = L Q.  For k = 0..min(m,n)-1 the
 * reflector H_k = I - tau_k v v' (v[k] = 1, v[j] = 0 for j < k) annihilates
 * D[k][k+1..n-1]: alpha = D[k][k], xn = sqrt(sum_{j>k} D[k][j]^2); if
 * xn == 0, tau_k = 0; else beta = -sign(alpha) sqrt(alpha^2 + xn^2),
 * tau_k = (beta - alpha)/beta, v[j] = D[k][j]/(alpha - beta) (stored in
 * D[k][j], j > k), D[k][k] = beta.  Then every row i > k is multiplied by
 * H_k from the right: w = D[i][k] + sum_{j>k} D[i][j] v[j],
 * D[i][k] -= tau w, D[i][j] -= tau w v[j].  On exit L is on and below the
 * diagonal of D, the reflectors above it (the compact form of LAPACK). */
void orc_dgelqf(int m, int n, const double *C, int ldc, double *D, int ldd,
                double *tau) {
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < m; ++i) EL(D, ldd, i, j) = EL(C, ldc, i, j);
  int mn = m < n ? m : n;
  for (int k = 0; k < mn; ++k) {
    double alpha = EL(D, ldd, k, k);
    double ss = 0.0;
    for (int j = k + 1; j < n; ++j) ss += EL(D, ldd, k, j) * EL(D, ldd, k, j);
    double xn = sqrt(ss);
    double t = 0.0;
    if (xn != 0.0) {
      double beta = -copysign(sqrt(alpha * alpha + ss), alpha);
      t = (beta - alpha) / beta;
      double sc = 1.0 / (alpha - beta);
      for (int j = k + 1; j < n; ++j) EL(D, ldd, k, j) *= sc;
      EL(D, ldd, k, k) = beta;
    }
    tau[k] = t;
    if (t == 0.0) continue;
    for (int i = k + 1; i < m; ++i) {
      double w = EL(D, ldd, i, k);
      for (int j = k + 1; j < n; ++j) w += EL(D, ldd, i, j) * EL(D, ldd, k, j);
      w *= t;
      EL(D, ldd, i, k) -= w;
      for (int j = k + 1; j < n; ++j) EL(D, ldd, i, j) -= w * EL(D, ldd, k, j);
    }
  }
}

/* trmm_rlnn, §5.2.2 (trmm paragraph; options right, lower, not transposed,
 * not unit) and §5.3 (the C step of the Riccati recursion):
 * D = alpha * B * A with A n-by-n lower triangular and B, D m-by-n, i.e.
 *   D[i][j] = alpha * sum_{k >= j} B[i][k] * A[k][j],  k ascending.
 * Only the lower triangle of A (diagonal included) is read.  D must not
 * overlap B or A. */
void orc_dtrmm_rlnn(int m, int n, double alpha, const double *A, int lda,
                    const double *B, int ldb, double *D, int ldd) {
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < m; ++i) {
      double s = 0.0;
      for (int k = j; k < n; ++k) s += EL(B, ldb, i, k) * EL(A, lda, k, j);
      EL(D, ldd, i, j) = alpha * s;
    }
}

/* trsm_rltn, §5.2.2 (trsm paragraph) and §4.7.2 (the A*L^-T step of the
 * range-space method): D = alpha * B * L^{-T} with L n-by-n lower triangular
 * (not unit) and B m-by-n, i.e. the X that solves X*L^T = alpha*B.  Row i of
 * X is found column by column,
 *   X[i][j] = (alpha*B[i][j] - sum_{k<j} X[i][k]*L[j][k]) * (1/L[j][j]).
 * Only the lower triangle of L is read.  B and D may be the same array. */
void orc_dtrsm_rltn(int m, int n, double alpha, const double *L, int ldl,
                    const double *B, int ldb, double *D, int ldd) {
  for (int j = 0; j < n; ++j) {
    double inv = 1.0 / EL(L, ldl, j, j);
    for (int i = 0; i < m; ++i) {
      double s = alpha * EL(B, ldb, i, j);
      for (int k = 0; k < j; ++k) s -= EL(D, ldd, i, k) * EL(L, ldl, j, k);
      EL(D, ldd, i, j) = s * inv;
    }
  }
}

/* syrk_potrf_ln, Appendix A.3 (LAPACK-like list) and §4.7.2 (concatenating
 * updates and downdates): L = chol(C + A*B^T), lower.  The oracle simply
 * runs syrk_ln (alpha = beta = 1) into a scratch matrix and then potrf_l;
 * the fused kernel computes the same mathematical result. */
int orc_dsyrk_dpotrf_ln(int m, int k, const double *A, int lda,
                        const double *B, int ldb, const double *C, int ldc,
                        double *D, int ldd, double *dA) {
  double *M = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1) *
                               (size_t)(m > 0 ? m : 1));
  if (!M) return -1;
  orc_dsyrk_ln(m, k, 1.0, A, lda, B, ldb, 1.0, C, ldc, M, m);
  int info = orc_dpotrf_l(m, M, m, D, ldd, dA);
  free(M);
  return info;
}

/* Cholesky solve with the lower factor L (trsv_lnn then trsv_ltn of the
 * level-2 list in Appendix A.3): for each of the nrhs columns b of B,
 * forward substitution L*y = b, then back substitution L^T*x = y.  Each
 * division is a multiplication by 1/L[j][j], the saved inverse diagonal of
 * §4.7.1. */
void orc_dpotrs_l(int n, int nrhs, const double *L, int ldl, const double *B,
                  int ldb, double *X, int ldx) {
  for (int r = 0; r < nrhs; ++r) {
    const double *b = B + (size_t)r * (size_t)ldb;
    double *x = X + (size_t)r * (size_t)ldx;
    for (int i = 0; i < n; ++i) {
      double s = b[i];
      for (int k = 0; k < i; ++k) s -= EL(L, ldl, i, k) * x[k];
      x[i] = s * (1.0 / EL(L, ldl, i, i));
    }
    for (int i = n - 1; i >= 0; --i) {
      double s = x[i];
      for (int k = i + 1; k < n; ++k) s -= EL(L, ldl, k, i) * x[k];
      x[i] = s * (1.0 / EL(L, ldl, i, i));
    }
  }
}

/* symv_l (level-2 list, Appendix A.3): z = alpha*A*x + beta*y with A
 * symmetric and only its lower triangle read. */
void orc_dsymv_l(int n, double alpha, const double *A, int lda,
                 const double *x, double beta, const double *y, double *z) {
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int k = 0; k < n; ++k) {
      double a = (k <= i) ? EL(A, lda, i, k) : EL(A, lda, k, i);
      s += a * x[k];
    }
    z[i] = beta * y[i] + alpha * s;
  }
}

/* Normwise backward error of an approximate solution x of A*x = b (A
 * symmetric, lower triangle read), in the Rigal-Gaches form
 *   eta = ||b - A*x||_inf / (||A||_inf * ||x||_inf + ||b||_inf).
 * Not from the paper: it is the acceptance test of the mixed-precision
 * solver. */
double orc_berr(int n, const double *A, int lda, const double *x,
                const double *b) {
  double rmax = 0.0, anorm = 0.0, xmax = 0.0, bmax = 0.0;
  for (int i = 0; i < n; ++i) {
    double s = 0.0, rowabs = 0.0;
    for (int k = 0; k < n; ++k) {
      double a = (k <= i) ? EL(A, lda, i, k) : EL(A, lda, k, i);
      s += a * x[k];
      rowabs += fabs(a);
    }
    double r = fabs(b[i] - s);
    /* maxima propagate NaN: a NaN anywhere gives eta = NaN */
    if (r > rmax || r != r) rmax = r;
    if (rowabs > anorm || rowabs != rowabs) anorm = rowabs;
    if (fabs(x[i]) > xmax || x[i] != x[i]) xmax = fabs(x[i]);
    if (fabs(b[i]) > bmax || b[i] != b[i]) bmax = fabs(b[i]);
  }
  double den = anorm * xmax + bmax;
  return den > 0.0 ? rmax / den : rmax;
}

/* Backward Riccati recursion in square-root form, §5.3.  With the dynamics
 * x+ = A x + B u (A nx-by-nx, B nx-by-nu), cost blocks Q (nx-by-nx), R
 * (nu-by-nu), S = 0, and terminal P_N, for n = N-1 down to 0:
 *   C   = [B^T; A^T] * Lc_{n+1}            (Lc_{n+1} lower, nx-by-nx)
 *   M   = [[R, 0], [0, Q]] + C*C^T         (lower triangle)
 *   F_n = chol(M) = [[Lambda_n, 0], [L_n, Lc_n]]
 * with Lc_N = chol(P_N).  The product with the lower triangular Lc sums only
 * over its nonzero entries.  F (N blocks of (nu+nx)^2, column-major, block n
 * at F + n*(nu+nx)^2) receives the lower triangles of the factors.  Returns
 * 0, or a nonzero code (1000*(stage+1) + pivot) if a factorization fails;
 * stage N denotes chol(P_N). */
int orc_ric_trf(int nx, int nu, int N, const double *A, int lda,
                const double *B, int ldb, const double *Q, int ldq,
                const double *R, int ldr, const double *PN, int ldp,
                double *F) {
  int nm = nu + nx;
  double *Lc = (double *)calloc((size_t)nx * nx, sizeof(double));
  double *C = (double *)calloc((size_t)nm * nx, sizeof(double));
  double *M = (double *)calloc((size_t)nm * nm, sizeof(double));
  if (!Lc || !C || !M) { free(Lc); free(C); free(M); return -1; }
  int info = orc_dpotrf_l(nx, PN, ldp, Lc, nx, NULL);
  if (info) { free(Lc); free(C); free(M); return 1000 * (N + 1) + info; }
  for (int n = N - 1; n >= 0; --n) {
    /* C = [B^T; A^T] * Lc: row r < nu is column r of B, row nu+r is column
     * r of A. */
    for (int j = 0; j < nx; ++j)
      for (int r = 0; r < nm; ++r) {
        double s = 0.0;
        for (int k = j; k < nx; ++k) {
          double x = (r < nu) ? EL(B, ldb, k, r) : EL(A, lda, k, r - nu);
          s += x * EL(Lc, nx, k, j);
        }
        EL(C, nm, r, j) = s;
      }
    /* M = blockdiag(R, Q) + C*C^T, lower triangle */
    for (int j = 0; j < nm; ++j)
      for (int i = j; i < nm; ++i) {
        double base = 0.0;
        if (i < nu && j < nu) base = EL(R, ldr, i, j);
        else if (i >= nu && j >= nu) base = EL(Q, ldq, i - nu, j - nu);
        double s = 0.0;
        for (int k = 0; k < nx; ++k) s += EL(C, nm, i, k) * EL(C, nm, j, k);
        EL(M, nm, i, j) = base + s;
      }
    double *Fn = F + (size_t)n * nm * nm;
    info = orc_dpotrf_l(nm, M, nm, Fn, nm, NULL);
    if (info) { free(Lc); free(C); free(M); return 1000 * (n + 1) + info; }
    for (int j = 0; j < nx; ++j)
      for (int i = j; i < nx; ++i) EL(Lc, nx, i, j) = EL(Fn, nm, nu + i, nu + j);
  }
  free(Lc); free(C); free(M);
  return 0;
}

/* Riccati solve: the solution of the linear-quadratic control problem whose
 * KKT matrix orc_ric_trf factors (§5.3 states the recursion as the
 * factorization of that KKT matrix; the substitution below is the standard
 * one of the square-root form, not printed in the paper):
 *   minimize  sum_n 1/2 u_n'R u_n + r_n'u_n + 1/2 x_n'Q x_n + q_n'x_n
 *             + 1/2 x_N'P_N x_N + q_N'x_N
 *   subject to x_{n+1} = A x_n + B u_n + b_n,  x_0 given,  n = 0..N-1.
 * With F_n = [[Lam_n, 0], [L_n, Lc_n]] the stage factors (F_n F_n' = M_n,
 * M_n = [[R + B'P B, B'P A], [A'P B, Q + A'P A]], P = P_{n+1} = Lc_{n+1} Lc_{n+1}'
 * and P_N given), the value function's linear term p_n follows backwards,
 *   w = P_{n+1} b_n + p_{n+1},  m_u = r_n + B'w,  m_x = q_n + A'w,
 *   l_n = Lam_n^{-1} m_u,       p_n = m_x - L_n l_n,       p_N = q_N,
 * and the controls and states forwards,
 *   u_n = -Lam_n^{-T} (L_n' x_n + l_n),  x_{n+1} = A x_n + B u_n + b_n.
 * F is as written by orc_ric_trf (N column-major (nu+nx)^2 blocks); only
 * the lower triangle of PN is read.  b: N x nx, r: N x nu, q: (N+1) x nx,
 * u: N x nu, x: (N+1) x nx, all row n contiguous. */
void orc_ric_trs(int nx, int nu, int N, const double *A, int lda,
                 const double *B, int ldb, const double *PN, int ldp,
                 const double *F, const double *b, const double *r,
                 const double *q, const double *x0, double *u, double *x) {
  int nm = nu + nx;
  double *p = (double *)calloc((size_t)nx, sizeof(double));
  double *w = (double *)calloc((size_t)nx, sizeof(double));
  double *s = (double *)calloc((size_t)nx, sizeof(double));
  double *m = (double *)calloc((size_t)nm, sizeof(double));
  double *l = (double *)calloc((size_t)N * nu + 1, sizeof(double));
  for (int i = 0; i < nx; ++i) p[i] = q[(size_t)N * nx + i];
  for (int n = N - 1; n >= 0; --n) {
    const double *bn = b + (size_t)n * nx;
    /* w = P_{n+1} b_n + p_{n+1} */
    if (n == N - 1) {
      for (int i = 0; i < nx; ++i) {
        double t = 0.0;
        for (int k = 0; k < nx; ++k)
          t += (k <= i ? EL(PN, ldp, i, k) : EL(PN, ldp, k, i)) * bn[k];
        w[i] = t + p[i];
      }
    } else {
      const double *Fn1 = F + (size_t)(n + 1) * nm * nm;  /* Lc_{n+1} = its trailing block */
      for (int j = 0; j < nx; ++j) {                      /* s = Lc' b */
        double t = 0.0;
        for (int i = j; i < nx; ++i) t += EL(Fn1, nm, nu + i, nu + j) * bn[i];
        s[j] = t;
      }
      for (int i = 0; i < nx; ++i) {                      /* w = Lc s + p */
        double t = 0.0;
        for (int k = 0; k <= i; ++k) t += EL(Fn1, nm, nu + i, nu + k) * s[k];
        w[i] = t + p[i];
      }
    }
    /* m = [r_n + B'w; q_n + A'w] */
    for (int j = 0; j < nu; ++j) {
      double t = 0.0;
      for (int i = 0; i < nx; ++i) t += EL(B, ldb, i, j) * w[i];
      m[j] = r[(size_t)n * nu + j] + t;
    }
    for (int j = 0; j < nx; ++j) {
      double t = 0.0;
      for (int i = 0; i < nx; ++i) t += EL(A, lda, i, j) * w[i];
      m[nu + j] = q[(size_t)n * nx + j] + t;
    }
    /* l_n = Lam_n^{-1} m_u (forward substitution), p_n = m_x - L_n l_n */
    const double *Fn = F + (size_t)n * nm * nm;
    double *ln = l + (size_t)n * nu;
    for (int i = 0; i < nu; ++i) {
      double t = m[i];
      for (int k = 0; k < i; ++k) t -= EL(Fn, nm, i, k) * ln[k];
      ln[i] = t / EL(Fn, nm, i, i);
    }
    for (int i = 0; i < nx; ++i) {
      double t = 0.0;
      for (int k = 0; k < nu; ++k) t += EL(Fn, nm, nu + i, k) * ln[k];
      p[i] = m[nu + i] - t;
    }
  }
  for (int i = 0; i < nx; ++i) x[i] = x0[i];
  for (int n = 0; n < N; ++n) {
    const double *Fn = F + (size_t)n * nm * nm;
    const double *xn = x + (size_t)n * nx;
    double *un = u + (size_t)n * nu;
    /* v = L_n' x_n + l_n, then u_n = -Lam_n^{-T} v (back substitution) */
    for (int j = 0; j < nu; ++j) {
      double t = 0.0;
      for (int i = 0; i < nx; ++i) t += EL(Fn, nm, nu + i, j) * xn[i];
      m[j] = t + l[(size_t)n * nu + j];
    }
    for (int i = nu - 1; i >= 0; --i) {
      double t = m[i];
      for (int k = i + 1; k < nu; ++k) t -= EL(Fn, nm, k, i) * un[k];
      un[i] = t / EL(Fn, nm, i, i);
    }
    for (int i = 0; i < nu; ++i) un[i] = -un[i];
    /* x_{n+1} = A x_n + B u_n + b_n */
    double *xn1 = x + (size_t)(n + 1) * nx;
    for (int i = 0; i < nx; ++i) {
      double t = 0.0;
      for (int k = 0; k < nx; ++k) t += EL(A, lda, i, k) * xn[k];
      for (int k = 0; k < nu; ++k) t += EL(B, ldb, i, k) * un[k];
      xn1[i] = t + b[(size_t)n * nx + i];
    }
  }
  free(p); free(w); free(s); free(m); free(l);
}

/* ---- single-precision pieces of the mixed-precision solve ----------------
 * Not from the paper: the FP32 factor-and-solve that iterative refinement
 * starts from.  Same definitions as orc_dpotrf_l / orc_dpotrs_l, with every
 * operation in IEEE single precision. */
int orc_spotrf_l(int m, const float *C, int ldc, float *D, int ldd) {
  for (int j = 0; j < m; ++j) {
    float d = EL(C, ldc, j, j);
    for (int k = 0; k < j; ++k) d -= EL(D, ldd, j, k) * EL(D, ldd, j, k);
    if (!(d > 0.0f)) return j + 1;
    float ljj = sqrtf(d);
    float inv = 1.0f / ljj;
    EL(D, ldd, j, j) = ljj;
    for (int i = j + 1; i < m; ++i) {
      float s = EL(C, ldc, i, j);
      for (int k = 0; k < j; ++k) s -= EL(D, ldd, i, k) * EL(D, ldd, j, k);
      EL(D, ldd, i, j) = s * inv;
    }
  }
  return 0;
}

/* sgemm_nt and ssyrk_ln in IEEE single precision (Appendix A.3: the routines
 * come in single- and double-precision variants): the definitions of
 * orc_dgemm_nt / orc_dsyrk_ln with every operation in float. */
void orc_sgemm_nt(int m, int n, int k, float alpha, const float *A, int lda,
                  const float *B, int ldb, float beta, const float *C,
                  int ldc, float *D, int ldd) {
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < m; ++i) {
      float s = 0.0f;
      for (int l = 0; l < k; ++l) s += EL(A, lda, i, l) * EL(B, ldb, j, l);
      EL(D, ldd, i, j) = beta * EL(C, ldc, i, j) + alpha * s;
    }
}

void orc_ssyrk_ln(int m, int k, float alpha, const float *A, int lda,
                  const float *B, int ldb, float beta, const float *C,
                  int ldc, float *D, int ldd) {
  for (int j = 0; j < m; ++j)
    for (int i = j; i < m; ++i) {
      float s = 0.0f;
      for (int l = 0; l < k; ++l) s += EL(A, lda, i, l) * EL(B, ldb, j, l);
      EL(D, ldd, i, j) = beta * EL(C, ldc, i, j) + alpha * s;
    }
}

void orc_spotrs_l(int n, const float *L, int ldl, const float *b, float *x) {
  for (int i = 0; i < n; ++i) {
    float s = b[i];
    for (int k = 0; k < i; ++k) s -= EL(L, ldl, i, k) * x[k];
    x[i] = s * (1.0f / EL(L, ldl, i, i));
  }
  for (int i = n - 1; i >= 0; --i) {
    float s = x[i];
    for (int k = i + 1; k < n; ++k) s -= EL(L, ldl, k, i) * x[k];
    x[i] = s * (1.0f / EL(L, ldl, i, i));
  }
}

/* IEEE binary16 value nearest to the binary32 value x (ties to even), as a
 * float.  Written from the format's definition: 11 significant bits, least
 * exponent -14 (subnormal quantum 2^-24), largest finite 65504. */
float orc_fl16(float x) {
  if (x != x) return x;
  const float ax = fabsf(x);
  if (ax >= 65520.0f) return copysignf(INFINITY, x); /* at/above the midpoint to 2^16 */
  if (ax < 6.103515625e-05f) {                      /* below 2^-14: fixed quantum */
    return copysignf(rintf(ax * 16777216.0f) / 16777216.0f, x);
  }
  int e;
  frexpf(ax, &e);                        /* ax = m 2^e, m in [0.5, 1) */
  const float q = ldexpf(1.0f, e - 11);  /* spacing of 11-bit significands */
  return copysignf(rintf(ax / q) * q, x);
}

/* Power-of-two diagonal scaling of the mixed-precision solve (not from the
 * paper): s_i = 2^-floor(e_i / 2) where a_ii = m 2^e_i, m in [0.5, 1), so
 * that s_i^2 a_ii lies in [0.5, 2) and S A S (S = diag(s)) is formed without
 * rounding.  s_i = 1 where a_ii is not a positive finite number. */
void orc_mixed_scale(int n, const double *A, int lda, double *s) {
  for (int i = 0; i < n; ++i) {
    const double d = EL(A, lda, i, i);
    s[i] = 1.0;
    if (d > 0.0 && isfinite(d)) {
      int e;
      frexp(d, &e);
      s[i] = ldexp(1.0, -(int)floor(e / 2.0));
    }
  }
}

/* Low-precision Cholesky factor of the scaled matrix fl32(S A S), lower
 * triangle of A read.  prec 1: every operation in binary32.  prec 2: the
 * same, except that both factors of every product in the downdate sums are
 * first rounded to binary16 (the products themselves are exact in binary32).
 * Returns 0 or the 1-based index of the first pivot that is not > 0. */
int orc_mixed_factor(int n, const double *A, int lda, int prec, float *L,
                     int ldl, double *s) {
  orc_mixed_scale(n, A, lda, s);
  for (int j = 0; j < n; ++j) {
    float d = (float)(EL(A, lda, j, j) * s[j] * s[j]);
    for (int k = 0; k < j; ++k) {
      const float u = prec == 2 ? orc_fl16(EL(L, ldl, j, k)) : EL(L, ldl, j, k);
      d -= u * u;
    }
    if (!(d > 0.0f)) return j + 1;
    const float ljj = sqrtf(d);
    const float inv = 1.0f / ljj;
    EL(L, ldl, j, j) = ljj;
    for (int i = j + 1; i < n; ++i) {
      float t = (float)(EL(A, lda, i, j) * s[i] * s[j]);
      for (int k = 0; k < j; ++k) {
        const float a = prec == 2 ? orc_fl16(EL(L, ldl, i, k)) : EL(L, ldl, i, k);
        const float b = prec == 2 ? orc_fl16(EL(L, ldl, j, k)) : EL(L, ldl, j, k);
        t -= a * b;
      }
      EL(L, ldl, i, j) = t * inv;
    }
    for (int i = 0; i < j; ++i) EL(L, ldl, i, j) = 0.0f;
  }
  return 0;
}

/* Iterative refinement in FP64 for one right-hand side (not from the
 * paper), given the low-precision factor L of S A S (orc_mixed_factor): a
 * correction solves A d = r as d = S solve32(fl32(S r)).  x0 is the
 * correction for r = b; then repeat: r = b - A x (FP64, lower triangle of A),
 * eta = backward error of x; stop if eta <= tol; give up if max_iter
 * corrections were applied or if eta did not decrease since the previous
 * test (stagnation); else x = x + d.  Returns the number of corrections
 * applied after x0 (>= 0) or -2 if refinement gives up; eta_out receives the
 * last backward error. */
int orc_mixed_refine(int n, const double *A, int lda, const float *L32,
                     int ldl, const double *s, const double *b, double tol,
                     int max_iter, double *x, double *eta_out) {
  float *v32 = (float *)calloc((size_t)n + 1, sizeof(float));
  float *d32 = (float *)calloc((size_t)n + 1, sizeof(float));
  double *r = (double *)calloc((size_t)n + 1, sizeof(double));
  int ret = -3;
  if (v32 && d32 && r) {
    for (int i = 0; i < n; ++i) v32[i] = (float)(s[i] * b[i]);
    orc_spotrs_l(n, L32, ldl, v32, d32);
    for (int i = 0; i < n; ++i) x[i] = s[i] * (double)d32[i];
    double prev = INFINITY;
    for (int it = 0;; ++it) {
      const double eta = orc_berr(n, A, lda, x, b);
      if (eta_out) *eta_out = eta;
      if (eta <= tol) { ret = it; break; }
      if (it >= max_iter || !(eta < prev)) { ret = -2; break; }
      prev = eta;
      orc_dsymv_l(n, -1.0, A, lda, x, 1.0, b, r);
      for (int i = 0; i < n; ++i) v32[i] = (float)(s[i] * r[i]);
      orc_spotrs_l(n, L32, ldl, v32, d32);
      for (int i = 0; i < n; ++i) x[i] += s[i] * (double)d32[i];
    }
  }
  free(v32); free(d32); free(r);
  return ret;
}

/* Mixed-precision solve of A x = b (one right-hand side): orc_mixed_factor
 * then orc_mixed_refine.  Returns the number of corrections after x0, -1 if
 * the low-precision factorization fails, -2 if refinement gives up. */
int orc_dposv_mixed(int n, const double *A, int lda, const double *b,
                    double tol, int max_iter, int prec, double *x,
                    double *eta_out) {
  float *L32 = (float *)malloc(sizeof(float) * ((size_t)n * n + 1));
  double *s = (double *)malloc(sizeof(double) * ((size_t)n + 1));
  int ret = -3;
  if (L32 && s) {
    if (orc_mixed_factor(n, A, lda, prec, L32, n, s))
      ret = -1;
    else
      ret = orc_mixed_refine(n, A, lda, L32, n, s, b, tol, max_iter, x, eta_out);
  }
  free(L32); free(s);
  return ret;
}
