/*
 * Batched drivers of the CPU oracle: an OpenMP loop over independent
 * instances, each handled by the plain per-instance routines of oracle.c.
 *
 * TEST INFRASTRUCTURE ONLY (tests, smoke check and the CPU-baseline leg of
 * the benchmark).  Instances are column-major and stored one after another.
 */
#include <stddef.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

void orc_dsyrk_ln(int m, int k, double alpha, const double *A, int lda,
                  const double *B, int ldb, double beta, const double *C,
                  int ldc, double *D, int ldd);
int orc_dpotrf_l(int m, const double *C, int ldc, double *D, int ldd,
                 double *dA);
void orc_dtrsm_rltn(int m, int n, double alpha, const double *L, int ldl,
                    const double *B, int ldb, double *D, int ldd);
void orc_dpotrs_l(int n, int nrhs, const double *L, int ldl, const double *B,
                  int ldb, double *X, int ldx);
int orc_ric_trf(int nx, int nu, int N, const double *A, int lda,
                const double *B, int ldb, const double *Q, int ldq,
                const double *R, int ldr, const double *PN, int ldp,
                double *F);
int orc_mixed_factor(int n, const double *A, int lda, int prec, float *L,
                     int ldl, double *s);
int orc_mixed_refine(int n, const double *A, int lda, const float *L32,
                     int ldl, const double *s, const double *b, double tol,
                     int max_iter, double *x, double *eta_out);

static int set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
  int used = 1;
#pragma omp parallel
  {
#pragma omp single
    used = omp_get_num_threads();
  }
  return used;
#else
  (void)nthreads;
  return 1;
#endif
}

/* Uniform batch of the range-space pair of §4.7.2: per instance
 *   L = chol(Q + B*B^T)   (syrk_ln then potrf_l),
 *   X = RHS * L^{-T}      (trsm_rltn),
 * with Q n-by-n (lower read), B n-by-k, RHS nrhs-by-n.  Returns the number
 * of threads used. */
int orc_batch_syrk_potrf_trsm(int batch, int n, int k, int nrhs,
                              const double *Q, const double *B,
                              const double *RHS, double *L, double *X,
                              double *dA, int *info, int nthreads) {
  int used = set_threads(nthreads);
  size_t sq = (size_t)n * n, sb = (size_t)n * k, sr = (size_t)nrhs * n;
#pragma omp parallel
  {
    double *M = (double *)malloc(sizeof(double) * (sq > 0 ? sq : 1));
#pragma omp for schedule(dynamic, 16)
    for (int b = 0; b < batch; ++b) {
      orc_dsyrk_ln(n, k, 1.0, B + b * sb, n, B + b * sb, n, 1.0, Q + b * sq,
                   n, M, n);
      int inf = orc_dpotrf_l(n, M, n, L + b * sq, n, dA + (size_t)b * n);
      info[b] = inf;
      if (inf == 0)
        orc_dtrsm_rltn(nrhs, n, 1.0, L + b * sq, n, RHS + b * sr, nrhs,
                       X + b * sr, nrhs);
    }
    free(M);
  }
  return used;
}

/* Uneven batch of Cholesky solves: instance b has order n[b]; its matrix
 * starts at A + offA[b] (column-major, lda = n[b]), its right-hand side at
 * rhs + offv[b]; L, dA and x use the same offsets.  Returns the number of
 * threads used. */
int orc_batch_potrf_potrs(int batch, const int *n, const long long *offA,
                          const long long *offv, const double *A,
                          const double *rhs, double *L, double *dA,
                          double *x, int *info, int nthreads) {
  int used = set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
  for (int b = 0; b < batch; ++b) {
    int nb = n[b];
    int inf = orc_dpotrf_l(nb, A + offA[b], nb, L + offA[b], nb, dA + offv[b]);
    info[b] = inf;
    if (inf == 0) orc_dpotrs_l(nb, 1, L + offA[b], nb, rhs + offv[b], nb,
                               x + offv[b], nb);
  }
  return used;
}

/* Batch of backward Riccati recursions (§5.3), one problem per instance,
 * all of the same sizes.  F receives N factors of order nu+nx per problem.
 * Returns the number of threads used. */
int orc_batch_ric_trf(int batch, int nx, int nu, int N, const double *A,
                      const double *B, const double *Q, const double *R,
                      const double *PN, double *F, int *info, int nthreads) {
  int used = set_threads(nthreads);
  size_t sa = (size_t)nx * nx, sbb = (size_t)nx * nu, sr = (size_t)nu * nu;
  size_t sf = (size_t)N * (nu + nx) * (nu + nx);
#pragma omp parallel for schedule(dynamic, 4)
  for (int b = 0; b < batch; ++b)
    info[b] = orc_ric_trf(nx, nu, N, A + b * sa, nx, B + b * sbb, nx,
                          Q + b * sa, nx, R + b * sr, nu, PN + b * sa, nx,
                          F + b * sf);
  return used;
}

/* Batch of mixed-precision solves A_b X_b = B_b (orc_mixed_factor once per
 * instance, orc_mixed_refine per right-hand side).  Instance b: A at
 * A + offA[b] (n_b x n_b, ld n_b), B and X at + offv[b] (n_b x nrhs, ld n_b).
 * iters[b] = the largest number of corrections over the right-hand sides, or
 * -1 (factorization failed) or -2 (some right-hand side gave up); eta[b] =
 * the largest final backward error.  Returns the number of threads used. */
int orc_batch_dposv_mixed(int batch, const int *n, const long long *offA,
                          const long long *offv, const double *A,
                          const double *B, int nrhs, double tol, int max_iter,
                          int prec, double *X, int *iters, double *eta,
                          int nthreads) {
  int used = set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
  for (int b = 0; b < batch; ++b) {
    const int nb = n[b];
    float *L = (float *)malloc(sizeof(float) * ((size_t)nb * nb + 1));
    double *s = (double *)malloc(sizeof(double) * ((size_t)nb + 1));
    iters[b] = -3;
    eta[b] = 0.0;
    if (L && s) {
      if (orc_mixed_factor(nb, A + offA[b], nb, prec, L, nb, s)) {
        iters[b] = -1;
      } else {
        int it = 0;
        for (int c = 0; c < nrhs; ++c) {
          double e = 0.0;
          const int r = orc_mixed_refine(nb, A + offA[b], nb, L, nb, s,
                                         B + offv[b] + (size_t)c * nb, tol,
                                         max_iter, X + offv[b] + (size_t)c * nb, &e);
          if (e > eta[b] || e != e) eta[b] = e;
          if (r < 0 || it < 0) it = it < 0 ? it : r; else if (r > it) it = r;
        }
        iters[b] = it;
      }
    }
    free(L);
    free(s);
  }
  return used;
}

double orc_berr(int n, const double *A, int lda, const double *x,
                const double *b);

/* Uniform-order chunk of Cholesky solves: `batch` instances of order n with
 * nrhs right-hand sides; instance b's matrix at A + b*n*n (column-major,
 * lower triangle read), its right-hand sides at B + b*n*nrhs (n x nrhs,
 * column-major); L, dA and X at the matching offsets (dA: b*n).  Instances
 * whose factorization fails leave X untouched.  Returns the number of
 * threads used. */
int orc_batch_dposv_uniform(int batch, int n, int nrhs, const double *A,
                            const double *B, double *L, double *dA, double *X,
                            int *info, int nthreads) {
  int used = set_threads(nthreads);
  const size_t sa = (size_t)n * n, sb = (size_t)n * nrhs;
#pragma omp parallel for schedule(dynamic, 2)
  for (int b = 0; b < batch; ++b) {
    const int inf = orc_dpotrf_l(n, A + b * sa, n, L + b * sa, n, dA + (size_t)b * n);
    info[b] = inf;
    if (inf == 0 && nrhs > 0)
      orc_dpotrs_l(n, nrhs, L + b * sa, n, B + b * sb, n, X + b * sb, n);
  }
  return used;
}

/* Normwise backward errors (orc_berr) of `batch` uniform-order instances:
 * eta[b] = the largest over the nrhs columns of X_b for A_b x = b_c (NaN
 * propagates).  Layouts as in orc_batch_dposv_uniform.  Returns the number
 * of threads used. */
int orc_batch_berr_uniform(int batch, int n, int nrhs, const double *A,
                           const double *X, const double *B, double *eta,
                           int nthreads) {
  int used = set_threads(nthreads);
  const size_t sa = (size_t)n * n, sb = (size_t)n * nrhs;
#pragma omp parallel for schedule(dynamic, 4)
  for (int b = 0; b < batch; ++b) {
    double worst = 0.0;
    for (int c = 0; c < nrhs; ++c) {
      const double e = orc_berr(n, A + b * sa, n, X + b * sb + (size_t)c * n,
                                B + b * sb + (size_t)c * n);
      if (e > worst || e != e) worst = e;
    }
    eta[b] = worst;
  }
  return used;
}
