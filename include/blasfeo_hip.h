/*
 * blasfeo_hip.h -- C ABI of an MI355X (gfx950) library of dense linear
 * algebra routines for small and medium matrices stored in the panel-major
 * format of "BLASFEO: basic linear algebra subroutines for embedded
 * optimization" (Frison et al., arXiv 1704.02457).
 *
 * Conventions (all entry points):
 *  - Matrices are described by a host-side struct blasfeo_dmat whose pointers
 *    pA and dA are DEVICE pointers, and are addressed by the paper's operand
 *    triple (sA, ai, aj): the working sub-matrix has its top-left element at
 *    row ai, column aj (§3 and Appendix A.2).  Char options are part of the
 *    routine name (Appendix A.2).
 *  - Panel-major storage (§4.3): rows are grouped in panels of BLASFEO_HIP_PS
 *    = 16 rows; inside a panel the storage is column-major with leading
 *    dimension 16; panels are 16*cn doubles apart, so element (i, j) is at
 *        pA[(i - i % 16) * cn + j * 16 + i % 16].
 *    A panel column (16 doubles) is one 128-byte line.  ps is a compile-time
 *    constant, as the paper requires for the shift/mask address arithmetic.
 *  - The caller owns every byte of memory.  No compute routine allocates
 *    (Appendix A.1.2); the only allocating calls are blasfeo_allocate_dmat /
 *    blasfeo_allocate_dvec / blasfeo_allocate_smat (hipMalloc) and plan
 *    creation (host memory and a small device table).  Scratch memory of
 *    the plan executions is a workspace argument, sized by a query.
 *  - All compute routines are asynchronous on the stream set with
 *    blasfeo_hip_set_stream (default: the null stream) or on the stream
 *    argument of the batched entry points (a hipStream_t passed as void*).
 *  - Routines are non-destructive: the output operand is a separate argument,
 *    which may coincide with an input where stated (Appendix A.2).
 *  - Single-instance routines return void, like the paper's API.  Argument
 *    errors are detected on the host before any launch; the routine then
 *    launches nothing and records the error, readable (and cleared) with
 *    blasfeo_hip_get_last_error().  Batched entry points return that code
 *    directly: 0 = success, -i = argument i invalid, > 0 = HIP error code.
 *  - Numerical failure of a Cholesky factorization is reported per instance
 *    in a device int array info: 0, or j+1 for the first column j (0-based,
 *    relative to the sub-matrix) whose pivot is not positive (LAPACK's
 *    convention).  Entries of that column and later ones are unspecified;
 *    the other instances of a batch are unaffected.
 *  - Thread safety: the stream setting and the last error are per host
 *    thread.  Calls that overlap on one device in different streams are
 *    independent unless their operands overlap.
 */
#ifndef BLASFEO_HIP_H
#define BLASFEO_HIP_H

#ifdef __cplusplus
extern "C" {
#endif

#define BLASFEO_HIP_PS 16  /* panel height for double precision */

/* Matrix handle (Appendix A.1.1).  pA, m, n and memsize are the paper's
 * common members; cn (the panel length "sda" of §4.3) and dA (the inverse
 * diagonal of §4.7.1) are the high-performance implementation's members;
 * pm (number of panels) and use_dA (dA holds the inverse diagonal of the
 * whole matrix, set by a factorization at (0,0)) are this library's.
 *   pA:  device pointer, pm*16*cn doubles, panel-major.
 *   dA:  device pointer, max(m,n) doubles (inverse diagonal).
 *   memsize: bytes of the chunk addressed by the struct, a multiple of 256,
 *        so consecutive chunks of memsize bytes stay aligned. */
struct blasfeo_dmat {
  double *pA;
  double *dA;
  int m;
  int n;
  int pm;
  int cn;
  int use_dA;
  int memsize;
};

/* Vector handle (Appendix A.1.1): unit stride, device pointer pa. */
struct blasfeo_dvec {
  double *pa;
  int m;
  int pm;
  int memsize;
};

/* ------------------------------------------------------------------------
 * Memory (Appendix A.1.2)
 * ---------------------------------------------------------------------- */

/* Bytes needed by an m-by-n matrix: pm*16*cn*8 for the panels (cn = n
 * rounded up to a multiple of 4, pm = ceil(m/16)) plus max(m,n)*8 for dA,
 * rounded up to 256.  Returns -1 if m < 0, n < 0 or the size overflows. */
int blasfeo_memsize_dmat(int m, int n);
/* Bytes needed by a vector of m doubles, rounded up to 256. */
int blasfeo_memsize_dvec(int m);

/* Sets the members of *sA so that it describes an m-by-n matrix living in
 * the device memory chunk `memory` (at least blasfeo_memsize_dmat(m,n)
 * bytes, 256-byte aligned).  The memory is not touched (Appendix A.1.2).
 * pA = memory, dA = memory + pm*16*cn doubles. */
void blasfeo_create_dmat(int m, int n, struct blasfeo_dmat *sA, void *memory);
void blasfeo_create_dvec(int m, struct blasfeo_dvec *sx, void *memory);

/* hipMalloc-backed creation and release (Appendix A.1.2). */
void blasfeo_allocate_dmat(int m, int n, struct blasfeo_dmat *sA);
void blasfeo_free_dmat(struct blasfeo_dmat *sA);
void blasfeo_allocate_dvec(int m, struct blasfeo_dvec *sx);
void blasfeo_free_dvec(struct blasfeo_dvec *sx);

/* Conversion between column-major device arrays and panel-major storage
 * (the packing routines of Appendix A.3), on the current stream.
 *   pack:   sB[bi:bi+m, bj:bj+n] = A (m-by-n, column-major, leading dim lda)
 *   unpack: B (m-by-n, leading dim ldb) = sA[ai:ai+m, aj:aj+n]
 * A and B are device pointers.  Elements outside the sub-matrix, including
 * panel padding, are not written.  A struct whose sub-matrix or sub-vector
 * does not fit (offset < 0 or past its size) is reported as an error at the
 * struct's argument position. */
void blasfeo_pack_dmat(int m, int n, const double *A, int lda,
                       struct blasfeo_dmat *sB, int bi, int bj);
void blasfeo_unpack_dmat(int m, int n, struct blasfeo_dmat *sA, int ai,
                         int aj, double *B, int ldb);
void blasfeo_pack_dvec(int m, const double *x, struct blasfeo_dvec *sy,
                       int yi);
void blasfeo_unpack_dvec(int m, struct blasfeo_dvec *sx, int xi, double *y);

/* ------------------------------------------------------------------------
 * Single-instance routines (Appendix A.2, A.3).  Sizes first, then
 * operands.  Every operand must lie inside its matrix: ai + rows <= m and
 * aj + cols <= n of the struct.
 * ---------------------------------------------------------------------- */

/* gemm_nt (Appendix A.2): D <- alpha*A*B^T + beta*C, A m-by-k at (ai,aj),
 * B n-by-k at (bi,bj), C and D m-by-n.  C and D may be the same matrix at
 * the same offsets; any other overlap of D with an input is undefined. */
void blasfeo_dgemm_nt(int m, int n, int k, double alpha,
                      struct blasfeo_dmat *sA, int ai, int aj,
                      struct blasfeo_dmat *sB, int bi, int bj, double beta,
                      struct blasfeo_dmat *sC, int ci, int cj,
                      struct blasfeo_dmat *sD, int di, int dj);

/* gemm_nn (§4.4, the NN variant: B read across panels): D <- alpha*A*B +
 * beta*C, A m-by-k at (ai,aj), B k-by-n at (bi,bj), C and D m-by-n.  C and
 * D may be the same matrix at the same offsets; any other overlap of D with
 * an input is undefined. */
void blasfeo_dgemm_nn(int m, int n, int k, double alpha,
                      struct blasfeo_dmat *sA, int ai, int aj,
                      struct blasfeo_dmat *sB, int bi, int bj, double beta,
                      struct blasfeo_dmat *sC, int ci, int cj,
                      struct blasfeo_dmat *sD, int di, int dj);

/* syrk_ln (§5.2.2): lower triangle of D <- alpha*A*B^T + beta*C, A and B
 * m-by-k (they may differ), C and D m-by-m.  Only elements on or below the
 * diagonal of the D sub-matrix are written and only those of C are read. */
void blasfeo_dsyrk_ln(int m, int k, double alpha, struct blasfeo_dmat *sA,
                      int ai, int aj, struct blasfeo_dmat *sB, int bi,
                      int bj, double beta, struct blasfeo_dmat *sC, int ci,
                      int cj, struct blasfeo_dmat *sD, int di, int dj);

/* trmm_rlnn (§5.2.2, trmm paragraph; the C step of the Riccati recursion,
 * §5.3): D <- alpha * B * A, A n-by-n lower triangular, not unit, at
 * (ai,aj) (only its lower triangle is read); B and D m-by-n.  D must not
 * share storage with B or A (error -10). */
void blasfeo_dtrmm_rlnn(int m, int n, double alpha, struct blasfeo_dmat *sA,
                        int ai, int aj, struct blasfeo_dmat *sB, int bi,
                        int bj, struct blasfeo_dmat *sD, int di, int dj);

/* trsm_rltn (§5.2.2, §4.7.2): D <- alpha * B * A^{-T}, A n-by-n lower
 * triangular, not unit, at (ai,aj) (only its lower triangle is read; the
 * reciprocals of its diagonal are formed by the routine); B and D m-by-n.
 * B and D may be the same matrix at the same offsets. */
void blasfeo_dtrsm_rltn(int m, int n, double alpha, struct blasfeo_dmat *sA,
                        int ai, int aj, struct blasfeo_dmat *sB, int bi,
                        int bj, struct blasfeo_dmat *sD, int di, int dj);

/* potrf_l (§5.2.2, §4.6, §4.7.1): lower Cholesky factor D of the m-by-m
 * matrix whose lower triangle is C.  Writes the lower triangle of D and
 * sD->dA[0..m-1] = 1/diag(D); sets sD->use_dA = (di == 0 && dj == 0).
 * C and D may be the same matrix at the same offsets. */
void blasfeo_dpotrf_l(int m, struct blasfeo_dmat *sC, int ci, int cj,
                      struct blasfeo_dmat *sD, int di, int dj);

/* potrf_l_mn (§4.7.2, stacking matrices): for the stacked m-by-n matrix
 * C = [H; A] (m >= n, H n-by-n SPD, lower triangle read; A (m-n)-by-n, all
 * read) writes D = [L; A L^{-T}] with L L^T = H (the lower triangle of the
 * top block and all of the bottom block) and sD->dA[0..n-1] = 1/diag(L):
 * potrf_l and trsm_rltn in one sweep.  Errors: -1 m < 0, -2 n < 0 or
 * n > m, -3 C, -6 D (or a NULL dA).  C and D may be the same matrix at the
 * same offsets. */
void blasfeo_dpotrf_l_mn(int m, int n, struct blasfeo_dmat *sC, int ci,
                         int cj, struct blasfeo_dmat *sD, int di, int dj);

/* getrf (§5.2.2; the API's getrf_pivot / getrf_nopivot): LU of the m-by-n
 * matrix C (m, n <= 256) into D: unit lower L below the diagonal, U on and
 * above it, sD->dA[k] = 1/U[k][k].  With pivoting, row k is swapped with
 * row ipiv[k] >= k (0-based, the first row of largest magnitude in column
 * k) before step k; ipiv is a device array of min(m,n) ints.  A zero pivot
 * does not stop the factorization (as in LAPACK; the batched entry point
 * reports it in info).  m, n <= 32: unblocked, the oracle's operations in
 * its order (identical bits); larger: blocked by panels of 16 columns with
 * the trailing update on the matrix cores (§5.2.2's blocked form; one wave
 * per instance with the matrix in registers up to 64, a workgroup per
 * instance above), the factors agreeing to rounding and the interchanges
 * wherever the pivot candidates differ by more than the rounding (the
 * reciprocal of a pivot is the hardware estimate refined by Newton steps,
 * within an ulp).  Errors: -1 m, -2 n (outside 0..256), -3 C,
 * -6 D (or a NULL dA), -9 a NULL ipiv.  C and D may be the same matrix at
 * the same offsets. */
void blasfeo_dgetrf_pivot(int m, int n, struct blasfeo_dmat *sC, int ci,
                          int cj, struct blasfeo_dmat *sD, int di, int dj,
                          int *ipiv);
void blasfeo_dgetrf_nopivot(int m, int n, struct blasfeo_dmat *sC, int ci,
                            int cj, struct blasfeo_dmat *sD, int di, int dj);

/* gelqf (§5.2.2): LQ factorization C = L Q of the m-by-n matrix C
 * (m, n <= 256) by Householder reflectors, in LAPACK's compact form: L on
 * and below the diagonal of D, reflector k's vector to the right of the
 * diagonal of row k (its k-th entry 1 implicit), tau_k in sD->dA[k]
 * (min(m,n) entries); Q = H_{min-1} ... H_0 with H_k = I - tau_k v v'.
 * m, n <= 32: unblocked, the oracle's operations in its order (identical
 * bits); larger: blocked by panels of 16 rows, the rows below a panel
 * updated as A2 -= ((A2 V^T) T) V on the matrix cores (one wave per
 * instance with the matrix in registers up to 64, a workgroup per instance
 * above; the factors agree to rounding).  Errors: -1 m, -2 n (outside 0..256), -3 C, -6 D (or a NULL
 * dA).  C and D may be the same matrix at the same offsets. */
void blasfeo_dgelqf(int m, int n, struct blasfeo_dmat *sC, int ci, int cj,
                    struct blasfeo_dmat *sD, int di, int dj);

/* syrk_potrf_ln (Appendix A.3, §4.7.2): D = chol(C + A*B^T), lower, with
 * A, B m-by-k, and sD->dA as in potrf_l; the product is never stored. */
void blasfeo_dsyrk_dpotrf_ln(int m, int k, struct blasfeo_dmat *sA, int ai,
                             int aj, struct blasfeo_dmat *sB, int bi,
                             int bj, struct blasfeo_dmat *sC, int ci,
                             int cj, struct blasfeo_dmat *sD, int di,
                             int dj);

/* Variants of potrf_l and syrk_potrf_ln that also write the failure code
 * (see Conventions) to the device int *info (may be NULL). */
void blasfeo_hip_dpotrf_l_info(int m, struct blasfeo_dmat *sC, int ci,
                               int cj, struct blasfeo_dmat *sD, int di,
                               int dj, int *info);
void blasfeo_hip_dsyrk_dpotrf_ln_info(int m, int k, struct blasfeo_dmat *sA,
                                      int ai, int aj,
                                      struct blasfeo_dmat *sB, int bi,
                                      int bj, struct blasfeo_dmat *sC,
                                      int ci, int cj,
                                      struct blasfeo_dmat *sD, int di,
                                      int dj, int *info);

/* ------------------------------------------------------------------------
 * Library state
 * ---------------------------------------------------------------------- */

/* Stream used by the single-instance routines of the calling host thread
 * (a hipStream_t; NULL = the null stream). */
void blasfeo_hip_set_stream(void *stream);
void *blasfeo_hip_get_stream(void);
/* Returns and clears the calling thread's last error (0 = none). */
int blasfeo_hip_get_last_error(void);
/* Static description of an error code. */
const char *blasfeo_hip_strerror(int code);
/* Library version as major*10000 + minor*100 + patch. */
int blasfeo_hip_version(void);

/* ------------------------------------------------------------------------
 * Uniform batches.  A uniform batch of matrices is `batch` consecutive
 * memory chunks of memsize bytes, each laid out as by blasfeo_create_dmat
 * (the paper's memsize guarantee keeps every chunk aligned).  The struct
 * argument describes instance 0; instance b uses pA and dA advanced by
 * b*memsize bytes.  Offsets (ai, aj) apply to every instance.  info is a
 * device array of `batch` ints (may be NULL where no factorization runs).
 * Returns 0, -i for an invalid argument i (nothing launched), or a HIP
 * error code.
 * ---------------------------------------------------------------------- */

/* Packing of a uniform batch: instance b of the column-major source starts
 * strideA doubles after instance b-1 (and of the destination, strideB). */
int blasfeo_hip_pack_dmat_batched(int batch, int m, int n, const double *A,
                                  int lda, long long strideA,
                                  const struct blasfeo_dmat *sB, int bi,
                                  int bj, void *stream);
int blasfeo_hip_unpack_dmat_batched(int batch, int m, int n,
                                    const struct blasfeo_dmat *sA, int ai,
                                    int aj, double *B, int ldb,
                                    long long strideB, void *stream);

/* Pack (to_panel = 1) or unpack (0) `count` m-by-n column-major matrices
 * (instance b at A + b*strideA, leading dimension lda) to/from panel-major
 * chunks (panel length round_up(n, 4)) starting at arena + dst_off[b]
 * doubles; dst_off is a device array.  Used to fill the arenas of a plan
 * size class by size class. */
int blasfeo_hip_pack_dmat_indexed(int count, int m, int n, const double *A,
                                  int lda, long long strideA,
                                  const long long *dst_off, double *arena,
                                  int to_panel, void *stream);

int blasfeo_hip_dgemm_nt_batched(int batch, int m, int n, int k,
                                 double alpha,
                                 const struct blasfeo_dmat *sA, int ai,
                                 int aj, const struct blasfeo_dmat *sB,
                                 int bi, int bj, double beta,
                                 const struct blasfeo_dmat *sC, int ci,
                                 int cj, const struct blasfeo_dmat *sD,
                                 int di, int dj, void *stream);

/* Uniform batch of gemm_nn (same conventions as the gemm_nt batch). */
int blasfeo_hip_dgemm_nn_batched(int batch, int m, int n, int k,
                                 double alpha,
                                 const struct blasfeo_dmat *sA, int ai,
                                 int aj, const struct blasfeo_dmat *sB,
                                 int bi, int bj, double beta,
                                 const struct blasfeo_dmat *sC, int ci,
                                 int cj, const struct blasfeo_dmat *sD,
                                 int di, int dj, void *stream);

/* Uniform batch of getrf (pivot = 1 with partial pivoting, 0 without;
 * m, n <= 256 as above): ipiv[b*min(m,n) + k] (device; may be NULL without
 * pivoting), info[b] = 0 or k+1 for the first zero pivot U[k][k] (device;
 * may be NULL).  Returns 0, -i for bad argument i, or a HIP error code. */
int blasfeo_hip_dgetrf_batched(int batch, int m, int n,
                               const struct blasfeo_dmat *sC, int ci, int cj,
                               const struct blasfeo_dmat *sD, int di, int dj,
                               int pivot, int *ipiv, int *info, void *stream);

/* Uniform batch of gelqf (m, n <= 256 as above; tau of instance b in its
 * D's dA).  Returns 0,
 * -i for bad argument i, or a HIP error code. */
int blasfeo_hip_dgelqf_batched(int batch, int m, int n,
                               const struct blasfeo_dmat *sC, int ci, int cj,
                               const struct blasfeo_dmat *sD, int di, int dj,
                               void *stream);

int blasfeo_hip_dsyrk_ln_batched(int batch, int m, int k, double alpha,
                                 const struct blasfeo_dmat *sA, int ai,
                                 int aj, const struct blasfeo_dmat *sB,
                                 int bi, int bj, double beta,
                                 const struct blasfeo_dmat *sC, int ci,
                                 int cj, const struct blasfeo_dmat *sD,
                                 int di, int dj, void *stream);

/* Uniform batch of trmm_rlnn (same sizes and offsets for every instance,
 * instance b of each operand at its dmat's pA + b * (memsize / 8)).
 * Returns 0, -i for bad argument i (a D sharing storage with B or A: -12),
 * or a HIP error code. */
int blasfeo_hip_dtrmm_rlnn_batched(int batch, int m, int n, double alpha,
                                   const struct blasfeo_dmat *sA, int ai,
                                   int aj, const struct blasfeo_dmat *sB,
                                   int bi, int bj,
                                   const struct blasfeo_dmat *sD, int di,
                                   int dj, void *stream);

int blasfeo_hip_dtrsm_rltn_batched(int batch, int m, int n, double alpha,
                                   const struct blasfeo_dmat *sA, int ai,
                                   int aj, const struct blasfeo_dmat *sB,
                                   int bi, int bj,
                                   const struct blasfeo_dmat *sD, int di,
                                   int dj, void *stream);

int blasfeo_hip_dpotrf_l_batched(int batch, int m,
                                 const struct blasfeo_dmat *sC, int ci,
                                 int cj, const struct blasfeo_dmat *sD,
                                 int di, int dj, int *info, void *stream);

/* Uniform batch of potrf_l_mn; info[b] as for potrf_l (first failing pivot,
 * 1-based, or 0).  Returns 0, -i for bad argument i, or a HIP error code. */
int blasfeo_hip_dpotrf_l_mn_batched(int batch, int m, int n,
                                    const struct blasfeo_dmat *sC, int ci,
                                    int cj, const struct blasfeo_dmat *sD,
                                    int di, int dj, int *info, void *stream);

/* The range-space pair of §4.7.2 as one persistent fused kernel: per
 * instance b
 *     L = chol(Q + A*A^T)         (syrk_ln fused with potrf_l)
 *     X = E * L^{-T}              (trsm_rltn)
 * with A m-by-k (the factor of the update; syrk with both factors equal),
 * Q m-by-m (lower read), E nrhs-by-m, outputs L (lower written, its dA
 * filled) and X nrhs-by-m.  All sub-matrices start at (0,0).  Limits:
 * 1 <= m <= 64, 0 <= k, 0 <= nrhs <= 16.  X may be NULL when nrhs == 0. */
int blasfeo_hip_dsyrk_dpotrf_trsm_batched(int batch, int m, int k, int nrhs,
                                          const struct blasfeo_dmat *sA,
                                          const struct blasfeo_dmat *sQ,
                                          const struct blasfeo_dmat *sE,
                                          const struct blasfeo_dmat *sL,
                                          const struct blasfeo_dmat *sX,
                                          int *info, void *stream);

/* Backward Riccati recursion in square-root form (§5.3), one problem per
 * instance, all N stages in one kernel with no host round trip:
 *   C = [B^T; A^T] Lc_{n+1},  M = blockdiag(R, Q) + C C^T,
 *   F_n = chol(M) = [[Lambda_n, 0], [L_n, Lc_n]],  Lc_N = chol(P_N),
 * for n = N-1 down to 0, with x+ = A x + B u and S = 0 (the reading of the
 * section's equations adopted by this library).  Inputs per instance (uniform
 * batches, lower triangles of Q, R, P_N read): A nx-by-nx, B nx-by-nu, Q, R,
 * P_N.  Output: F is a uniform batch of batch*N matrices of order nu+nx;
 * chunk b*N + n receives the lower triangle of F_n of problem b.  info[b] =
 * 0, or 1000*(n+1) + j for the first failing pivot j (1-based, unpadded)
 * of stage n (n = N for chol(P_N)).  Limits: 1 <= nx <= 32, 1 <= nu <= 16. */
int blasfeo_hip_dric_trf_batched(int batch, int nx, int nu, int N,
                                 const struct blasfeo_dmat *sA,
                                 const struct blasfeo_dmat *sB,
                                 const struct blasfeo_dmat *sQ,
                                 const struct blasfeo_dmat *sR,
                                 const struct blasfeo_dmat *sP,
                                 const struct blasfeo_dmat *sF, int *info,
                                 void *stream);

/* Solution of the linear-quadratic problem whose KKT matrix the recursion
 * above factors (§5.3 gives the factorization; the substitution is the
 * standard one of the square-root form):
 *   min sum_n 1/2 u_n'R u_n + r_n'u_n + 1/2 x_n'Q x_n + q_n'x_n
 *       + 1/2 x_N'P_N x_N + q_N'x_N,
 *   s.t. x_{n+1} = A x_n + B u_n + b_n (n = 0..N-1), x_0 given.
 * Backward: w = P_{n+1} b_n + p_{n+1}, l_n = Lambda_n^{-1}(r_n + B'w),
 * p_n = q_n + A'w - L_n l_n, p_N = q_N, with P_{n+1} = Lc_{n+1} Lc_{n+1}'
 * (P_N for n = N-1); forward: u_n = -Lambda_n^{-T}(L_n' x_n + l_n),
 * x_{n+1} = A x_n + B u_n + b_n.  sA, sB, sP and sF as given to and written
 * by blasfeo_hip_dric_trf_batched (same batch, nx, nu, N; Q and R enter
 * through F).  Vectors are plain device arrays, problem-major, stage rows
 * contiguous: b[(p*N + n)*nx + i], r[(p*N + n)*nu + i],
 * q[(p*(N+1) + n)*nx + i], x0[p*nx + i]; outputs u[(p*N + n)*nu + i] and
 * x[(p*(N+1) + n)*nx + i] (x_0 copied).  The caller owns every buffer.
 * Returns 0, -i for bad argument i, or a HIP error code.  The factors must
 * come from a factorization with info = 0 (no check is made). */
int blasfeo_hip_dric_trs_batched(int batch, int nx, int nu, int N,
                                 const struct blasfeo_dmat *sA,
                                 const struct blasfeo_dmat *sB,
                                 const struct blasfeo_dmat *sP,
                                 const struct blasfeo_dmat *sF,
                                 const double *b, const double *r,
                                 const double *q, const double *x0,
                                 double *u, double *x, void *stream);

/* ------------------------------------------------------------------------
 * Single precision (Appendix A.3 lists every routine in single and double
 * precision; §4.8 sizes the panel per precision so that a panel column fills
 * a cache line).  struct blasfeo_smat has the members of blasfeo_dmat with
 * float pointers; its panels hold BLASFEO_HIP_PS_S = 32 rows, so element
 * (i, j) is at pA[(i - i % 32) * cn + j * 32 + i % 32], cn = round_up(n, 4),
 * and a panel column is again one 128-byte line.  dA holds max(m, n)
 * floats after the panels; memsize is a multiple of 256 bytes.
 * The routines have the arguments, operand rules, error codes and
 * asynchronous behaviour of their double-precision namesakes; alpha and
 * beta are float.  Products accumulate in FP32 on the matrix cores; the
 * 16x16 diagonal blocks of spotrf_l are factored in FP64 and rounded, so
 * L and dA agree with an all-FP32 factorization to FP32 rounding error.
 * ---------------------------------------------------------------------- */
#define BLASFEO_HIP_PS_S 32

struct blasfeo_smat {
  float *pA;
  float *dA;
  int m;
  int n;
  int pm;
  int cn;
  int use_dA;
  int memsize;
};

/* Bytes for an m-by-n single-precision matrix (-1 for a bad size). */
int blasfeo_memsize_smat(int m, int n);
void blasfeo_create_smat(int m, int n, struct blasfeo_smat *sA, void *memory);
void blasfeo_allocate_smat(int m, int n, struct blasfeo_smat *sA);
void blasfeo_free_smat(struct blasfeo_smat *sA);
/* As blasfeo_pack_dmat / blasfeo_unpack_dmat (A, B float device arrays). */
void blasfeo_pack_smat(int m, int n, const float *A, int lda,
                       struct blasfeo_smat *sB, int bi, int bj);
void blasfeo_unpack_smat(int m, int n, struct blasfeo_smat *sA, int ai,
                         int aj, float *B, int ldb);
/* As the dmat batched pack / unpack; strides in floats. */
int blasfeo_hip_pack_smat_batched(int batch, int m, int n, const float *A,
                                  int lda, long long strideA,
                                  const struct blasfeo_smat *sB, int bi,
                                  int bj, void *stream);
int blasfeo_hip_unpack_smat_batched(int batch, int m, int n,
                                    const struct blasfeo_smat *sA, int ai,
                                    int aj, float *B, int ldb,
                                    long long strideB, void *stream);

/* sgemm_nt: D <- alpha*A*B^T + beta*C (as dgemm_nt; errors -1 m, -2 n,
 * -3 k, -5 A, -8 B, -12 C, -15 D through blasfeo_hip_get_last_error). */
void blasfeo_sgemm_nt(int m, int n, int k, float alpha,
                      struct blasfeo_smat *sA, int ai, int aj,
                      struct blasfeo_smat *sB, int bi, int bj, float beta,
                      struct blasfeo_smat *sC, int ci, int cj,
                      struct blasfeo_smat *sD, int di, int dj);
/* ssyrk_ln: lower triangle of D <- alpha*A*B^T + beta*C, A, B m-by-k; the
 * strictly upper part of D is not written (errors -1 m, -2 k, -4 A, -7 B,
 * -11 C, -14 D). */
void blasfeo_ssyrk_ln(int m, int k, float alpha, struct blasfeo_smat *sA,
                      int ai, int aj, struct blasfeo_smat *sB, int bi,
                      int bj, float beta, struct blasfeo_smat *sC, int ci,
                      int cj, struct blasfeo_smat *sD, int di, int dj);
/* spotrf_l: lower Cholesky factor D of the m-by-m SPD matrix C (lower
 * triangle read, strictly upper part of D not written), sD->dA[i] =
 * 1/D[i][i] (errors -1 m, -2 C, -5 D or a NULL dA).  A pivot that is not
 * positive leaves the factor unspecified from that column on. */
void blasfeo_spotrf_l(int m, struct blasfeo_smat *sC, int ci, int cj,
                      struct blasfeo_smat *sD, int di, int dj);
/* Uniform batches (instance b at b*memsize bytes; batch <= 65535).  Error
 * codes are those of the single-instance routine shifted by one (argument
 * i of the batched call is -i), -1 for a bad batch.  info (device, batch
 * ints, may be NULL) receives 0 or the first failing pivot (1-based). */
int blasfeo_hip_sgemm_nt_batched(int batch, int m, int n, int k, float alpha,
                                 const struct blasfeo_smat *sA, int ai, int aj,
                                 const struct blasfeo_smat *sB, int bi, int bj,
                                 float beta, const struct blasfeo_smat *sC,
                                 int ci, int cj, const struct blasfeo_smat *sD,
                                 int di, int dj, void *stream);
int blasfeo_hip_ssyrk_ln_batched(int batch, int m, int k, float alpha,
                                 const struct blasfeo_smat *sA, int ai, int aj,
                                 const struct blasfeo_smat *sB, int bi, int bj,
                                 float beta, const struct blasfeo_smat *sC,
                                 int ci, int cj, const struct blasfeo_smat *sD,
                                 int di, int dj, void *stream);
int blasfeo_hip_spotrf_l_batched(int batch, int m,
                                 const struct blasfeo_smat *sC, int ci, int cj,
                                 const struct blasfeo_smat *sD, int di, int dj,
                                 int *info, void *stream);

/* ------------------------------------------------------------------------
 * Uneven batches: plans.  A plan is created once for a list of orders and
 * executed many times (the embedded-optimization pattern of §2: the same
 * structure is re-solved at every sampling time).
 *
 * Operation per instance i (potrf_l then the forward/back substitution of
 * trsv_lnn/trsv_ltn, §5.2.2 and Appendix A.3):
 *     L_i = chol(A_i),   X_i = A_i^{-1} B_i = L_i^{-T} L_i^{-1} B_i.
 * Memory layout (fixed by the plan, queried with blasfeo_hip_plan_layout):
 *   - A_i (lower part read) is a blasfeo_dmat(n_i, n_i) chunk at byte offset
 *     mat_off[i] of a matrix arena of mat_bytes bytes; L_i (lower part and
 *     its dA written) lives at the same offset of a second arena.
 *   - B_i and X_i are column-major n_i x nrhs blocks, leading dimension
 *     round_up(n_i, 16), at byte offset vec_off[i] of two vector arenas of
 *     vec_bytes bytes.
 * The plan sorts the instances into size classes (n <= 16, 32, 48, 64: one
 * wavefront per instance; 64 < n <= 192 and n > 192: one workgroup per
 * instance, largest first) and launches one kernel per class.
 * Memory: plan creation allocates with hipMalloc a small device table
 * (orders, offsets, class lists).  Scratch memory is the caller's: a device
 * WORKSPACE of the size reported at creation (or by
 * blasfeo_hip_plan_workspace), 256-byte aligned, holding for the instances
 * with n > 64 the inverses of the 16x16 diagonal blocks of L (2 KiB per
 * 16-row block, kept for the back substitution).  Execution and the
 * mixed-precision call allocate nothing and instantiate nothing; a hipGraph
 * of the class launches is recorded only by blasfeo_hip_plan_capture.
 * Concurrent calls on one plan must use distinct workspaces (the workspace
 * is per call, the plan itself is read-only during execution).
 * ---------------------------------------------------------------------- */
typedef struct blasfeo_hip_plan blasfeo_hip_plan;

/* batch >= 0 instances of orders n_host[i] in 1..512, nrhs in 0..16.
 * Returns 0 or -i / HIP error; *plan receives the plan and
 * *workspace_bytes (may be NULL) the bytes of the workspace that
 * blasfeo_hip_dposv_vbatched needs (0 when no order exceeds 64). */
int blasfeo_hip_dposv_vbatched_plan(int batch, const int *n_host, int nrhs,
                                    blasfeo_hip_plan **plan,
                                    long long *workspace_bytes);
/* Workspace sizes: fp64_bytes for blasfeo_hip_dposv_vbatched,
 * mixed_bytes for blasfeo_hip_dposv_mixed_vbatched (0 if the plan cannot
 * run mixed-precision solves: no right-hand sides, or an order/nrhs whose
 * working set exceeds the 160 KiB of LDS of a workgroup).  Either pointer
 * may be NULL.  Returns 0 or -1 (no plan). */
int blasfeo_hip_plan_workspace(const blasfeo_hip_plan *plan,
                               long long *fp64_bytes, long long *mixed_bytes);
/* Byte offsets of every instance (arrays of `batch` entries, may be NULL)
 * and the arena sizes. */
int blasfeo_hip_plan_layout(const blasfeo_hip_plan *plan, long long *mat_off,
                            long long *vec_off, long long *mat_bytes,
                            long long *vec_bytes);
/* Factor and solve every instance (device arenas A, L, B, X; info is a
 * device array of `batch` ints, may be NULL; work: the caller's workspace,
 * may be NULL when its size is 0).  If a graph was captured for exactly
 * these seven pointers, it is replayed; otherwise the class kernels are
 * launched directly.  Allocates nothing.  Asynchronous on `stream`.
 * Returns 0, -i for bad argument i (-7: workspace missing or not 256-byte
 * aligned), or a HIP error. */
int blasfeo_hip_dposv_vbatched(blasfeo_hip_plan *plan, const void *A,
                               void *L, const void *B, void *X, int *info,
                               void *work, void *stream);
/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, environments that forbid hipMalloc): the
 * same operation as blasfeo_hip_dposv_vbatched, with the workspace taken
 * from a fixed device array inside the library instead of a caller's
 * buffer.  The array holds BLASFEO_HIP_NOALLOC_SCRATCH_BYTES (32 MiB) per
 * GPU for the life of the process; a plan whose fp64 workspace is larger
 * (about 16384 diagonal blocks of orders above 64, e.g. 1024 instances of
 * order 256) is rejected with -1, as is a NULL plan.  The class kernels are
 * launched directly (a captured graph is not used).  Nothing is allocated:
 * the array's address is looked up once per device (hipGetSymbolAddress),
 * by blasfeo_hip_noalloc_init or else by the first call on that device,
 * with the device current.  Every call on one GPU shares that GPU's array;
 * calls that overlap in time on one GPU (different streams or threads) race
 * on it and give undefined results.  The array needs no clearing (each
 * block's inverse is written before it is read).  Returns 0, -i for bad
 * argument i, or a HIP error. */
#define BLASFEO_HIP_NOALLOC_SCRATCH_BYTES (32LL << 20)
int blasfeo_hip_noalloc_init(void);
int blasfeo_hip_dposv_vbatched_noalloc(const blasfeo_hip_plan *plan,
                                       const void *A, void *L, const void *B,
                                       void *X, int *info, void *stream);
/* Records the class launches of an execution with these pointers into a
 * hipGraph and instantiates it (replaces any earlier graph of the plan).
 * The size classes touch disjoint instances and become parallel branches of
 * the graph (forked from and joined to the capturing stream through
 * streams and events the plan created), so that one class's last
 * workgroups overlap the others'.  A set-up call: it launches nothing. */
int blasfeo_hip_plan_capture(blasfeo_hip_plan *plan, const void *A, void *L,
                             const void *B, void *X, int *info, void *work);
/* Picks the launch configuration of every size class (the tile and panel
 * shapes of the project's own autotuner, not a paper passage).  A class
 * found in the process's tuning cache (below) takes the cached value and is
 * not run; every other class has each candidate configuration timed on the
 * given data (which is overwritten like an execution), keeps the fastest
 * (waves per workgroup, kernel variant) and enters it into the cache.
 * Synchronizes the stream when anything was timed and drops the captured
 * graph (capture again afterwards).  Returns 0, -1 for a NULL plan, the
 * argument errors of blasfeo_hip_dposv_vbatched, or a HIP error. */
int blasfeo_hip_plan_autotune(blasfeo_hip_plan *plan, const void *A, void *L,
                              const void *B, void *X, int *info, void *work,
                              void *stream);
/* Tuning cache: one process-wide table (guarded by a mutex) from a size
 * class to its configuration.  The key is the device's architecture name
 * and compute-unit count, the class kind (1..4: n <= 16, 32, 48, 64; 0: the
 * n > 64 classes), nrhs, the number of instances and their smallest,
 * largest and summed order; a plan over the same orders on the same kind
 * of device therefore skips the timing runs.  The file is plain text, one
 * entry per line: "arch cus kind nrhs count nmin nmax nsum cfg ms" ('#'
 * starts a comment line; ms is the time measured for cfg, informative).
 *   _load: merges the file's entries into the table; returns their number,
 *          0 if the file does not exist, -1 for a NULL path, -2 for a
 *          malformed line or an invalid configuration (then nothing is
 *          merged).
 *   _save: writes the whole table (through a temporary file renamed into
 *          place); returns the number of entries, -1 for a NULL path, -2 for
 *          an I/O error.
 *   _clear: empties the table and zeroes the counters.
 *   _stats: entries in the table, lookups that hit and that missed (any
 *          pointer may be NULL). */
int blasfeo_hip_tune_cache_load(const char *path);
int blasfeo_hip_tune_cache_save(const char *path);
int blasfeo_hip_tune_cache_clear(void);
int blasfeo_hip_tune_cache_stats(long long *entries, long long *hits, long long *misses);
/* on = 0 never replays a graph (and drops the captured one); on = 1 allows
 * the replay of a graph recorded by blasfeo_hip_plan_capture. */
int blasfeo_hip_plan_set_graph(blasfeo_hip_plan *plan, int on);
/* Writes the chosen configuration of every size class to cfg_out (may be
 * NULL) and returns the number of classes.  Classes 0..3 (n <= 16, 32, 48,
 * 64): wavefronts per workgroup, 1, 2 or 4.  Classes 4 (192 < n <= 512)
 * and 5 (64 < n <= 192): waves per instance, 1, 2, 4, 8 or 16, plus 100 for
 * the variant that stages each block column of the factor in LDS (104, 108,
 * 116), plus 200 for the variant that factors two block columns per step
 * with one block row per downdate group of a wave (201, 202, 204), plus 210
 * for the same with two block rows per group (211, 212, 214). */
int blasfeo_hip_plan_config(const blasfeo_hip_plan *plan, int *cfg_out);
/* Sets the configuration of every size class (count = the number of
 * classes; values as above); drops the captured graph.  Returns 0, -2 for
 * an invalid value, -3 for a wrong count. */
int blasfeo_hip_plan_set_config(blasfeo_hip_plan *plan, const int *cfg, int count);
void blasfeo_hip_plan_destroy(blasfeo_hip_plan *plan);

/* ------------------------------------------------------------------------
 * Mixed-precision solves of a plan's batch (not part of the paper; built on
 * its panel-major storage, §4.3, and blocked Cholesky, §4.6).  Per instance:
 *   S = diag(s), s_p = 2^-floor(e_p / 2) where a_pp = m 2^e_p, m in [0.5, 1)
 *       (exact scaling; s_p = 1 where a_pp is not positive and finite);
 *   L32 = Cholesky factor of fl32(S A S) in single precision: prec 1 with
 *       FP32 matrix-core products, prec 2 with binary16 operands and FP32
 *       accumulation in the downdates;
 *   x0 = S L32^-T L32^-1 fl32(S b); then in FP64: r = b - A x, per
 *       right-hand side eta_c = |r_c|_inf / (|A|_inf |x_c|_inf + |b_c|_inf);
 *       stop when every eta_c <= tol; give up after max_iter corrections or
 *       when some eta_c did not decrease; else x_c += S L32^-T L32^-1
 *       fl32(S r_c) on the columns with eta_c > tol.
 * Arguments: A, B, X are the plan's matrix and vector arenas (same layout
 * as blasfeo_hip_dposv_vbatched; A lower part read; the plan needs
 * nrhs >= 1).  iters (int), berr (double) and fallback (int) are device
 * arrays of `batch` entries:
 *   iters[i]    corrections applied after x0 (largest over the columns),
 *   berr[i]     largest final eta_c (+inf if the factorization failed),
 *   fallback[i] 0 = converged, 1 = low-precision factorization failed
 *               (non-positive pivot), 2 = refinement gave up.
 * If L (a matrix arena) is not NULL, every instance with fallback[i] != 0
 * is then solved again by the FP64 kernels of blasfeo_hip_dposv_vbatched:
 * X_i and L_i receive the FP64 result and info[i] its potrf info.  info
 * (may be NULL) is 0 for every other instance.  If L is NULL, X_i of a
 * fallen-back instance holds the last iterate (factorization failure: X_i
 * untouched).
 * work is the caller's workspace of blasfeo_hip_plan_workspace's
 * mixed_bytes (256-byte aligned): the FP64 workspace of the fallback solves,
 * then the FP32 factor tiles (4 KiB per 16x16 block pair, about
 * 2 n^2 + 32 n floats per instance).  Allocates nothing.  Returns 0, -i for
 * bad argument i (-1 also: a plan whose mixed_bytes is 0), or a HIP error.
 * Asynchronous on `stream`.
 * ---------------------------------------------------------------------- */
#define BLASFEO_HIP_FP32 1
#define BLASFEO_HIP_FP16_SCALED 2
int blasfeo_hip_dposv_mixed_vbatched(blasfeo_hip_plan *plan, int prec,
                                     double tol, int max_iter, const void *A,
                                     const void *B, void *X, void *L,
                                     int *info, int *iters, double *berr,
                                     int *fallback, void *work, void *stream);
/* The FP32 factor L32 of instance i (of S A S, lower triangle, zeros above)
 * left in the workspace `work` by the last mixed-precision call that used
 * it, into the column-major device array dst (leading dimension
 * ldd >= n_i).  Asynchronous on `stream`. */
int blasfeo_hip_plan_mixed_factor(const blasfeo_hip_plan *plan, int i,
                                  const void *work, float *dst, int ldd,
                                  void *stream);

/* ------------------------------------------------------------------------
 * Measurement probes (not part of the paper's API): the attainable rates a
 * roofline of the kernels above is read against, next to the published
 * peaks.  Both are asynchronous on `stream`; the caller times them.
 * ---------------------------------------------------------------------- */
/* Launches `blocks` workgroups of four wavefronts; each wavefront runs
 * `iters` rounds of four independent 16x16x4 FP64 matrix-core products.
 * sink: a device double per block (written only if the accumulated value
 * is -1, i.e. never for these inputs).  Returns the flop count of the
 * launch (> 0), -i for bad argument i, or a HIP error code. */
long long blasfeo_hip_probe_dmfma(int blocks, int iters, double *sink, void *stream);
/* dst = src, `bytes` bytes (a multiple of 16; both 16-byte aligned device
 * pointers), 16-byte accesses in a grid-stride loop.  Returns 0, -i, or a
 * HIP error code. */
int blasfeo_hip_probe_copy(const void *src, void *dst, long long bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* BLASFEO_HIP_H */
