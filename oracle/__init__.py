"""CPU oracle for the panel-major FP64 routines of BLASFEO (arXiv 1704.02457).

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The library in
``paper_1704_02457_amd`` never imports, links or calls it, and the two share no
code: the oracle is plain column-major C triple loops (``oracle.c``,
``batch.c``) plus an independent numpy decoder of the panel-major layout
(``panel.py``).

Every wrapper takes and returns numpy arrays in column-major (Fortran) order.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_ip = ctypes.POINTER(ctypes.c_int)
_lp = ctypes.POINTER(ctypes.c_longlong)
_i, _d = ctypes.c_int, ctypes.c_double


def lib():
    """Load liborc.so, building it with gcc first if it is not there."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.orc_dgemm_nt.argtypes = [_i, _i, _i, _d, _dp, _i, _dp, _i, _d, _dp, _i, _dp, _i]
        L.orc_dsyrk_ln.argtypes = [_i, _i, _d, _dp, _i, _dp, _i, _d, _dp, _i, _dp, _i]
        L.orc_dgemm_nn.argtypes = [_i, _i, _i, _d, _dp, _i, _dp, _i, _d, _dp, _i, _dp, _i]
        L.orc_dpotrf_l.argtypes = [_i, _dp, _i, _dp, _i, _dp]
        L.orc_dpotrf_l.restype = _i
        L.orc_dtrsm_rltn.argtypes = [_i, _i, _d, _dp, _i, _dp, _i, _dp, _i]
        L.orc_dtrmm_rlnn.argtypes = [_i, _i, _d, _dp, _i, _dp, _i, _dp, _i]
        L.orc_dpotrf_l_mn.argtypes = [_i, _i, _dp, _i, _dp, _i, _dp]
        L.orc_dpotrf_l_mn.restype = _i
        L.orc_dgetrf.argtypes = [_i, _i, _dp, _i, _dp, _i, _ip, _dp, _i]
        L.orc_dgetrf.restype = _i
        L.orc_dgelqf.argtypes = [_i, _i, _dp, _i, _dp, _i, _dp]
        L.orc_dsyrk_dpotrf_ln.argtypes = [_i, _i, _dp, _i, _dp, _i, _dp, _i, _dp, _i, _dp]
        L.orc_dsyrk_dpotrf_ln.restype = _i
        L.orc_dpotrs_l.argtypes = [_i, _i, _dp, _i, _dp, _i, _dp, _i]
        L.orc_dsymv_l.argtypes = [_i, _d, _dp, _i, _dp, _d, _dp, _dp]
        L.orc_berr.argtypes = [_i, _dp, _i, _dp, _dp]
        L.orc_berr.restype = _d
        L.orc_ric_trf.argtypes = [_i, _i, _i, _dp, _i, _dp, _i, _dp, _i, _dp, _i, _dp, _i, _dp]
        L.orc_ric_trf.restype = _i
        L.orc_ric_trs.argtypes = [_i, _i, _i, _dp, _i, _dp, _i, _dp, _i, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_spotrf_l.argtypes = [_i, _fp, _i, _fp, _i]
        L.orc_spotrf_l.restype = _i
        L.orc_spotrs_l.argtypes = [_i, _fp, _i, _fp, _fp]
        L.orc_sgemm_nt.argtypes = [_i, _i, _i, ctypes.c_float, _fp, _i, _fp, _i, ctypes.c_float, _fp, _i, _fp, _i]
        L.orc_ssyrk_ln.argtypes = [_i, _i, ctypes.c_float, _fp, _i, _fp, _i, ctypes.c_float, _fp, _i, _fp, _i]
        L.orc_dposv_mixed.argtypes = [_i, _dp, _i, _dp, _d, _i, _i, _dp, _dp]
        L.orc_dposv_mixed.restype = _i
        L.orc_fl16.argtypes = [ctypes.c_float]
        L.orc_fl16.restype = ctypes.c_float
        L.orc_mixed_scale.argtypes = [_i, _dp, _i, _dp]
        L.orc_mixed_factor.argtypes = [_i, _dp, _i, _i, _fp, _i, _dp]
        L.orc_mixed_factor.restype = _i
        L.orc_batch_dposv_mixed.argtypes = [_i, _ip, _lp, _lp, _dp, _dp, _i, _d, _i, _i, _dp, _ip, _dp, _i]
        L.orc_batch_dposv_mixed.restype = _i
        L.orc_batch_syrk_potrf_trsm.argtypes = [_i, _i, _i, _i, _dp, _dp, _dp, _dp, _dp, _dp, _ip, _i]
        L.orc_batch_syrk_potrf_trsm.restype = _i
        L.orc_batch_potrf_potrs.argtypes = [_i, _ip, _lp, _lp, _dp, _dp, _dp, _dp, _dp, _ip, _i]
        L.orc_batch_potrf_potrs.restype = _i
        L.orc_batch_ric_trf.argtypes = [_i, _i, _i, _i, _dp, _dp, _dp, _dp, _dp, _dp, _ip, _i]
        L.orc_batch_ric_trf.restype = _i
        L.orc_batch_dposv_uniform.argtypes = [_i, _i, _i, _dp, _dp, _dp, _dp, _dp, _ip, _i]
        L.orc_batch_dposv_uniform.restype = _i
        L.orc_batch_berr_uniform.argtypes = [_i, _i, _i, _dp, _dp, _dp, _dp, _i]
        L.orc_batch_berr_uniform.restype = _i
        _lib = L
    return _lib


def _f64(a):
    a = np.asarray(a, dtype=np.float64)
    return np.asfortranarray(a)


def _p(a):
    return a.ctypes.data_as(_dp)


def _ld(a):
    return max(1, a.shape[0])


def dgemm_nt(A, B, C, alpha=1.0, beta=1.0):
    """D = alpha*A*B^T + beta*C (Appendix A.2)."""
    A, B, C = _f64(A), _f64(B), _f64(C)
    m, k = A.shape
    n = B.shape[0]
    assert B.shape == (n, k) and C.shape == (m, n)
    D = np.zeros((m, n), order="F")
    lib().orc_dgemm_nt(m, n, k, alpha, _p(A), _ld(A), _p(B), _ld(B), beta, _p(C), _ld(C), _p(D), _ld(D))
    return D


def dgemm_nn(A, B, C, alpha=1.0, beta=1.0):
    """D = alpha*A*B + beta*C."""
    A, B, C = _f64(A), _f64(B), _f64(C)
    m, k = A.shape
    n = B.shape[1]
    assert B.shape == (k, n) and C.shape == (m, n)
    D = np.zeros((m, n), order="F")
    lib().orc_dgemm_nn(m, n, k, alpha, _p(A), _ld(A), _p(B), _ld(B), beta, _p(C), _ld(C), _p(D), _ld(D))
    return D


def dsyrk_ln(A, B, C, alpha=1.0, beta=1.0):
    """Lower triangle of alpha*A*B^T + beta*C; strictly upper part of D is 0."""
    A, B, C = _f64(A), _f64(B), _f64(C)
    m, k = A.shape
    assert B.shape == (m, k) and C.shape == (m, m)
    D = np.zeros((m, m), order="F")
    lib().orc_dsyrk_ln(m, k, alpha, _p(A), _ld(A), _p(B), _ld(B), beta, _p(C), _ld(C), _p(D), _ld(D))
    return D


def dpotrf_l(C):
    """(L, dA, info): lower Cholesky factor of the lower triangle of C."""
    C = _f64(C)
    m = C.shape[0]
    D = np.zeros((m, m), order="F")
    dA = np.zeros(max(m, 1))
    info = lib().orc_dpotrf_l(m, _p(C), _ld(C), _p(D), _ld(D), _p(dA))
    return D, dA[:m], info


def dpotrf_l_mn(C, n):
    """(D, dA, info): D = [L; A L^{-T}] for the stacked m-by-n C = [H; A]."""
    C = _f64(C)
    m = C.shape[0]
    assert C.shape[1] == n and m >= n
    D = np.zeros((m, n), order="F")
    dA = np.zeros(max(n, 1))
    info = lib().orc_dpotrf_l_mn(m, n, _p(C), _ld(C), _p(D), _ld(D), _p(dA))
    return D, dA[:n], info


def dgetrf(C, pivot=True):
    """(D, ipiv, dA, info): LU of C (L unit lower below the diagonal, U
    upper), ipiv 0-based row interchanges, dA = 1/diag(U)."""
    C = _f64(C)
    m, n = C.shape
    D = np.zeros((m, n), order="F")
    mn = min(m, n)
    ipiv = np.zeros(max(mn, 1), dtype=np.int32)
    dA = np.zeros(max(mn, 1))
    info = lib().orc_dgetrf(m, n, _p(C), _ld(C), _p(D), _ld(D), ipiv.ctypes.data_as(_ip), _p(dA), int(pivot))
    return D, ipiv[:mn], dA[:mn], info


def dgelqf(C):
    """(D, tau): compact LQ of C (L on and below the diagonal, the
    Householder vectors above it, v[k] = 1 implicit)."""
    C = _f64(C)
    m, n = C.shape
    D = np.zeros((m, n), order="F")
    tau = np.zeros(max(min(m, n), 1))
    lib().orc_dgelqf(m, n, _p(C), _ld(C), _p(D), _ld(D), _p(tau))
    return D, tau[:min(m, n)]


def lq_q(D, tau):
    """The n-by-n orthogonal Q = H_{k-1} ... H_0 of the compact LQ form
    (A = L Q[:min(m,n)] with L the lower part of D)."""
    D = np.asarray(D, dtype=np.float64)
    n = D.shape[1]
    Q = np.eye(n)
    for k in range(len(tau)):
        v = np.zeros(n)
        v[k] = 1.0
        v[k + 1:] = D[k, k + 1:]
        Q = Q - tau[k] * np.outer(Q @ v, v)  # Q <- Q H_k, H_k = I - tau v v'
    return Q.T


def dtrmm_rlnn(A, B, alpha=1.0):
    """D = alpha * B * A with A lower triangular (only its lower part read)."""
    A, B = _f64(A), _f64(B)
    m, n = B.shape
    assert A.shape == (n, n)
    D = np.zeros((m, n), order="F")
    lib().orc_dtrmm_rlnn(m, n, alpha, _p(A), _ld(A), _p(B), _ld(B), _p(D), _ld(D))
    return D


def dtrsm_rltn(L, B, alpha=1.0):
    """X = alpha * B * L^{-T} with L lower triangular."""
    L, B = _f64(L), _f64(B)
    m, n = B.shape
    assert L.shape == (n, n)
    D = np.zeros((m, n), order="F")
    lib().orc_dtrsm_rltn(m, n, alpha, _p(L), _ld(L), _p(B), _ld(B), _p(D), _ld(D))
    return D


def dsyrk_dpotrf_ln(A, B, C):
    """(L, dA, info) with L = chol(C + A*B^T)."""
    A, B, C = _f64(A), _f64(B), _f64(C)
    m, k = A.shape
    D = np.zeros((m, m), order="F")
    dA = np.zeros(max(m, 1))
    info = lib().orc_dsyrk_dpotrf_ln(m, k, _p(A), _ld(A), _p(B), _ld(B), _p(C), _ld(C), _p(D), _ld(D), _p(dA))
    return D, dA[:m], info


def dpotrs_l(L, B):
    """X solving (L L^T) X = B, column by column."""
    L = _f64(L)
    B = _f64(B if np.ndim(B) == 2 else np.reshape(B, (-1, 1)))
    n, nrhs = B.shape
    X = np.zeros((n, nrhs), order="F")
    lib().orc_dpotrs_l(n, nrhs, _p(L), _ld(L), _p(B), _ld(B), _p(X), _ld(X))
    return X


def dsymv_l(A, x, y, alpha=1.0, beta=1.0):
    A = _f64(A)
    x, y = _f64(x).ravel(), _f64(y).ravel()
    z = np.zeros(A.shape[0])
    lib().orc_dsymv_l(A.shape[0], alpha, _p(A), _ld(A), _p(x), beta, _p(y), _p(z))
    return z


def berr(A, x, b):
    """Normwise backward error of x for A x = b (lower triangle of A read)."""
    A = _f64(A)
    x, b = _f64(x).ravel(), _f64(b).ravel()
    return lib().orc_berr(A.shape[0], _p(A), _ld(A), _p(x), _p(b))


def ric_trf(A, B, Q, R, PN, N):
    """(F, info): the N stage factors of the square-root Riccati recursion.

    F has shape (N, nu+nx, nu+nx); F[n] is the lower factor of stage n.
    """
    A, B, Q, R, PN = (_f64(x) for x in (A, B, Q, R, PN))
    nx, nu = B.shape
    nm = nu + nx
    F = np.zeros((N * nm * nm,))
    info = lib().orc_ric_trf(nx, nu, N, _p(A), _ld(A), _p(B), _ld(B), _p(Q), _ld(Q), _p(R), _ld(R), _p(PN), _ld(PN), _p(F))
    return F.reshape(N, nm, nm).transpose(0, 2, 1).copy(), info


def ric_trs(A, B, PN, F, b, r, q, x0):
    """(u, x): controls (N, nu) and states (N+1, nx) of the linear-quadratic
    problem whose stage factors F (from ric_trf) are given; b (N, nx),
    r (N, nu), q (N+1, nx), x0 (nx,)."""
    A, B, PN = (_f64(x) for x in (A, B, PN))
    nx, nu = B.shape
    N = F.shape[0]
    Fc = np.ascontiguousarray(np.asarray(F, dtype=np.float64).transpose(0, 2, 1))  # column-major blocks
    b, r, q, x0 = (np.ascontiguousarray(np.asarray(v, dtype=np.float64)) for v in (b, r, q, x0))
    assert b.shape == (N, nx) and r.shape == (N, nu) and q.shape == (N + 1, nx) and x0.shape == (nx,)
    u = np.zeros((N, nu))
    x = np.zeros((N + 1, nx))
    lib().orc_ric_trs(nx, nu, N, _p(A), _ld(A), _p(B), _ld(B), _p(PN), _ld(PN), _p(Fc), _p(b), _p(r), _p(q),
                      _p(x0), _p(u), _p(x))
    return u, x


def spotrf_l(C):
    C = np.asfortranarray(np.asarray(C, dtype=np.float32))
    m = C.shape[0]
    D = np.zeros((m, m), dtype=np.float32, order="F")
    info = lib().orc_spotrf_l(m, C.ctypes.data_as(_fp), max(1, m), D.ctypes.data_as(_fp), max(1, m))
    return D, info


def _f32(a):
    return np.asfortranarray(np.asarray(a, dtype=np.float32))


def sgemm_nt(A, B, C, alpha=1.0, beta=1.0):
    """Single precision D = alpha*A*B^T + beta*C."""
    A, B, C = _f32(A), _f32(B), _f32(C)
    m, k = A.shape
    n = B.shape[0]
    D = np.zeros((m, n), dtype=np.float32, order="F")
    fp = lambda x: x.ctypes.data_as(_fp)  # noqa: E731
    lib().orc_sgemm_nt(m, n, k, alpha, fp(A), max(1, m), fp(B), max(1, n), beta, fp(C), max(1, m), fp(D), max(1, m))
    return D


def ssyrk_ln(A, B, C, alpha=1.0, beta=1.0):
    """Single precision lower(alpha*A*B^T + beta*C); the strictly upper part is 0."""
    A, B, C = _f32(A), _f32(B), _f32(C)
    m, k = A.shape
    D = np.zeros((m, m), dtype=np.float32, order="F")
    fp = lambda x: x.ctypes.data_as(_fp)  # noqa: E731
    lib().orc_ssyrk_ln(m, k, alpha, fp(A), max(1, m), fp(B), max(1, m), beta, fp(C), max(1, m), fp(D), max(1, m))
    return D


FP32, FP16_SCALED = 1, 2


def fl16(x):
    """Nearest binary16 value of the binary32 value x, as a Python float."""
    return float(lib().orc_fl16(float(np.float32(x))))


def mixed_scale(A):
    """Power-of-two diagonal scaling s of the mixed-precision solve."""
    A = _f64(A)
    n = A.shape[0]
    s = np.zeros(n)
    lib().orc_mixed_scale(n, _p(A), _ld(A), _p(s))
    return s


def mixed_factor(A, prec=FP32):
    """(L32, s, info): low-precision Cholesky factor of S A S, S = diag(s)."""
    A = _f64(A)
    n = A.shape[0]
    L = np.zeros((n, n), dtype=np.float32, order="F")
    s = np.zeros(n)
    info = lib().orc_mixed_factor(n, _p(A), _ld(A), prec, L.ctypes.data_as(_fp), max(1, n), _p(s))
    return L, s, info


def dposv_mixed(A, b, tol=1e-12, max_iter=10, prec=FP32):
    """(x, corrections or negative code, eta) of the low-precision-factor +
    FP64-refinement solve (-1: factorization failed, -2: gave up)."""
    A = _f64(A)
    b = _f64(b).ravel()
    n = A.shape[0]
    x = np.zeros(n)
    eta = np.zeros(1)
    it = lib().orc_dposv_mixed(n, _p(A), _ld(A), _p(b), tol, max_iter, prec, _p(x), _p(eta))
    return x, it, float(eta[0])


# ---- batched drivers (column-major instances stored one after another) ----

def batch_syrk_potrf_trsm(Q, B, RHS, nthreads=0):
    """Q (b,n,n), B (b,n,k), RHS (b,nrhs,n) as C-order stacks of matrices.

    Returns (L, X, dA, info, threads) with L (b,n,n), X (b,nrhs,n).
    """
    bq, n, _ = Q.shape
    k = B.shape[2]
    nrhs = RHS.shape[1]
    # column-major instances: transpose the last two axes into contiguous storage
    Qc = np.ascontiguousarray(np.swapaxes(Q, 1, 2), dtype=np.float64)
    Bc = np.ascontiguousarray(np.swapaxes(B, 1, 2), dtype=np.float64)
    Rc = np.ascontiguousarray(np.swapaxes(RHS, 1, 2), dtype=np.float64)
    L = np.zeros((bq, n, n))
    X = np.zeros((bq, n, nrhs))
    dA = np.zeros((bq, n))
    info = np.zeros(bq, dtype=np.int32)
    used = lib().orc_batch_syrk_potrf_trsm(bq, n, k, nrhs, _p(Qc), _p(Bc), _p(Rc), _p(L), _p(X), _p(dA),
                                           info.ctypes.data_as(_ip), nthreads)
    return np.swapaxes(L, 1, 2), np.swapaxes(X, 1, 2), dA, info, used


def batch_potrf_potrs(mats, rhs, nthreads=0):
    """Uneven batch: lists of (n,n) matrices and (n,) vectors.

    Returns (list of L, list of x, list of dA, info, threads).
    """
    bsz = len(mats)
    ns = np.array([m.shape[0] for m in mats], dtype=np.int32)
    offA = np.zeros(bsz, dtype=np.int64)
    offv = np.zeros(bsz, dtype=np.int64)
    offA[1:] = np.cumsum(ns.astype(np.int64) ** 2)[:-1]
    offv[1:] = np.cumsum(ns.astype(np.int64))[:-1]
    Aall = np.concatenate([np.asarray(m, dtype=np.float64).ravel(order="F") for m in mats]) if bsz else np.zeros(1)
    ball = np.concatenate([np.asarray(v, dtype=np.float64).ravel() for v in rhs]) if bsz else np.zeros(1)
    L = np.zeros_like(Aall)
    x = np.zeros_like(ball)
    dA = np.zeros_like(ball)
    info = np.zeros(max(bsz, 1), dtype=np.int32)
    used = lib().orc_batch_potrf_potrs(bsz, ns.ctypes.data_as(_ip), offA.ctypes.data_as(_lp), offv.ctypes.data_as(_lp),
                                       _p(Aall), _p(ball), _p(L), _p(dA), _p(x), info.ctypes.data_as(_ip), nthreads)
    Ls, xs, ds = [], [], []
    for i in range(bsz):
        n = int(ns[i])
        Ls.append(L[offA[i]:offA[i] + n * n].reshape(n, n, order="F"))
        xs.append(x[offv[i]:offv[i] + n])
        ds.append(dA[offv[i]:offv[i] + n])
    return Ls, xs, ds, info[:bsz], used


def batch_ric_trf(A, B, Q, R, PN, N, nthreads=0):
    """A,Q,PN (b,nx,nx), B (b,nx,nu), R (b,nu,nu) C-order stacks.

    Returns (F (b,N,nm,nm), info, threads).
    """
    bsz, nx, nu = B.shape
    nm = nx + nu
    conv = [np.ascontiguousarray(np.swapaxes(x, 1, 2), dtype=np.float64) for x in (A, B, Q, R, PN)]
    F = np.zeros((bsz, N, nm, nm))
    info = np.zeros(bsz, dtype=np.int32)
    used = lib().orc_batch_ric_trf(bsz, nx, nu, N, *[_p(c) for c in conv], _p(F), info.ctypes.data_as(_ip), nthreads)
    return np.swapaxes(F, 2, 3), info, used


def batch_dposv_mixed(mats, rhs, tol=1e-12, max_iter=10, prec=FP32, nthreads=0):
    """Uneven batch of mixed-precision solves: lists of (n,n) matrices and
    (n,nrhs) right-hand sides.  Returns (list of X, iters, eta, threads)."""
    bsz = len(mats)
    ns = np.array([m.shape[0] for m in mats], dtype=np.int32)
    nrhs = int(np.asarray(rhs[0]).reshape(ns[0], -1).shape[1]) if bsz else 1
    offA = np.zeros(bsz, dtype=np.int64)
    offv = np.zeros(bsz, dtype=np.int64)
    offA[1:] = np.cumsum(ns.astype(np.int64) ** 2)[:-1]
    offv[1:] = np.cumsum(ns.astype(np.int64) * nrhs)[:-1]
    Aall = np.concatenate([np.asarray(m, dtype=np.float64).ravel(order="F") for m in mats]) if bsz else np.zeros(1)
    Ball = np.concatenate([np.asarray(v, dtype=np.float64).reshape(m.shape[0], nrhs).ravel(order="F")
                           for m, v in zip(mats, rhs)]) if bsz else np.zeros(1)
    X = np.zeros_like(Ball)
    iters = np.zeros(max(bsz, 1), dtype=np.int32)
    eta = np.zeros(max(bsz, 1))
    used = lib().orc_batch_dposv_mixed(bsz, ns.ctypes.data_as(_ip), offA.ctypes.data_as(_lp), offv.ctypes.data_as(_lp),
                                       _p(Aall), _p(Ball), nrhs, tol, max_iter, prec, _p(X),
                                       iters.ctypes.data_as(_ip), _p(eta), nthreads)
    Xs = [X[offv[i]:offv[i] + int(ns[i]) * nrhs].reshape(int(ns[i]), nrhs, order="F") for i in range(bsz)]
    return Xs, iters[:bsz], eta[:bsz], used


def _colmajor_stack(M):
    """(b, r, c) C-order stack -> contiguous stack of column-major instances."""
    return np.ascontiguousarray(np.swapaxes(np.asarray(M, dtype=np.float64), 1, 2))


def batch_dposv_uniform(A, B, nthreads=0):
    """Chunk of Cholesky solves of one order: A (b,n,n) (lower triangle
    read), B (b,n,nrhs) C-order stacks.  Returns (L (b,n,n), X (b,n,nrhs),
    dA (b,n), info, threads); X of a failed instance is zero."""
    bsz, n, _ = A.shape
    nrhs = B.shape[2]
    Ac, Bc = _colmajor_stack(A), _colmajor_stack(B)
    L = np.zeros((bsz, n, n))
    X = np.zeros((bsz, nrhs, n))
    dA = np.zeros((bsz, n))
    info = np.zeros(max(bsz, 1), dtype=np.int32)
    used = lib().orc_batch_dposv_uniform(bsz, n, nrhs, _p(Ac), _p(Bc), _p(L), _p(dA), _p(X),
                                         info.ctypes.data_as(_ip), nthreads)
    return np.swapaxes(L, 1, 2), np.swapaxes(X, 1, 2), dA, info[:bsz], used


def batch_berr_uniform(A, X, B, nthreads=0):
    """Largest normwise backward error over the columns of X_b for
    A_b x = b (lower triangle of A_b read), for a (b,n,n) stack A and
    (b,n,nrhs) stacks X, B.  Returns (eta (b,), threads)."""
    bsz, n, _ = A.shape
    nrhs = B.shape[2]
    Ac, Xc, Bc = _colmajor_stack(A), _colmajor_stack(X), _colmajor_stack(B)
    eta = np.zeros(max(bsz, 1))
    used = lib().orc_batch_berr_uniform(bsz, n, nrhs, _p(Ac), _p(Xc), _p(Bc), _p(eta), nthreads)
    return eta[:bsz], used
