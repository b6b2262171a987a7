"""Pins of the CPU oracle against facts that do not come from the oracle itself:
hand-derived fixtures, closed forms, exact rational arithmetic on tiny inputs,
50-digit decimal Cholesky, invariants and special cases.  CPU only."""
import ctypes
import os
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")
U = 2.0 ** -53


def _read_fixture(name):
    rows = {}
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            rows.setdefault(key, []).append(vals)
    return rows


def _frac_mat(X):
    return [[Fraction(float(v)) for v in row] for row in np.asarray(X)]


# ----------------------------------------------------------------- gemm_nt

@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (3, 5, 2), (7, 4, 8), (8, 8, 8)])
def test_gemm_nt_exact_rational_bound(m, n, k):
    """Every entry lies within the standard dot-product bound of the exact
    rational value of alpha*A*B^T + beta*C."""
    rng = np.random.default_rng(100 + m * 31 + n * 7 + k)
    A, B, C = rng.uniform(-1, 1, (m, k)), rng.uniform(-1, 1, (n, k)), rng.uniform(-1, 1, (m, n))
    alpha, beta = 0.75, -1.25
    D = oracle.dgemm_nt(A, B, C, alpha, beta)
    Af, Bf, Cf = _frac_mat(A), _frac_mat(B), _frac_mat(C)
    gam = (k + 2) * U / (1 - (k + 2) * U)
    for i in range(m):
        for j in range(n):
            ex = Fraction(beta) * Cf[i][j] + Fraction(alpha) * sum(Af[i][l] * Bf[j][l] for l in range(k))
            mag = abs(beta * C[i, j]) + abs(alpha) * sum(abs(A[i, l] * B[j, l]) for l in range(k))
            assert abs(float(Fraction(D[i, j]) - ex)) <= gam * mag + 1e-300


def test_gemm_nt_integers_exact():
    rng = np.random.default_rng(5)
    A = rng.integers(-9, 10, (6, 5)).astype(float)
    B = rng.integers(-9, 10, (4, 5)).astype(float)
    C = rng.integers(-9, 10, (6, 4)).astype(float)
    D = oracle.dgemm_nt(A, B, C, 2.0, -3.0)
    exp = [[-3 * int(C[i, j]) + 2 * sum(int(A[i, l]) * int(B[j, l]) for l in range(5)) for j in range(4)] for i in range(6)]
    assert np.array_equal(D, np.array(exp, dtype=float))


def test_gemm_nt_identity_right_factor():
    """With B = I, D = A + C exactly (alpha = beta = 1)."""
    rng = np.random.default_rng(6)
    A, C = rng.standard_normal((9, 9)), rng.standard_normal((9, 9))
    assert np.array_equal(oracle.dgemm_nt(A, np.eye(9), C), A + C)


def test_gemm_nt_in_place_c_equals_d():
    """C and D may coincide (Appendix A.2)."""
    rng = np.random.default_rng(7)
    A, B = rng.integers(-3, 4, (5, 3)).astype(float), rng.integers(-3, 4, (4, 3)).astype(float)
    C = np.asfortranarray(rng.integers(-3, 4, (5, 4)).astype(float))
    exp = C + A @ B.T
    L = oracle.lib()
    p = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    Af, Bf = np.asfortranarray(A), np.asfortranarray(B)
    L.orc_dgemm_nt(5, 4, 3, 1.0, p(Af), 5, p(Bf), 4, 1.0, p(C), 5, p(C), 5)
    assert np.array_equal(C, exp)


# ----------------------------------------------------------------- syrk_ln

def test_syrk_ln_rational_and_upper_untouched():
    rng = np.random.default_rng(8)
    m, k = 7, 5
    A, B, C = rng.uniform(-1, 1, (m, k)), rng.uniform(-1, 1, (m, k)), rng.uniform(-1, 1, (m, m))
    Af, Bf, Cf = (np.asfortranarray(x) for x in (A, B, C))
    D = np.full((m, m), 123.5, order="F")
    p = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    oracle.lib().orc_dsyrk_ln(m, k, 0.5, p(Af), m, p(Bf), m, 2.0, p(Cf), m, p(D), m)
    gam = (k + 2) * U / (1 - (k + 2) * U)
    for i in range(m):
        for j in range(m):
            if i < j:
                assert D[i, j] == 123.5
                continue
            ex = 2 * Fraction(C[i, j]) + Fraction(0.5) * sum(Fraction(A[i, l]) * Fraction(B[j, l]) for l in range(k))
            mag = 2 * abs(C[i, j]) + 0.5 * sum(abs(A[i, l] * B[j, l]) for l in range(k))
            assert abs(float(Fraction(D[i, j]) - ex)) <= gam * mag


def test_syrk_ln_two_different_factors():
    """A and B may differ: the result is the lower part of C + A B^T, not of
    C + A A^T or C + B A^T (catches a swapped operand)."""
    A = np.array([[1.0, 2.0], [3.0, 4.0], [5.0, 6.0]])
    B = np.array([[0.0, 1.0], [1.0, 0.0], [2.0, -1.0]])
    C = np.zeros((3, 3))
    D = oracle.dsyrk_ln(A, B, C)
    exp = np.tril(A @ B.T)
    assert np.array_equal(D, exp)
    assert not np.array_equal(exp, np.tril(B @ A.T))


# ----------------------------------------------------------------- potrf_l

def test_potrf_golden_4x4():
    g = _read_fixture("chol_4x4.txt")
    L = np.array(g["L"], dtype=float)
    A = np.array(g["A"], dtype=float)
    dA = np.array(g["dA"][0], dtype=float)
    assert np.array_equal(L @ L.T, A)  # the fixture is self-consistent
    D, d, info = oracle.dpotrf_l(A)
    assert info == 0
    assert np.array_equal(D, L)
    assert np.array_equal(d, dA)


@pytest.mark.parametrize("n", [1, 2, 5, 16, 33, 64])
def test_potrf_small_integer_exact(n):
    L, A = synth.small_integer_factor(n, seed=n)
    D, dA, info = oracle.dpotrf_l(A)
    assert info == 0
    assert np.array_equal(D, L)
    assert np.array_equal(dA, 1.0 / np.diag(L))


def test_potrf_reads_only_lower():
    L, A = synth.small_integer_factor(12, seed=3)
    A2 = A.copy()
    A2[np.triu_indices(12, 1)] = np.nan
    D, _, info = oracle.dpotrf_l(A2)
    assert info == 0 and np.array_equal(D, L)


def test_potrf_identity_and_diagonal():
    D, dA, info = oracle.dpotrf_l(np.eye(7))
    assert info == 0 and np.array_equal(D, np.eye(7)) and np.array_equal(dA, np.ones(7))
    d = np.array([2.0, 3.0, 0.5, 7.0, 1e-3, 1e5])
    D, dA, info = oracle.dpotrf_l(np.diag(d))
    assert info == 0
    assert np.array_equal(np.diag(D), np.sqrt(d))
    assert np.array_equal(dA, 1.0 / np.sqrt(d))
    assert np.count_nonzero(D - np.diag(np.diag(D))) == 0


@pytest.mark.parametrize("n", [2, 3, 5, 8])
def test_potrf_decimal_50_digits(n):
    """Cholesky in 50-digit decimal arithmetic agrees to ~n*u relative."""
    getcontext().prec = 50
    rng = np.random.default_rng(40 + n)
    M = rng.uniform(-1, 1, (n, n))
    A = M @ M.T + n * np.eye(n)
    A = 0.5 * (A + A.T)
    Ad = [[Decimal(float(A[i, j])) for j in range(n)] for i in range(n)]
    Ld = [[Decimal(0)] * n for _ in range(n)]
    for j in range(n):
        s = Ad[j][j] - sum(Ld[j][k] * Ld[j][k] for k in range(j))
        Ld[j][j] = s.sqrt()
        for i in range(j + 1, n):
            Ld[i][j] = (Ad[i][j] - sum(Ld[i][k] * Ld[j][k] for k in range(j))) / Ld[j][j]
    Lref = np.array([[float(v) for v in row] for row in Ld])
    D, _, info = oracle.dpotrf_l(A)
    assert info == 0
    assert np.linalg.norm(D - Lref) / np.linalg.norm(Lref) <= 4 * n * U


def test_potrf_residual_and_numpy_crosscheck():
    rng = np.random.default_rng(9)
    n = 40
    G = rng.standard_normal((n, n))
    A = G @ G.T + n * np.eye(n)
    D, _, info = oracle.dpotrf_l(A)
    assert info == 0
    assert np.linalg.norm(D @ D.T - A) / np.linalg.norm(A) <= 10 * n * U
    assert np.allclose(D, np.linalg.cholesky(A), rtol=0, atol=1e-12)
    assert np.all(np.diag(D) > 0) and np.count_nonzero(np.triu(D, 1)) == 0


@pytest.mark.parametrize("bad", [0, 3, 9])
def test_potrf_info_first_failing_pivot(bad):
    L, A = synth.small_integer_factor(10, seed=21)
    A = A.copy()
    # make the pivot of column `bad` exactly zero: d_bad = A[bad,bad] - sum L[bad,k]^2 = 0
    A[bad, bad] -= L[bad, bad] ** 2
    D, _, info = oracle.dpotrf_l(A)
    assert info == bad + 1
    assert np.array_equal(D[:, :bad], L[:, :bad])
    A[bad, bad] -= 1.0  # negative pivot
    assert oracle.dpotrf_l(A)[2] == bad + 1


# ----------------------------------------------------------------- gemm_nn

def test_gemm_nn_integer_exact_and_against_nt():
    rng = np.random.default_rng(70)
    for m, n, k in ((1, 1, 1), (7, 5, 9), (33, 17, 40)):
        A = rng.integers(-4, 5, (m, k))
        B = rng.integers(-4, 5, (k, n))
        C = rng.integers(-4, 5, (m, n))
        exact = (A.astype(np.int64) @ B.astype(np.int64)) * 3 - 2 * C.astype(np.int64)
        D = oracle.dgemm_nn(A.astype(float), B.astype(float), C.astype(float), alpha=3.0, beta=-2.0)
        assert np.array_equal(D, exact.astype(float))
        # the NN product is the NT product with the transposed right factor
        Af, Bf, Cf = (rng.uniform(-1, 1, s) for s in ((m, k), (k, n), (m, n)))
        assert np.array_equal(oracle.dgemm_nn(Af, Bf, Cf, 0.5, 1.5), oracle.dgemm_nt(Af, Bf.T, Cf, 0.5, 1.5))


# ----------------------------------------------------------------- getrf

def test_getrf_matches_lapack_pivots_and_factors():
    """Partial pivoting: the same interchanges as LAPACK's getrf (scipy's
    lu_factor, 0-based) and the same packed L\\U, on square and
    rectangular matrices."""
    import scipy.linalg as sl
    rng = np.random.default_rng(80)
    for m, n in ((1, 1), (6, 6), (40, 40), (64, 64), (30, 17), (17, 30)):
        C = rng.standard_normal((m, n))
        D, ipiv, dA, info = oracle.dgetrf(C, pivot=True)
        assert info == 0
        lu, piv = sl.lu_factor(C)
        assert np.array_equal(ipiv, piv[:min(m, n)])
        assert np.linalg.norm(D - lu) <= 1e-13 * max(m, n) * np.linalg.norm(lu)
        assert np.array_equal(dA, 1.0 / np.diag(D)[:min(m, n)])


def test_getrf_exact_small_integers():
    """A = L U with unit-lower integer L and integer U whose diagonal is a
    power of two: no pivoting returns L and U exactly; with pivoting
    P A = L' U' holds exactly for the returned factors."""
    rng = np.random.default_rng(81)
    for n in (5, 23, 64):
        Lm = np.tril(rng.integers(-2, 3, (n, n)), -1) + np.eye(n)
        U = np.triu(rng.integers(-2, 3, (n, n)), 1) + np.diag(rng.choice([1.0, 2.0, -1.0, 4.0], n))
        A = Lm @ U
        D, ipiv, _, info = oracle.dgetrf(A, pivot=False)
        assert info == 0 and np.array_equal(ipiv, np.arange(n))
        assert np.array_equal(np.tril(D, -1) + np.eye(n), Lm) and np.array_equal(np.triu(D), U)
        D, ipiv, _, info = oracle.dgetrf(A, pivot=True)
        PA = A.copy()
        for k, pk in enumerate(ipiv):
            PA[[k, pk]] = PA[[pk, k]]
        L2, U2 = np.tril(D, -1) + np.eye(n), np.triu(D)
        assert np.linalg.norm(L2 @ U2 - PA) <= 1e-12 * np.linalg.norm(A)
        assert np.all(np.abs(np.tril(D, -1)) <= 1.0)  # partial pivoting bounds the multipliers


def test_getrf_zero_pivot_info():
    A = np.array([[0.0, 1.0], [1.0, 1.0]])
    assert oracle.dgetrf(A, pivot=False)[3] == 1
    D, ipiv, _, info = oracle.dgetrf(A, pivot=True)
    assert info == 0 and list(ipiv) == [1, 1]
    assert oracle.dgetrf(np.array([[1.0, 2.0], [2.0, 4.0]]), pivot=True)[3] == 2


# ----------------------------------------------------------------- gelqf

@pytest.mark.parametrize("m,n", [(1, 1), (3, 5), (5, 5), (7, 4), (40, 64), (64, 64), (64, 17)])
def test_gelqf_matches_lapack_and_reconstructs(m, n):
    """The compact LQ form equals LAPACK's QR of A^T transposed (the same
    reflectors: geqrf on A^T annihilates the columns that gelqf annihilates
    in the rows of A), L Q reproduces A, Q is orthogonal."""
    import scipy.linalg.lapack as la
    rng = np.random.default_rng(m * 100 + n)
    A = rng.standard_normal((m, n))
    D, tau = oracle.dgelqf(A)
    qr, t2, _, info = la.dgeqrf(np.asfortranarray(A.T))
    assert info == 0
    assert np.abs(D - qr.T).max() <= 1e-14 * max(m, n) * np.abs(qr).max()
    assert np.abs(tau - t2[:min(m, n)]).max() <= 1e-14 * max(m, n)
    Q = oracle.lq_q(D, tau)
    k = min(m, n)
    assert np.abs(np.tril(D)[:, :k] @ Q[:k] - A).max() <= 1e-14 * max(m, n) * np.abs(A).max()
    assert np.abs(Q @ Q.T - np.eye(n)).max() <= 1e-14 * n


def test_gelqf_special_cases():
    # a row already zero to the right of the diagonal gives tau = 0 (H = I)
    A = np.array([[3.0, 0.0, 0.0], [1.0, 2.0, 2.0]])
    D, tau = oracle.dgelqf(A)
    assert tau[0] == 0.0 and D[0, 0] == 3.0
    # a 3-4-5 row: beta = -5, tau = 8/5, v = [1, 1/2]
    D, tau = oracle.dgelqf(np.array([[3.0, 4.0]]))
    assert D[0, 0] == -5.0 and tau[0] == 1.6 and D[0, 1] == 0.5


# ----------------------------------------------------------------- potrf_l_mn (stacking)

def test_potrf_l_mn_exact_stacked():
    """C = [L L^T; Y L^T] from a small-integer L with power-of-two diagonal
    and an integer Y is exact in FP64, and so is every step of the
    factorization: the result must be [L; Y] exactly."""
    for m, n, seed in ((5, 3, 50), (40, 24, 51), (70, 33, 52), (16, 16, 53)):
        L, LL = synth.small_integer_factor(n, seed=seed)
        Y = np.random.default_rng(seed).integers(-3, 4, (m - n, n)).astype(float)
        C = np.vstack([LL, Y @ L.T])
        C[:n][np.triu_indices(n, 1)] = np.nan  # the top block's upper part is not read
        D, dA, info = oracle.dpotrf_l_mn(C, n)
        assert info == 0
        assert np.array_equal(D, np.vstack([L, Y]))
        assert np.array_equal(dA, 1.0 / np.diag(L))


def test_potrf_l_mn_square_is_potrf_and_failure():
    rng = np.random.default_rng(54)
    G = rng.standard_normal((9, 9))
    H = G @ G.T + 9 * np.eye(9)
    D, dA, info = oracle.dpotrf_l_mn(H, 9)
    Lr, dAr, ir = oracle.dpotrf_l(H)
    assert info == ir == 0 and np.array_equal(D, Lr) and np.array_equal(dA, dAr)
    C = np.vstack([H, rng.standard_normal((4, 9))])
    C[5, 5] = -50.0
    assert oracle.dpotrf_l_mn(C, 9)[2] == 6


def test_range_space_chain_matches_dense_kkt():
    """The range-space method of the stacking passage: potrf_l_mn([H; A]) =
    [L; Y], then chol(Y Y^T) = chol(A H^-1 A^T); solving the normal
    equations with it gives the multipliers and the primal solution of the
    dense KKT system."""
    rng = np.random.default_rng(55)
    n, ma = 24, 10
    G = rng.standard_normal((n, n))
    H = G @ G.T / n + np.eye(n)
    A = rng.standard_normal((ma, n))
    g, bvec = rng.standard_normal(n), rng.standard_normal(ma)
    D, _, info = oracle.dpotrf_l_mn(np.vstack([H, A]), n)
    assert info == 0
    L, Y = D[:n], D[n:]
    Ls, _, info2 = oracle.dsyrk_dpotrf_ln(Y, Y, np.zeros((ma, ma)))
    assert info2 == 0
    # normal equations A H^-1 A^T lam = b - A H^-1 g, with H^-1 = L^-T L^-1
    Hinv_g = np.linalg.solve(L.T, np.linalg.solve(L, g))
    rhs = bvec - A @ Hinv_g
    lam = np.linalg.solve(Ls.T, np.linalg.solve(Ls, rhs))
    x = -np.linalg.solve(L.T, np.linalg.solve(L, g + A.T @ lam))
    K = np.block([[H, A.T], [A, np.zeros((ma, ma))]])
    ref = np.linalg.solve(K, np.concatenate([-g, -bvec]))
    assert np.linalg.norm(x - ref[:n]) <= 1e-12 * np.linalg.norm(ref[:n])
    assert np.linalg.norm(lam - ref[n:]) <= 1e-12 * np.linalg.norm(ref[n:])


# ----------------------------------------------------------------- trmm_rlnn

def test_trmm_rlnn_integer_exact():
    """Small integers: every product and partial sum is exact, so the oracle
    must equal the exact integer product B * tril(A) computed in int64."""
    rng = np.random.default_rng(40)
    for m, n in ((1, 1), (5, 9), (17, 33), (40, 40)):
        A = rng.integers(-4, 5, (n, n))
        B = rng.integers(-4, 5, (m, n))
        exact = B.astype(np.int64) @ np.tril(A).astype(np.int64)
        assert np.array_equal(oracle.dtrmm_rlnn(A.astype(float), B.astype(float)), exact.astype(float))
        assert np.array_equal(oracle.dtrmm_rlnn(A.astype(float), B.astype(float), alpha=-2.0),
                              -2.0 * exact.astype(float))


def test_trmm_rlnn_rational_tiny():
    """Against exact rational arithmetic for a 3x4 times 4x4 lower product."""
    rng = np.random.default_rng(41)
    A = rng.uniform(-1, 1, (4, 4))
    B = rng.uniform(-1, 1, (3, 4))
    alpha = 0.75
    Af, Bf = _frac_mat(A), _frac_mat(B)
    D = oracle.dtrmm_rlnn(A, B, alpha)
    for i in range(3):
        for j in range(4):
            e = Fraction(alpha) * sum(Bf[i][k] * Af[k][j] for k in range(j, 4))
            assert abs(float(Fraction(D[i, j]) - e)) <= 4e-16 * (1 + abs(float(e)))


def test_trmm_rlnn_reads_only_lower_and_special_cases():
    rng = np.random.default_rng(42)
    A = np.tril(rng.integers(-3, 4, (7, 7)).astype(float))
    B = rng.integers(-3, 4, (5, 7)).astype(float)
    A2 = A.copy()
    A2[np.triu_indices(7, 1)] = np.nan
    assert np.array_equal(oracle.dtrmm_rlnn(A2, B), oracle.dtrmm_rlnn(A, B))
    # identity and diagonal factors scale the columns of B
    assert np.array_equal(oracle.dtrmm_rlnn(np.eye(7), B, alpha=3.0), 3.0 * B)
    d = np.arange(1.0, 8.0)
    assert np.array_equal(oracle.dtrmm_rlnn(np.diag(d), B), B * d)
    # the last column of D only sees the last column of B
    assert np.array_equal(oracle.dtrmm_rlnn(A, B)[:, 6], B[:, 6] * A[6, 6])


# ----------------------------------------------------------------- trsm_rltn

def test_trsm_rltn_integer_recovery():
    L, _ = synth.small_integer_factor(11, seed=13)
    rng = np.random.default_rng(14)
    X = rng.integers(-5, 6, (6, 11)).astype(float)
    B = X @ L.T
    assert np.array_equal(oracle.dtrsm_rltn(L, B), X)
    assert np.array_equal(oracle.dtrsm_rltn(L, 2.0 * B, alpha=0.5), X)


def test_trsm_rltn_rational_tiny():
    """Against exact rational forward substitution for a 3x3 lower L."""
    rng = np.random.default_rng(15)
    L = np.tril(rng.uniform(-1, 1, (3, 3))) + 2 * np.eye(3)
    B = rng.uniform(-1, 1, (2, 3))
    alpha = 1.5
    Lf, Bf = _frac_mat(L), _frac_mat(B)
    X = oracle.dtrsm_rltn(L, B, alpha)
    for i in range(2):
        x = []
        for j in range(3):
            x.append((Fraction(alpha) * Bf[i][j] - sum(x[k] * Lf[j][k] for k in range(j))) / Lf[j][j])
        for j in range(3):
            assert abs(float(Fraction(X[i, j]) - x[j])) <= 1e-15 * max(1.0, abs(float(x[j])))


def test_trsm_rltn_reads_only_lower():
    L, _ = synth.small_integer_factor(6, seed=16)
    L2 = L.copy()
    L2[np.triu_indices(6, 1)] = np.nan
    X = np.arange(12.0).reshape(2, 6)
    assert np.array_equal(oracle.dtrsm_rltn(L2, X @ L.T), X)


# ----------------------------------------------------------------- syrk_potrf

def test_syrk_potrf_exact():
    L, LL = synth.small_integer_factor(20, seed=17)
    rng = np.random.default_rng(18)
    A = rng.integers(-2, 3, (20, 9)).astype(float)
    B = rng.integers(-2, 3, (20, 9)).astype(float)
    S = A @ B.T
    C = LL - np.tril(S) - np.tril(S, -1).T  # lower part of C + A B^T equals L L^T
    D, dA, info = oracle.dsyrk_dpotrf_ln(A, B, C)
    assert info == 0 and np.array_equal(D, L) and np.array_equal(dA, 1.0 / np.diag(L))


# ----------------------------------------------------------------- potrs / symv / berr

def test_potrs_golden_and_exact():
    g = _read_fixture("chol_4x4.txt")
    L = np.array(g["L"], dtype=float)
    A = np.array(g["A"], dtype=float)
    x = np.array(g["x"][0], dtype=float)
    b = np.array(g["b"][0], dtype=float)
    assert np.array_equal(A @ x, b)
    assert np.array_equal(oracle.dpotrs_l(L, b)[:, 0], x)
    L2, _ = synth.small_integer_factor(30, seed=19)
    X = np.random.default_rng(20).integers(-4, 5, (30, 3)).astype(float)
    assert np.array_equal(oracle.dpotrs_l(L2, (L2 @ L2.T) @ X), X)


def test_symv_and_berr_closed_forms():
    g = _read_fixture("chol_4x4.txt")
    A = np.array(g["A"], dtype=float)
    x = np.array(g["x"][0], dtype=float)
    b = np.array(g["b"][0], dtype=float)
    Al = np.tril(A)  # only the lower triangle is read
    assert np.array_equal(oracle.dsymv_l(Al, x, b, -1.0, 1.0), np.zeros(4))
    assert oracle.berr(Al, x, b) == 0.0
    # A = I, x = b + delta e_0: eta = delta / (||x||_inf + ||b||_inf)
    bb = np.array([1.0, -2.0, 0.5])
    xx = bb.copy()
    xx[0] += 0.25
    assert oracle.berr(np.eye(3), xx, bb) == pytest.approx(0.25 / (2.0 + 2.0), rel=1e-15)
    # a NaN anywhere makes the norm, and so eta, NaN (never a pass)
    for k in range(3):
        xn = xx.copy()
        xn[k] = np.nan
        assert np.isnan(oracle.berr(np.eye(3), xn, bb))


# ----------------------------------------------------------------- Riccati

def test_riccati_scalar_golden():
    g = _read_fixture("riccati_scalar.txt")
    a, b, q, r, pn = (float(g[k][0][0]) for k in ("a", "b", "q", "r", "PN"))
    N = int(g["N"][0][0])
    F, info = oracle.ric_trf(np.array([[a]]), np.array([[b]]), np.array([[q]]), np.array([[r]]), np.array([[pn]]), N)
    assert info == 0
    for n_s, lam2, llam, pn_s in g["S"]:
        n = int(n_s)
        Fn = F[n]
        assert Fn[0, 0] ** 2 == pytest.approx(float(Fraction(lam2)), rel=4 * U)
        assert Fn[1, 0] * Fn[0, 0] == pytest.approx(float(Fraction(llam)), rel=8 * U)
        assert Fn[1, 1] ** 2 == pytest.approx(float(Fraction(pn_s)), rel=16 * U)
        assert Fn[0, 1] == 0.0
    # stage 1 in closed form: Lambda = 2, L = 3, Lc = 2 (to a few ulps, since
    # Lc_2 = sqrt(3) is rounded)
    assert np.allclose(F[1], [[2.0, 0.0], [3.0, 2.0]], rtol=8 * U, atol=0)


def test_riccati_closed_form_no_input():
    """B = 0, A = I, Q = I, P_N = I: P_n = (N - n + 1) I, Lc_n = sqrt(N-n+1) I,
    Lambda_n = chol(R), L_n = 0."""
    nx, nu, N = 5, 3, 6
    R = np.diag([0.25, 4.0, 1.0])
    F, info = oracle.ric_trf(np.eye(nx), np.zeros((nx, nu)), np.eye(nx), R, np.eye(nx), N)
    assert info == 0
    for n in range(N):
        assert np.array_equal(F[n][:nu, :nu], np.diag([0.5, 2.0, 1.0]))
        assert np.count_nonzero(F[n][nu:, :nu]) == 0
        # sqrt(k)^2 is rounded, so each stage may move the result by an ulp
        Lc = F[n][nu:, nu:]
        assert np.count_nonzero(Lc - np.diag(np.diag(Lc))) == 0
        assert np.allclose(np.diag(Lc), np.sqrt(N - n + 1.0), rtol=4 * N * U, atol=0)


def _dense_kkt_lq(A, B, Q, R, PN, b, r, q, x0):
    """Solution (u, x) of the linear-quadratic problem from its full KKT
    system, assembled and solved densely (numpy LU): variables
    z = [u_0, x_1, u_1, x_2, ..., u_{N-1}, x_N], one multiplier per dynamics
    equation x_{n+1} - A x_n - B u_n = b_n."""
    nx, nu = B.shape
    N = b.shape[0]
    nz = N * (nu + nx)
    H = np.zeros((nz, nz))
    g = np.zeros(nz)
    G = np.zeros((N * nx, nz))
    h = np.zeros(N * nx)
    iu = lambda n: n * (nu + nx)            # noqa: E731
    ix = lambda n: (n - 1) * (nu + nx) + nu  # noqa: E731  (x_n for n >= 1)
    for n in range(N):
        H[iu(n):iu(n) + nu, iu(n):iu(n) + nu] = R
        g[iu(n):iu(n) + nu] = r[n]
        if n >= 1:
            H[ix(n):ix(n) + nx, ix(n):ix(n) + nx] = Q
            g[ix(n):ix(n) + nx] = q[n]
    H[ix(N):ix(N) + nx, ix(N):ix(N) + nx] = PN
    g[ix(N):ix(N) + nx] = q[N]
    for n in range(N):
        rows = slice(n * nx, (n + 1) * nx)
        G[rows, ix(n + 1):ix(n + 1) + nx] = np.eye(nx)
        G[rows, iu(n):iu(n) + nu] = -B
        if n >= 1:
            G[rows, ix(n):ix(n) + nx] = -A
            h[rows] = b[n]
        else:
            h[rows] = b[0] + A @ x0
    K = np.block([[H, G.T], [G, np.zeros((N * nx, N * nx))]])
    sol = np.linalg.solve(K, np.concatenate([-g, h]))
    z = sol[:nz]
    u = np.array([z[iu(n):iu(n) + nu] for n in range(N)])
    x = np.array([x0] + [z[ix(n):ix(n) + nx] for n in range(1, N + 1)])
    return u, x


@pytest.mark.parametrize("nx,nu,N", [(1, 1, 1), (3, 2, 4), (5, 3, 7), (32, 8, 20)])
def test_riccati_solve_matches_dense_kkt(nx, nu, N):
    """The backward/forward substitution on the stage factors gives the same
    controls and states as the dense KKT solve of the whole problem."""
    rng = np.random.default_rng(nx * 10 + N)
    A = np.eye(nx) + 0.1 * rng.standard_normal((nx, nx))
    B = rng.standard_normal((nx, nu)) / 2
    G = rng.standard_normal((nx, nx))
    Q = G @ G.T / nx + np.eye(nx)
    R = 0.5 * np.eye(nu) + 0.1 * np.ones((nu, nu))
    PN = 2.0 * np.eye(nx)
    b, r, q = rng.standard_normal((N, nx)), rng.standard_normal((N, nu)), rng.standard_normal((N + 1, nx))
    x0 = rng.standard_normal(nx)
    F, info = oracle.ric_trf(A, B, Q, R, PN, N)
    assert info == 0
    u, x = oracle.ric_trs(A, B, PN, F, b, r, q, x0)
    ud, xd = _dense_kkt_lq(A, B, Q, R, PN, b, r, q, x0)
    assert np.linalg.norm(u - ud) <= 1e-10 * np.linalg.norm(ud)
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
    # the dynamics hold exactly as computed (same order of operations)
    for n in range(N):
        assert np.allclose(x[n + 1], A @ x[n] + B @ u[n] + b[n], rtol=0, atol=1e-12 * (1 + np.abs(x[n + 1]).max()))


def test_riccati_solve_scalar_closed_form():
    """One state, one input, one stage, by hand: minimizing
    1/2 R u^2 + r u + 1/2 P (a x0 + c u + d)^2 + q1 (a x0 + c u + d)
    over u gives u = -(r + c (P (a x0 + d) + q1)) / (R + c^2 P)."""
    a, c, d, R, r, P, q1, x0 = 0.9, 0.5, 0.2, 0.3, -0.4, 2.0, 0.7, 1.5
    F, info = oracle.ric_trf(np.array([[a]]), np.array([[c]]), np.array([[1.0]]), np.array([[R]]),
                             np.array([[P]]), 1)
    u, x = oracle.ric_trs(np.array([[a]]), np.array([[c]]), np.array([[P]]), F, np.array([[d]]),
                          np.array([[r]]), np.array([[0.3], [q1]]), np.array([x0]))
    ue = -(r + c * (P * (a * x0 + d) + q1)) / (R + c * c * P)
    assert abs(u[0, 0] - ue) <= 1e-15 * 4
    assert abs(x[1, 0] - (a * x0 + c * ue + d)) <= 1e-15 * 8


def test_riccati_matches_classical_form():
    """Square-root recursion vs the classical Riccati difference equation with
    explicit P (numpy, independent algorithm)."""
    d = synth.riccati_batch(2, seed=3, nx=6, nu=2)
    for s in range(2):
        A, B, Q, R, PN = (d[k][s] for k in ("A", "B", "Q", "R", "PN"))
        N = 7
        F, info = oracle.ric_trf(A, B, Q, R, PN, N)
        assert info == 0
        P = PN.copy()
        nu = B.shape[1]
        for n in range(N - 1, -1, -1):
            S = R + B.T @ P @ B
            K = np.linalg.solve(S, B.T @ P @ A)
            Pn = Q + A.T @ P @ A - A.T @ P @ B @ K
            Lc = F[n][nu:, nu:]
            Lam = F[n][:nu, :nu]
            assert np.allclose(Lc @ Lc.T, Pn, rtol=1e-12, atol=1e-12)
            assert np.allclose(Lam @ Lam.T, S, rtol=1e-12, atol=1e-12)
            P = 0.5 * (Pn + Pn.T)


# ----------------------------------------------------------------- mixed precision

def test_single_precision_gemm_syrk_pins():
    """Small integers are exact in float: sgemm_nt and ssyrk_ln equal the
    int64 products; on general data they are the double-precision routines'
    results rounded step by step (within n float ulps)."""
    rng = np.random.default_rng(95)
    A, B, C = (rng.integers(-4, 5, s) for s in ((9, 7), (5, 7), (9, 5)))
    exact = 2 * (A.astype(np.int64) @ B.T.astype(np.int64)) - C
    assert np.array_equal(oracle.sgemm_nt(A, B, C, 2.0, -1.0), exact.astype(np.float32))
    S = rng.integers(-4, 5, (9, 9))
    ex = np.tril(A.astype(np.int64) @ A.T.astype(np.int64) + S)
    assert np.array_equal(oracle.ssyrk_ln(A, A, S), ex.astype(np.float32))
    Af, Bf, Cf = (rng.uniform(-1, 1, s) for s in ((20, 30), (11, 30), (20, 11)))
    D32 = oracle.sgemm_nt(Af, Bf, Cf, 0.5, 1.5).astype(np.float64)
    D64 = oracle.dgemm_nt(Af.astype(np.float32), Bf.astype(np.float32), Cf.astype(np.float32), 0.5, 1.5)
    assert np.abs(D32 - D64).max() <= 30 * 2 ** -24 * (1 + np.abs(D64).max())


def test_spotrf_small_integer_exact_in_fp32():
    L, A = synth.small_integer_factor(24, seed=22)
    D, info = oracle.spotrf_l(A.astype(np.float32))
    assert info == 0 and np.array_equal(D.astype(float), L)


def test_single_precision_binary32_rounding_pins():
    """Hand-derived cases whose binary32 result differs from the FP64 result
    rounded once to binary32, so an oracle that accumulated or multiplied in
    double would fail them (u32 = 2^-24, ties to even):
      * 1 + 2^-24 + 2^-24 summed in float, k ascending: each addition is a
        tie that rounds back to 1, so the sum is 1 (in double: 1 + 2^-23,
        which is a float); with the small terms first the sum is 1 + 2^-23;
      * (1 + 2^-12)^2 = 1 + 2^-11 + 2^-24 rounds (tie, to even) to 1 + 2^-11,
        so -1 + (1 + 2^-12)^2 gives 2^-11 (in double: 2^-11 + 2^-24);
      * Cholesky of [[1, a], [a, 1 + 2^-11 + 2^-22]], a = 1 + 2^-12: the
        pivot 1 + 2^-11 + 2^-22 - fl(a^2) = 2^-22 exactly, L11 = 2^-11
        (in double the pivot is 3 * 2^-24 and L11 = sqrt(3) * 2^-12)."""
    t = 2.0 ** -24
    D = oracle.sgemm_nt(np.array([[1.0, 1.0, 1.0]]), np.array([[1.0, t, t]]), np.zeros((1, 1)))
    assert D[0, 0] == np.float32(1.0)
    D = oracle.sgemm_nt(np.array([[1.0, 1.0, 1.0]]), np.array([[t, t, 1.0]]), np.zeros((1, 1)))
    assert D[0, 0] == np.float32(1.0 + 2.0 ** -23)
    a = 1.0 + 2.0 ** -12
    D = oracle.sgemm_nt(np.array([[a]]), np.array([[a]]), np.array([[-1.0]]))
    assert D[0, 0] == np.float32(2.0 ** -11)
    assert oracle.dgemm_nt(np.array([[a]]), np.array([[a]]), np.array([[-1.0]]))[0, 0] == 2.0 ** -11 + 2.0 ** -24
    # syrk_ln: the same accumulation in the (1,0) entry; the upper part stays 0
    A = np.array([[1.0, 1.0, 1.0], [1.0, t, t]])
    D = oracle.ssyrk_ln(A, A, np.zeros((2, 2)))
    assert D[1, 0] == np.float32(1.0) and D[0, 0] == np.float32(3.0) and D[0, 1] == 0.0
    # potrf_l
    C = np.array([[1.0, a], [a, 1.0 + 2.0 ** -11 + 2.0 ** -22]])
    L32, info = oracle.spotrf_l(C)
    assert info == 0
    assert L32[0, 0] == 1.0 and L32[1, 0] == np.float32(a) and L32[1, 1] == np.float32(2.0 ** -11)
    L64 = oracle.dpotrf_l(C)[0]
    assert abs(L64[1, 1] - np.sqrt(3.0) * 2.0 ** -12) <= 2.0 ** -60


def test_uniform_chunk_drivers_match_single_calls():
    """The uniform-order OpenMP drivers used by the full-size parity checks
    are the per-instance routines, bit for bit."""
    ns, mats, rhs = synth.conditioned_batch(6, 1e3, seed=40, nrhs=3, sizes=[37] * 6)
    A, B = np.stack(mats), np.stack(rhs)
    A[2, 5, 5] = -1.0  # a failing factorization
    L, X, dA, info, used = oracle.batch_dposv_uniform(A, B, nthreads=3)
    assert used >= 1
    for i in range(6):
        Lr, dAr, ir = oracle.dpotrf_l(A[i])
        assert info[i] == ir and np.array_equal(L[i], Lr) and np.array_equal(dA[i], dAr)
        if ir == 0:
            assert np.array_equal(X[i], oracle.dpotrs_l(Lr, B[i]))
        else:
            assert ir == 6 and not X[i].any()
    eta, _ = oracle.batch_berr_uniform(A, X, B, nthreads=2)
    for i in (0, 1, 3):
        assert eta[i] == max(oracle.berr(A[i], X[i][:, c], B[i][:, c]) for c in range(3))
    Xn = X.copy()
    Xn[4, 7, 1] = np.nan
    assert np.isnan(oracle.batch_berr_uniform(A, Xn, B)[0][4])


def test_fl16_matches_ieee_binary16():
    """The binary16 rounding against numpy's float16 conversion (an
    independent implementation of the same IEEE definition)."""
    rng = np.random.default_rng(0)
    xs = np.concatenate([
        rng.standard_normal(4000) * 10.0 ** rng.integers(-9, 6, 4000),
        [0.0, -0.0, 1.0, 65504.0, 65519.0, 65520.0, -65520.0, 7e4, 2.0 ** -14, 2.0 ** -24,
         2.0 ** -25, 3 * 2.0 ** -26, 2.0 ** -26, 1.0 + 2.0 ** -11, 1.0 + 3 * 2.0 ** -11, 2049.0, 2051.0],
    ]).astype(np.float32)
    for x in xs:
        with np.errstate(over="ignore"):
            want = float(np.float32(x).astype(np.float16))
        got = oracle.fl16(x)
        assert got == want or (np.isinf(got) and np.isinf(want) and np.sign(got) == np.sign(want)), (x, got, want)
    assert np.isnan(oracle.fl16(np.nan))


def test_mixed_scale_powers_of_two():
    rng = np.random.default_rng(1)
    d = 10.0 ** rng.uniform(-300, 300, 200)
    A = np.diag(np.concatenate([d, [0.0, -3.0, 1.0, 2.0, 0.5]]))
    s = oracle.mixed_scale(A)
    m, e = np.frexp(s)
    assert np.all(m == 0.5)  # exact powers of two
    t = s[:200] ** 2 * d
    assert np.all((t >= 0.5) & (t < 2.0))
    assert list(s[200:]) == [1.0, 1.0, 1.0, 0.5, 1.0]


@pytest.mark.parametrize("prec", [1, 2])
def test_mixed_factor_exact_on_integer_factor(prec):
    """A = L L^T with a small-integer L: the factor of S A S is S L exactly."""
    L, A = synth.structured_integer_factor(70, seed=3)
    L32, s, info = oracle.mixed_factor(A, prec)
    assert info == 0
    assert np.array_equal(L32.astype(np.float64), s[:, None] * L)


@pytest.mark.parametrize("n", [50, 200])
def test_mixed_factor_backward_error(n):
    """Backward error of the low-precision factors against the unit roundoff
    of each format: FP32 within c n u32; FP16 operands within c n u16 and
    visibly above the FP32 level (the half rounding is really applied)."""
    ns, mats, rhs = synth.conditioned_batch(1, 1e2, seed=4, sizes=[n])
    A = mats[0]
    res = {}
    for prec in (1, 2):
        L32, s, info = oracle.mixed_factor(A, prec)
        assert info == 0
        As = s[:, None] * A * s[None, :]
        L = L32.astype(np.float64)
        res[prec] = np.linalg.norm(L @ L.T - As) / np.linalg.norm(As)
        assert np.all(np.triu(L32, 1) == 0) and np.all(np.diag(L32) > 0)
    assert res[1] < n * 2.0 ** -24
    assert res[2] < n * 2.0 ** -11
    assert res[2] > 10 * res[1]


@pytest.mark.parametrize("cond", [1e2, 1e4, 1e6])
def test_dposv_mixed_reaches_fp64_backward_error(cond):
    ns, mats, rhs = synth.conditioned_batch(1, cond, seed=4, sizes=[40])
    A, b = mats[0], rhs[0][:, 0]
    x, it, eta = oracle.dposv_mixed(A, b, tol=1e-12, max_iter=30)
    assert it >= 0 and eta <= 1e-12
    assert eta == oracle.berr(A, x, b)
    xr = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xr) / np.linalg.norm(xr) <= 1e-12 * cond * 40
    if cond >= 1e4:
        assert it >= 1  # FP32 alone cannot reach 1e-12


def test_dposv_mixed_non_spd():
    A = np.diag([1.0, -1.0, 2.0])
    x, it, eta = oracle.dposv_mixed(A, np.ones(3))
    assert it == -1


def test_dposv_mixed_fp16_by_condition():
    """FP16 operands with scaling: converge at cond 1e2 (more corrections
    than FP32), and the factorization breaks down at cond 1e6."""
    ns, mats, rhs = synth.conditioned_batch(2, 1e2, seed=4, sizes=[60, 200])
    for A, b in zip(mats, rhs):
        x, it16, eta = oracle.dposv_mixed(A, b[:, 0], prec=2, max_iter=30)
        _, it32, _ = oracle.dposv_mixed(A, b[:, 0], prec=1, max_iter=30)
        assert 0 < it32 < it16 and eta <= 1e-12
        assert eta == oracle.berr(A, x, b[:, 0])
    ns, mats, rhs = synth.conditioned_batch(1, 1e6, seed=4, sizes=[200])
    assert oracle.dposv_mixed(mats[0], rhs[0][:, 0], prec=2)[1] == -1


def test_dposv_mixed_exact_and_give_up():
    """Exact data: x0 is exact, no correction.  max_iter = 0 on a system
    that needs corrections: gives up with the backward error of x0."""
    L, A = synth.structured_integer_factor(40, seed=5)
    xt = np.random.default_rng(2).integers(-3, 4, 40).astype(float)
    for prec in (1, 2):
        x, it, eta = oracle.dposv_mixed(A, A @ xt, prec=prec)
        assert it == 0 and eta == 0.0 and np.array_equal(x, xt)
    ns, mats, rhs = synth.conditioned_batch(1, 1e4, seed=4, sizes=[60])
    x, it, eta = oracle.dposv_mixed(mats[0], rhs[0][:, 0], max_iter=0)
    assert it == -2 and eta > 1e-12 and eta == oracle.berr(mats[0], x, rhs[0][:, 0])


def test_batch_dposv_mixed_matches_single():
    ns, mats, rhs = synth.conditioned_batch(4, 1e3, seed=4, nrhs=3, sizes=[17, 64, 33, 90])
    Xs, iters, eta, used = oracle.batch_dposv_mixed(mats, rhs, nthreads=2)
    for i in range(4):
        its, etas = [], []
        for c in range(3):
            x, it, e = oracle.dposv_mixed(mats[i], rhs[i][:, c])
            assert np.array_equal(x, Xs[i][:, c])
            its.append(it)
            etas.append(e)
        assert iters[i] == max(its) and eta[i] == max(etas)


# ----------------------------------------------------------------- batched drivers

def test_batch_drivers_match_single():
    d = synth.uniform_batch(5, n=20, k=12, nrhs=3)
    L, X, dA, info, used = oracle.batch_syrk_potrf_trsm(d["Q"], d["B"], d["RHS"], nthreads=2)
    assert used >= 1 and np.all(info == 0)
    for b in range(5):
        Lb, db, ib = oracle.dsyrk_dpotrf_ln(d["B"][b], d["B"][b], d["Q"][b])
        assert np.array_equal(L[b], Lb) and np.array_equal(dA[b], db)
        assert np.array_equal(X[b], oracle.dtrsm_rltn(Lb, d["RHS"][b]))
    ns, mats, rhs = synth.uneven_batch(6, step=8, nmax=40)
    Ls, xs, ds, info, _ = oracle.batch_potrf_potrs(mats, rhs, nthreads=2)
    for i in range(6):
        Li, di, ii = oracle.dpotrf_l(mats[i])
        assert np.array_equal(Ls[i], Li) and np.array_equal(xs[i], oracle.dpotrs_l(Li, rhs[i])[:, 0])
    r = synth.riccati_batch(3, nx=4, nu=2)
    F, info, _ = oracle.batch_ric_trf(r["A"], r["B"], r["Q"], r["R"], r["PN"], 5, nthreads=2)
    for b in range(3):
        Fb, ib = oracle.ric_trf(r["A"][b], r["B"][b], r["Q"][b], r["R"][b], r["PN"][b], 5)
        assert np.array_equal(F[b], Fb)
