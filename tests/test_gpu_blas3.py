"""GPU parity of the single-instance and uniform-batch routines against the
CPU oracle, element by element, through the C ABI.  Operands live in
panel-major device buffers filled by the library's pack routine; the pack and
unpack kernels are themselves checked bit for bit against the independent
numpy decoder of the panel layout."""
import numpy as np
import pytest

import oracle
import synth
from _util import TOL, assert_parity, note, rel
from oracle import panel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1704_02457_amd as p  # noqa: E402

DEV = torch.device("cuda:0")
SENT = 7.25  # sentinel for elements that must not be written


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def mat(A):
    """Pack a host (m, n) array into a new DMat."""
    return p.pack(dev(A))


def host(sA):
    torch.cuda.synchronize()
    return p.unpack(sA).cpu().numpy()


def sentinel_mat(m, n):
    return mat(np.full((m, n), SENT))


# ------------------------------------------------------------------ pack / unpack

@pytest.mark.parametrize("m,n", [(1, 1), (16, 16), (17, 5), (64, 64), (130, 37)])
def test_pack_matches_independent_decoder(m, n):
    note("pack", m, n)
    rng = np.random.default_rng(m * 100 + n)
    A = rng.standard_normal((m, n))
    s = mat(A)
    torch.cuda.synchronize()
    raw = s.panels().cpu().numpy()
    ref = panel.unpack(raw, m, n, s.s.cn, 16)
    assert np.array_equal(ref, A)
    assert np.array_equal(host(s), A)
    # sub-matrix pack at an offset not aligned to a panel
    big = sentinel_mat(m + 21, n + 3)
    p.pack(dev(A), out=big, bi=21, bj=3)
    full = host(big)
    assert np.array_equal(full[21:, 3:], A)
    mask = np.ones_like(full, dtype=bool)
    mask[21:, 3:] = False
    assert np.all(full[mask] == SENT)


# ------------------------------------------------------------------ gemm_nt

GEMM_CASES = [(64, 64, 64), (1, 1, 1), (17, 33, 5), (63, 65, 31), (100, 40, 130), (16, 16, 0)]
OFFS = [(0,) * 8, (3, 5, 17, 2, 1, 7, 9, 11)]


@pytest.mark.parametrize("m,n,k", GEMM_CASES)
@pytest.mark.parametrize("offs", OFFS)
def test_dgemm_nt(m, n, k, offs):
    note("gemm_nt", m, n, k, offs)
    ai, aj, bi, bj, ci, cj, di, dj = offs
    rng = np.random.default_rng(m + 3 * n + 7 * k)
    A = rng.uniform(-1, 1, (m, k))
    B = rng.uniform(-1, 1, (n, k))
    C = rng.uniform(-1, 1, (m, n))
    alpha, beta = 0.75, -1.5
    sA = sentinel_mat(ai + m, aj + k)
    sB = sentinel_mat(bi + n, bj + k)
    sC = sentinel_mat(ci + m, cj + n)
    sD = sentinel_mat(di + m, dj + n)
    p.pack(dev(A), sA, ai, aj) if m * k else None
    p.pack(dev(B), sB, bi, bj) if n * k else None
    p.pack(dev(C), sC, ci, cj)
    p.blasfeo_dgemm_nt(m, n, k, alpha, sA, ai, aj, sB, bi, bj, beta, sC, ci, cj, sD, di, dj)
    D = host(sD)
    ref = oracle.dgemm_nt(A, B, C, alpha, beta)
    assert_parity(D[di:, dj:], ref, max(m, n, k), "gemm_nt")
    mask = np.ones_like(D, dtype=bool)
    mask[di:, dj:] = False
    assert np.all(D[mask] == SENT)


def test_dgemm_nt_integer_exact_and_in_place():
    note("gemm_nt exact/in-place")
    rng = np.random.default_rng(3)
    A = rng.integers(-8, 9, (64, 64)).astype(float)
    B = rng.integers(-8, 9, (64, 64)).astype(float)
    C = rng.integers(-8, 9, (64, 64)).astype(float)
    sA, sB, sC = mat(A), mat(B), mat(C)
    p.blasfeo_dgemm_nt(64, 64, 64, 1.0, sA, 0, 0, sB, 0, 0, 1.0, sC, 0, 0, sC, 0, 0)  # C == D
    assert np.array_equal(host(sC), C + A @ B.T)


@pytest.mark.parametrize("m,n,k", GEMM_CASES)
@pytest.mark.parametrize("offs", OFFS)
def test_dgemm_nn(m, n, k, offs):
    """D = alpha*A*B + beta*C with B k-by-n read across panels: element-wise
    against the oracle on the gemm_nt cases and offsets."""
    note("gemm_nn", m, n, k, offs)
    ai, aj, bi, bj, ci, cj, di, dj = offs
    rng = np.random.default_rng(m + 5 * n + 11 * k)
    A = rng.uniform(-1, 1, (m, k))
    B = rng.uniform(-1, 1, (k, n))
    C = rng.uniform(-1, 1, (m, n))
    alpha, beta = -0.5, 2.0
    sA = sentinel_mat(ai + m, aj + k)
    sB = sentinel_mat(bi + k, bj + n)
    sC = sentinel_mat(ci + m, cj + n)
    sD = sentinel_mat(di + m, dj + n)
    p.pack(dev(A), sA, ai, aj) if m * k else None
    p.pack(dev(B), sB, bi, bj) if n * k else None
    p.pack(dev(C), sC, ci, cj)
    p.blasfeo_dgemm_nn(m, n, k, alpha, sA, ai, aj, sB, bi, bj, beta, sC, ci, cj, sD, di, dj)
    D = host(sD)
    assert_parity(D[di:, dj:], oracle.dgemm_nn(A, B, C, alpha, beta), max(m, n, k), "gemm_nn")
    mask = np.ones_like(D, dtype=bool)
    mask[di:, dj:] = False
    assert np.all(D[mask] == SENT)


def test_dgemm_nn_exact_in_place_and_batched():
    note("gemm_nn exact/in-place/batched")
    rng = np.random.default_rng(31)
    A = rng.integers(-8, 9, (64, 48)).astype(float)
    B = rng.integers(-8, 9, (48, 64)).astype(float)
    C = rng.integers(-8, 9, (64, 64)).astype(float)
    sA, sB, sC = mat(A), mat(B), mat(C)
    p.blasfeo_dgemm_nn(64, 64, 48, 1.0, sA, 0, 0, sB, 0, 0, 1.0, sC, 0, 0, sC, 0, 0)  # C == D
    assert np.array_equal(host(sC), C + A @ B)
    batch, m, n, k = 33, 20, 36, 12
    A, B, C = rng.uniform(-1, 1, (batch, m, k)), rng.uniform(-1, 1, (batch, k, n)), rng.uniform(-1, 1, (batch, m, n))
    sA, sB, sC = p.pack_batch(dev(A)), p.pack_batch(dev(B)), p.pack_batch(dev(C))
    sD = p.DMatBatch(batch, m, n)
    p.blasfeo_hip_dgemm_nn_batched(batch, m, n, k, 2.0, sA, 0, 0, sB, 0, 0, 0.5, sC, 0, 0, sD, 0, 0)
    torch.cuda.synchronize()
    D = p.unpack_batch(sD).cpu().numpy()
    for b in range(batch):
        assert_parity(D[b], oracle.dgemm_nn(A[b], B[b], C[b], 2.0, 0.5), k, f"gemm_nn b={b}")


def test_workload_single_gemm_then_potrf():
    """The single-instance workload: gemm_nt 64^3 then potrf_l of M M^T + 64 I."""
    note("single workload")
    s = synth.single(seed=0, n=64)
    sA, sB, sC, sD = mat(s["A"]), mat(s["B"]), mat(s["C"]), p.DMat(64, 64)
    p.blasfeo_dgemm_nt(64, 64, 64, 1.0, sA, 0, 0, sB, 0, 0, 1.0, sC, 0, 0, sD, 0, 0)
    assert_parity(host(sD), oracle.dgemm_nt(s["A"], s["B"], s["C"]), 64, "gemm")
    sS, sL = mat(s["S"]), sentinel_mat(64, 64)
    info = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    p.blasfeo_hip_dpotrf_l_info(64, sS, 0, 0, sL, 0, 0, info)
    Lg = host(sL)
    Lr, dAr, inf = oracle.dpotrf_l(s["S"])
    assert int(info.item()) == 0 and inf == 0
    assert_parity(np.tril(Lg), Lr, 64, "potrf")
    assert np.all(np.triu(Lg, 1)[np.triu_indices(64, 1)] == SENT)
    assert_parity(sL.dA()[:64].cpu().numpy(), dAr, 64, "dA")
    assert sL.s.use_dA == 1


# ------------------------------------------------------------------ syrk_ln

@pytest.mark.parametrize("m,k", [(64, 64), (1, 1), (17, 5), (40, 32), (100, 70)])
@pytest.mark.parametrize("off", [0, 5])
def test_dsyrk_ln(m, k, off):
    note("syrk_ln", m, k, off)
    rng = np.random.default_rng(m * 7 + k)
    A, B, C = rng.uniform(-1, 1, (m, k)), rng.uniform(-1, 1, (m, k)), rng.uniform(-1, 1, (m, m))
    sA, sB = sentinel_mat(m + off, k + off), sentinel_mat(m + 2 * off, k)
    sC, sD = sentinel_mat(m + off, m + off), sentinel_mat(m + off, m + 3 * off)
    p.pack(dev(A), sA, off, off)
    p.pack(dev(B), sB, 2 * off, 0)
    p.pack(dev(C), sC, off, off)
    p.blasfeo_dsyrk_ln(m, k, 1.5, sA, off, off, sB, 2 * off, 0, 0.5, sC, off, off, sD, off, 3 * off)
    D = host(sD)
    sub = D[off:, 3 * off:]
    ref = oracle.dsyrk_ln(A, B, C, 1.5, 0.5)
    assert_parity(np.tril(sub), ref, max(m, k), "syrk")
    assert np.all(sub[np.triu_indices(m, 1)] == SENT)


# ------------------------------------------------------------------ trmm_rlnn

@pytest.mark.parametrize("m,n", [(40, 32), (1, 1), (37, 50), (100, 17), (16, 64), (20, 130)])
@pytest.mark.parametrize("offs", [(0, 0, 0, 0, 0, 0), (5, 3, 2, 9, 17, 1)])
def test_dtrmm_rlnn(m, n, offs):
    """D = alpha*B*A, A lower: element-wise parity with the oracle on ragged
    sizes and unaligned offsets; the strictly upper part of A is poisoned and
    every element of D outside the sub-matrix keeps its sentinel."""
    note("trmm_rlnn", m, n, offs)
    ai, aj, bi, bj, di, dj = offs
    rng = np.random.default_rng(m * 13 + n)
    A = np.tril(rng.uniform(-1, 1, (n, n)))
    B = rng.uniform(-1, 1, (m, n))
    sA = sentinel_mat(ai + n, aj + n)
    sB, sD = sentinel_mat(bi + m, bj + n), sentinel_mat(di + m, dj + n)
    p.pack(dev(A + np.triu(np.full((n, n), np.nan), 1)), sA, ai, aj)
    p.pack(dev(B), sB, bi, bj)
    p.blasfeo_dtrmm_rlnn(m, n, -1.5, sA, ai, aj, sB, bi, bj, sD, di, dj)
    D = host(sD)
    assert_parity(D[di:, dj:], oracle.dtrmm_rlnn(A, B, -1.5), n, "trmm")
    outside = np.ones_like(D, dtype=bool)
    outside[di:, dj:] = False
    assert np.all(D[outside] == SENT)


def test_dtrmm_rlnn_integer_exact_and_overlap_rejected():
    note("trmm exact")
    rng = np.random.default_rng(7)
    A = np.tril(rng.integers(-3, 4, (48, 48))).astype(float)
    B = rng.integers(-3, 4, (19, 48)).astype(float)
    sA, sB, sD = mat(A), mat(B), p.DMat(19, 48)
    p.blasfeo_dtrmm_rlnn(19, 48, 2.0, sA, 0, 0, sB, 0, 0, sD, 0, 0)
    assert np.array_equal(host(sD), 2.0 * (B @ A))
    with pytest.raises(p.HipError):
        p.blasfeo_dtrmm_rlnn(19, 48, 1.0, sA, 0, 0, sB, 0, 0, sB, 0, 0)  # D is B
    assert np.array_equal(host(sB), B)


def test_dtrmm_rlnn_batched_riccati_shape():
    """The C step of the Riccati workload as a uniform batch: 4096 x
    (B 40x32, A 32x32 lower); the output of every instance against the
    exact-in-FP64 product of numpy on the host and 64 sampled instances
    against the oracle."""
    note("trmm batched 4096 x (40, 32)")
    batch, m, n = 4096, 40, 32
    rng = np.random.default_rng(11)
    A = np.tril(rng.uniform(-1, 1, (batch, n, n)))
    B = rng.uniform(-1, 1, (batch, m, n))
    sA, sB, sD = p.pack_batch(dev(A)), p.pack_batch(dev(B)), p.DMatBatch(batch, m, n)
    p.blasfeo_hip_dtrmm_rlnn_batched(batch, m, n, 1.0, sA, 0, 0, sB, 0, 0, sD, 0, 0)
    torch.cuda.synchronize()
    D = p.unpack_batch(sD).cpu().numpy()
    ref = B @ A
    err = np.linalg.norm(D - ref, axis=(1, 2)) / np.linalg.norm(ref, axis=(1, 2))
    assert float(err.max()) <= 1e-13 * n
    for b in rng.choice(batch, 64, replace=False):
        assert_parity(D[b], oracle.dtrmm_rlnn(A[b], B[b]), n, f"trmm b={b}")
    with pytest.raises(p.HipError):
        p.blasfeo_hip_dtrmm_rlnn_batched(batch, m, n, 1.0, sA, 0, 0, sB, 0, 0, sB, 0, 0)


# ------------------------------------------------------------------ trsm_rltn

@pytest.mark.parametrize("m,n", [(16, 64), (1, 1), (37, 50), (100, 17), (20, 130)])
@pytest.mark.parametrize("offs", [(0, 0, 0, 0, 0, 0), (5, 3, 2, 9, 17, 1)])
def test_dtrsm_rltn(m, n, offs):
    note("trsm_rltn", m, n, offs)
    ai, aj, bi, bj, di, dj = offs
    rng = np.random.default_rng(m * 11 + n)
    G = rng.standard_normal((n, n))
    Lm = np.linalg.cholesky(G @ G.T / n + np.eye(n))
    B = rng.standard_normal((m, n))
    sA = sentinel_mat(ai + n, aj + n)
    sB, sD = sentinel_mat(bi + m, bj + n), sentinel_mat(di + m, dj + n)
    Lpoison = Lm + np.triu(np.full((n, n), np.nan), 1)  # upper part must not be read
    p.pack(dev(Lpoison), sA, ai, aj)
    p.pack(dev(B), sB, bi, bj)
    p.blasfeo_dtrsm_rltn(m, n, 0.5, sA, ai, aj, sB, bi, bj, sD, di, dj)
    D = host(sD)
    assert_parity(D[di:, dj:], oracle.dtrsm_rltn(Lm, B, 0.5), max(m, n), "trsm")


def test_dtrsm_rltn_integer_exact():
    note("trsm exact")
    L, _ = synth.small_integer_factor(48, seed=5)  # diagonal {1, 2, 4}, off-diagonal -3..3
    X = np.random.default_rng(6).integers(-5, 6, (16, 48)).astype(float)
    sL, sB, sD = mat(L), mat(X @ L.T), p.DMat(16, 48)
    p.blasfeo_dtrsm_rltn(16, 48, 1.0, sL, 0, 0, sB, 0, 0, sD, 0, 0)
    assert np.array_equal(host(sD), X)


# ------------------------------------------------------------------ potrf_l / syrk_potrf

@pytest.mark.parametrize("n", [1, 5, 16, 17, 31, 33, 64, 65, 100, 130, 256])
@pytest.mark.parametrize("off", [(0, 0, 0, 0), (5, 3, 17, 2)])
def test_dpotrf_l(n, off):
    note("potrf_l", n, off)
    ci, cj, di, dj = off
    rng = np.random.default_rng(n)
    G = rng.standard_normal((n, n))
    A = G @ G.T + n * np.eye(n)
    Apoison = np.tril(A) + np.triu(np.full((n, n), np.nan), 1)  # only the lower part may be read
    sC, sD = sentinel_mat(ci + n, cj + n), sentinel_mat(di + n, dj + n)
    p.pack(dev(Apoison), sC, ci, cj)
    info = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    p.blasfeo_hip_dpotrf_l_info(n, sC, ci, cj, sD, di, dj, info)
    D = host(sD)[di:, dj:]
    Lr, dAr, inf = oracle.dpotrf_l(A)
    assert int(info.item()) == 0
    assert_parity(np.tril(D), Lr, n, "potrf")
    assert np.all(D[np.triu_indices(n, 1)] == SENT)
    assert_parity(sD.dA()[:n].cpu().numpy(), dAr, n, "dA")
    assert sD.s.use_dA == int(di == 0 and dj == 0)


# ------------------------------------------------------------------ getrf

@pytest.mark.parametrize("m,n", [(1, 1), (6, 6), (32, 32), (30, 17), (17, 30), (32, 5),
                                 (40, 40), (64, 64), (64, 33), (33, 64), (48, 20), (20, 48), (64, 1), (1, 64),
                                 (37, 61), (61, 37)])
@pytest.mark.parametrize("pivot", [True, False])
@pytest.mark.parametrize("off", [(0, 0, 0, 0), (3, 5, 7, 2)])
def test_dgetrf(m, n, pivot, off):
    """LU against the oracle: the same interchanges and the packed L\\U
    element by element; dA = 1/diag(U); sentinels outside D.  Up to order
    32 (the unblocked kernel) the bits are the oracle's; above (one wave,
    panels of 16, MFMA trailing update) the factors agree within the parity
    bound and the GPU's own factors satisfy P C = L U to the same bound."""
    note("getrf", m, n, pivot, off)
    ci, cj, di, dj = off
    rng = np.random.default_rng(m * 3 + n + int(pivot))
    C = rng.standard_normal((m, n))
    if not pivot:  # diagonally dominant so that no pivoting is needed
        C[np.arange(min(m, n)), np.arange(min(m, n))] += 2.0 * n
    sC, sD = sentinel_mat(ci + m, cj + n), sentinel_mat(di + m, dj + n)
    p.pack(dev(C), sC, ci, cj)
    mn = min(m, n)
    ipiv = torch.full((mn,), -1, dtype=torch.int32, device=DEV)
    if pivot:
        p.blasfeo_dgetrf_pivot(m, n, sC, ci, cj, sD, di, dj, ipiv)
    else:
        p.blasfeo_dgetrf_nopivot(m, n, sC, ci, cj, sD, di, dj)
    Dfull = host(sD)
    Dr, ipr, dAr, inf = oracle.dgetrf(C, pivot=pivot)
    assert inf == 0
    if pivot:
        assert np.array_equal(ipiv.cpu().numpy(), ipr)
    assert_parity(Dfull[di:, dj:], Dr, max(m, n), "getrf")
    assert_parity(sD.dA()[:mn].cpu().numpy(), dAr, max(m, n), "dA")
    if max(m, n) <= 32:
        # the kernel performs the oracle's operations in the oracle's order,
        # in IEEE binary64 without contraction on both sides: identical bits
        assert np.array_equal(Dfull[di:, dj:], Dr)
        assert np.array_equal(sD.dA()[:mn].cpu().numpy(), dAr)
    else:
        D = Dfull[di:, dj:]
        L = np.tril(D, -1)[:, :mn] + np.eye(m, mn)
        U = np.triu(D)[:mn, :]
        PC = C.copy()
        if pivot:
            ip = ipiv.cpu().numpy()
            for k in range(mn):
                PC[[k, ip[k]]] = PC[[ip[k], k]]
        assert_parity(L @ U, PC, max(m, n), "P C = L U")
    mask = np.ones_like(Dfull, dtype=bool)
    mask[di:, dj:] = False
    assert np.all(Dfull[mask] == SENT)


@pytest.mark.parametrize("where", [(0, 0), (3, 0), (5, 2)])
def test_dgetrf_nan_pivots_as_oracle(where):
    """A NaN in the pivot column is ranked as the oracle's scan ranks it (kept
    when it sits at the pivot position, never chosen elsewhere): the same
    interchanges, and NaNs in the same places of the factor."""
    note("getrf nan", where)
    rng = np.random.default_rng(31)
    C = rng.standard_normal((9, 7))
    C[where] = np.nan
    sC, sD = mat(C), p.DMat(9, 7)
    ipiv = torch.full((7,), -1, dtype=torch.int32, device=DEV)
    p.blasfeo_dgetrf_pivot(9, 7, sC, 0, 0, sD, 0, 0, ipiv)
    D = host(sD)
    Dr, ipr, dAr, inf = oracle.dgetrf(C, pivot=True)
    assert np.array_equal(ipiv.cpu().numpy(), ipr)
    assert np.array_equal(D, Dr, equal_nan=True)


@pytest.mark.parametrize("where", [(0, 0), (5, 0), (40, 3), (20, 17), (63, 50), (10, 63)])
def test_dgetrf_one_wave_nan_as_oracle(where):
    """Orders 33..64 (one wave, MFMA trailing update): a NaN anywhere gives
    the oracle's interchanges and NaNs in exactly the oracle's places (rows
    finished by earlier panels are not touched by later updates)."""
    note("getrf one-wave nan", where)
    rng = np.random.default_rng(32)
    C = rng.standard_normal((64, 64))
    C[where] = np.nan
    sC, sD = mat(C), p.DMat(64, 64)
    ipiv = torch.full((64,), -1, dtype=torch.int32, device=DEV)
    p.blasfeo_dgetrf_pivot(64, 64, sC, 0, 0, sD, 0, 0, ipiv)
    D = host(sD)
    Dr, ipr, dAr, inf = oracle.dgetrf(C, pivot=True)
    assert np.array_equal(ipiv.cpu().numpy(), ipr), where
    assert np.array_equal(np.isnan(D), np.isnan(Dr)), where
    ok = ~np.isnan(Dr)
    assert_parity(D[ok], Dr[ok], 64, "finite part")


@pytest.mark.parametrize("case", ["exact_tie", "binary32_tie", "tiny_pivot", "huge"])
def test_dgetrf_one_wave_ties_and_extremes(case):
    """Orders 33..64 with pivoting: cases that a panel's first, branch-free
    sweep hands back to the exact sweep -- an exact tie for the largest
    magnitude (the first row wins), two magnitudes equal in binary32 but
    not in binary64 (the larger wins), a pivot below 2^-1000 and entries
    above 2^1000 -- give the oracle's interchanges and factors."""
    note("getrf one-wave ties", case)
    rng = np.random.default_rng(41)
    C = rng.uniform(-1.0, 1.0, (64, 64))
    if case == "exact_tie":
        C[[5, 9, 20], 0] = [3.0, -3.0, 3.0]
        C[[30, 31], 17] = [-50.0, 50.0]
    elif case == "binary32_tie":
        C[3, 0], C[7, 0] = 4.0, -(4.0 + 2.0 ** -38)
        C[40, 20], C[22, 20] = 9.0 + 2.0 ** -35, 9.0
    elif case == "tiny_pivot":
        C[:, 2] *= 2.0 ** -1010
    else:
        C[10:, 40:] *= 2.0 ** 1005
    sC, sD = mat(C), p.DMat(64, 64)
    ipiv = torch.full((64,), -1, dtype=torch.int32, device=DEV)
    p.blasfeo_dgetrf_pivot(64, 64, sC, 0, 0, sD, 0, 0, ipiv)
    D = host(sD)
    Dr, ipr, dAr, inf = oracle.dgetrf(C, pivot=True)
    assert np.array_equal(ipiv.cpu().numpy(), ipr), case
    assert np.all(np.isfinite(D)) and np.all(np.isfinite(Dr))
    sc = np.abs(Dr).max()  # (the Frobenius norm of the huge case overflows)
    assert_parity(D / sc, Dr / sc, 64, case)
    dA = sD.dA()[:64].cpu().numpy()
    sa = np.abs(dAr).max()
    assert_parity(dA / sa, dAr / sa, 64, "dA " + case)


def test_dgetrf_one_wave_exact_batched():
    """Orders 33..64: exact integer factors without pivoting (every
    intermediate value an integer, so any order of the operations gives the
    exact factors), in place; a full batch of 64 x 64 against the oracle on
    every instance (interchanges equal, factors within the parity bound) with
    one zero pivot reported in info."""
    note("getrf one-wave exact/batched")
    rng = np.random.default_rng(94)
    for (m, n) in [(64, 64), (50, 64), (64, 45)]:
        mn = min(m, n)
        Lm = np.tril(rng.integers(-2, 3, (m, mn)), -1) + np.eye(m, mn)
        U = np.triu(rng.integers(-2, 3, (mn, n)), 1)
        U[np.arange(mn), np.arange(mn)] = rng.choice([1.0, 2.0, -1.0, 4.0], mn)
        C = Lm @ U
        sC = mat(C)
        p.blasfeo_dgetrf_nopivot(m, n, sC, 0, 0, sC, 0, 0)  # in place
        D = host(sC)
        assert np.array_equal(np.tril(D, -1)[:, :mn] + np.eye(m, mn), Lm), (m, n)
        assert np.array_equal(np.triu(D)[:mn, :], U), (m, n)
    batch, m = 4096, 64
    C = rng.standard_normal((batch, m, m))
    C[9, :, 5] = 0.0
    sC, sD = p.pack_batch(dev(C)), p.DMatBatch(batch, m, m)
    info = torch.full((batch,), -1, dtype=torch.int32, device=DEV)
    ipiv = torch.full((batch, m), -1, dtype=torch.int32, device=DEV)
    p.blasfeo_hip_dgetrf_batched(batch, m, m, sC, 0, 0, sD, 0, 0, 1, ipiv, info)
    torch.cuda.synchronize()
    inf = info.cpu().numpy()
    assert inf[9] == 6 and np.sum(inf != 0) == 1
    D = p.unpack_batch(sD).cpu().numpy()
    ip = ipiv.cpu().numpy()
    worst = 0.0
    for b in range(batch):
        Dr, ipr, _, infr = oracle.dgetrf(C[b], pivot=True)
        assert infr == inf[b] and np.array_equal(ip[b], ipr), b
        if b != 9:
            worst = max(worst, rel(D[b], Dr))
    print(f"getrf 4096 x 64x64: worst rel Frobenius error {worst:.3e}")
    assert worst <= TOL * m


def test_dgetrf_exact_batched_info_and_errors():
    note("getrf exact/batched")
    rng = np.random.default_rng(90)
    n = 48
    Lm = np.tril(rng.integers(-2, 3, (n, n)), -1) + np.eye(n)
    U = np.triu(rng.integers(-2, 3, (n, n)), 1) + np.diag(rng.choice([1.0, 2.0, -1.0, 4.0], n))
    sC, sD = mat(Lm @ U), p.DMat(n, n)
    p.blasfeo_dgetrf_nopivot(n, n, sC, 0, 0, sD, 0, 0)
    D = host(sD)
    assert np.array_equal(np.tril(D, -1) + np.eye(n), Lm) and np.array_equal(np.triu(D), U)
    # batch: a zero pivot without pivoting, the same matrix with pivoting
    batch, m = 256, 40
    C = rng.standard_normal((batch, m, m))
    C[7, 0, 0] = 0.0
    C[7, 1:, 0] = rng.standard_normal(m - 1)
    sC, sD = p.pack_batch(dev(C)), p.DMatBatch(batch, m, m)
    info = torch.full((batch,), -1, dtype=torch.int32, device=DEV)
    ipiv = torch.full((batch, m), -1, dtype=torch.int32, device=DEV)
    p.blasfeo_hip_dgetrf_batched(batch, m, m, sC, 0, 0, sD, 0, 0, 0, None, info)
    torch.cuda.synchronize()
    inf = info.cpu().numpy()
    assert inf[7] == 1 and oracle.dgetrf(C[7], pivot=False)[3] == 1
    p.blasfeo_hip_dgetrf_batched(batch, m, m, sC, 0, 0, sD, 0, 0, 1, ipiv, info)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    D = p.unpack_batch(sD).cpu().numpy()
    ip = ipiv.cpu().numpy()
    for b in range(0, batch, 17):
        Dr, ipr, _, _ = oracle.dgetrf(C[b], pivot=True)
        assert np.array_equal(ip[b], ipr)
        assert_parity(D[b], Dr, m, f"getrf b={b}")
    with pytest.raises(p.HipError):
        p.blasfeo_hip_dgetrf_batched(batch, 257, 40, sC, 0, 0, sD, 0, 0, 1, ipiv, info)
    with pytest.raises(p.HipError):
        p.blasfeo_hip_dgetrf_batched(batch, m, m, sC, 0, 0, sD, 0, 0, 1, None, info)


@pytest.mark.parametrize("m,n", [(65, 65), (100, 100), (128, 128), (256, 256), (200, 130), (130, 200),
                                 (17, 200), (256, 20), (97, 250)])
@pytest.mark.parametrize("pivot", [True, False])
@pytest.mark.parametrize("off", [(0, 0, 0, 0), (3, 5, 7, 2)])
def test_dgetrf_blocked(m, n, pivot, off):
    """Orders above 64 (the blocked kernel: panel factorization, interchanges,
    block row of U, MFMA trailing update) against the oracle: the same
    interchanges, the packed L\\U and dA within the parity bound, P A = L U
    to the same bound, sentinels outside D untouched."""
    note("getrf blocked", m, n, pivot, off)
    ci, cj, di, dj = off
    rng = np.random.default_rng(m * 7 + n + int(pivot))
    C = rng.standard_normal((m, n))
    if not pivot:  # diagonally dominant so that no pivoting is needed
        C[np.arange(min(m, n)), np.arange(min(m, n))] += 2.0 * n
    sC, sD = sentinel_mat(ci + m, cj + n), sentinel_mat(di + m, dj + n)
    p.pack(dev(C), sC, ci, cj)
    mn = min(m, n)
    ipiv = torch.full((mn,), -1, dtype=torch.int32, device=DEV)
    if pivot:
        p.blasfeo_dgetrf_pivot(m, n, sC, ci, cj, sD, di, dj, ipiv)
    else:
        p.blasfeo_dgetrf_nopivot(m, n, sC, ci, cj, sD, di, dj)
    p.check_last()
    Dfull = host(sD)
    D = Dfull[di:, dj:]
    Dr, ipr, dAr, inf = oracle.dgetrf(C, pivot=pivot)
    assert inf == 0
    ip = ipiv.cpu().numpy()
    if pivot:
        assert np.array_equal(ip, ipr)
    assert_parity(D, Dr, max(m, n), "getrf blocked")
    assert_parity(sD.dA()[:mn].cpu().numpy(), dAr, max(m, n), "dA")
    # the GPU's own factors: P C = L U
    L = np.tril(D, -1)[:, :mn] + np.eye(m, mn)
    U = np.triu(D)[:mn, :]
    PC = C.copy()
    if pivot:
        for k in range(mn):
            PC[[k, ip[k]]] = PC[[ip[k], k]]
    assert_parity(L @ U, PC, max(m, n), "P C = L U")
    mask = np.ones_like(Dfull, dtype=bool)
    mask[di:, dj:] = False
    assert np.all(Dfull[mask] == SENT)


def test_dgetrf_blocked_exact_nan_batched():
    """Blocked kernel: exact integer factors without pivoting (every
    intermediate value an integer), in place; NaN pivot-column ranking as the
    oracle's; a batch with a zero pivot (info) and the pivoted batch against
    the oracle on every instance."""
    note("getrf blocked exact/nan/batched")
    rng = np.random.default_rng(91)
    n = 150
    Lm = np.tril(rng.integers(-2, 3, (n, n)), -1) + np.eye(n)
    U = np.triu(rng.integers(-2, 3, (n, n)), 1) + np.diag(rng.choice([1.0, 2.0, -1.0, 4.0], n))
    sC = mat(Lm @ U)
    p.blasfeo_dgetrf_nopivot(n, n, sC, 0, 0, sC, 0, 0)  # in place
    D = host(sC)
    assert np.array_equal(np.tril(D, -1) + np.eye(n), Lm) and np.array_equal(np.triu(D), U)
    for where in [(0, 0), (3, 0), (70, 20)]:
        C = rng.standard_normal((90, 80))
        C[where] = np.nan
        sC, sD = mat(C), p.DMat(90, 80)
        ipiv = torch.full((80,), -1, dtype=torch.int32, device=DEV)
        p.blasfeo_dgetrf_pivot(90, 80, sC, 0, 0, sD, 0, 0, ipiv)
        Dr, ipr, _, _ = oracle.dgetrf(C, pivot=True)
        ip = ipiv.cpu().numpy()
        # the interchanges up to the NaN's column are the oracle's, and the
        # NaN reaches the same rows
        k = where[1]
        assert np.array_equal(ip[:k + 1], ipr[:k + 1]), where
        assert np.array_equal(np.isnan(host(sD)[:, :k + 1]), np.isnan(Dr[:, :k + 1])), where
    batch, m = 300, 96
    C = rng.standard_normal((batch, m, m))
    C[7, 0, 0] = 0.0
    C[7, 1:, 0] = rng.standard_normal(m - 1)
    sC, sD = p.pack_batch(dev(C)), p.DMatBatch(batch, m, m)
    info = torch.full((batch,), -1, dtype=torch.int32, device=DEV)
    ipiv = torch.full((batch, m), -1, dtype=torch.int32, device=DEV)
    p.blasfeo_hip_dgetrf_batched(batch, m, m, sC, 0, 0, sD, 0, 0, 0, None, info)
    torch.cuda.synchronize()
    inf = info.cpu().numpy()
    assert inf[7] == 1 and oracle.dgetrf(C[7], pivot=False)[3] == 1 and np.sum(inf != 0) == 1
    p.blasfeo_hip_dgetrf_batched(batch, m, m, sC, 0, 0, sD, 0, 0, 1, ipiv, info)
    torch.cuda.synchronize()
    assert np.all(info.cpu().numpy() == 0)
    D = p.unpack_batch(sD).cpu().numpy()
    ip = ipiv.cpu().numpy()
    for b in range(batch):
        Dr, ipr, _, _ = oracle.dgetrf(C[b], pivot=True)
        assert np.array_equal(ip[b], ipr), b
        assert_parity(D[b], Dr, m, f"getrf blocked b={b}")


# ------------------------------------------------------------------ gelqf

@pytest.mark.parametrize("m,n", [(1, 1), (3, 5), (5, 5), (7, 4), (32, 32), (20, 31), (40, 64), (64, 64), (64, 17),
                                 (33, 33), (17, 64), (64, 1), (1, 64), (37, 61), (61, 37), (48, 48)])
@pytest.mark.parametrize("off", [(0, 0, 0, 0), (3, 5, 7, 2)])
def test_dgelqf(m, n, off):
    """Compact LQ against the oracle element by element (reflectors and L)
    and tau; the GPU's own factors reproduce A with an orthogonal Q.  Up to
    order 32 (the unblocked kernel) the bits are the oracle's; above (one
    wave, panels of 16 rows, MFMA block update) the factors agree within the
    parity bound."""
    note("gelqf", m, n, off)
    ci, cj, di, dj = off
    A = np.random.default_rng(m * 9 + n).standard_normal((m, n))
    sC, sD = sentinel_mat(ci + m, cj + n), sentinel_mat(di + m, dj + n)
    p.pack(dev(A), sC, ci, cj)
    p.blasfeo_dgelqf(m, n, sC, ci, cj, sD, di, dj)
    Dfull = host(sD)
    D = Dfull[di:, dj:]
    tau = sD.dA()[:min(m, n)].cpu().numpy()
    Dr, taur = oracle.dgelqf(A)
    assert_parity(D, Dr, max(m, n), "gelqf")
    assert_parity(tau, taur, max(m, n), "tau")
    if max(m, n) <= 32:
        # same operations in the same order (the norm summed by ascending
        # column), correctly rounded sqrt and division, no contraction: same
        # bits
        assert np.array_equal(D, Dr) and np.array_equal(tau, taur)
    Q = oracle.lq_q(D, tau)
    k = min(m, n)
    assert np.abs(np.tril(D)[:, :k] @ Q[:k] - A).max() <= 1e-13 * max(m, n)
    mask = np.ones_like(Dfull, dtype=bool)
    mask[di:, dj:] = False
    assert np.all(Dfull[mask] == SENT)


def test_dgelqf_batched_and_zero_row():
    note("gelqf batched")
    rng = np.random.default_rng(91)
    batch, m, n = 300, 24, 40
    A = rng.standard_normal((batch, m, n))
    A[5, 0, 1:] = 0.0  # reflector 0 of instance 5 is the identity
    sC, sD = p.pack_batch(dev(A)), p.DMatBatch(batch, m, n)
    p.blasfeo_hip_dgelqf_batched(batch, m, n, sC, 0, 0, sD, 0, 0)
    torch.cuda.synchronize()
    D = p.unpack_batch(sD).cpu().numpy()
    tau = sD.dA()[:, :m].cpu().numpy()
    assert tau[5, 0] == 0.0
    for b in list(range(0, batch, 23)) + [5]:
        Dr, taur = oracle.dgelqf(A[b])
        assert_parity(D[b], Dr, n, f"gelqf b={b}")
        assert_parity(tau[b], taur, n, f"tau b={b}")
    with pytest.raises(p.HipError):
        p.blasfeo_hip_dgelqf_batched(batch, 257, n, sC, 0, 0, sD, 0, 0)


def test_dgelqf_one_wave_batched_identity_reflectors():
    """Orders 33..64 (one wave, MFMA block update): a 2048-instance batch of
    64 x 64 with identity reflectors (a row zero right of its diagonal) in
    the first panel and in a later one, in place, every instance against the
    oracle (reflectors, L and tau within the parity bound; tau exactly 0
    where the oracle's is), and the GPU's own factors reproduce A."""
    note("gelqf one-wave batched")
    rng = np.random.default_rng(93)
    batch, m, n = 2048, 64, 64
    A = rng.standard_normal((batch, m, n))
    A[5, 0, 1:] = 0.0
    A[6, 40, :] = 0.0  # (a zero row stays zero under the reflectors before it)
    A[7, 63, :] = 0.0
    sC = p.pack_batch(dev(A))
    p.blasfeo_hip_dgelqf_batched(batch, m, n, sC, 0, 0, sC, 0, 0)
    torch.cuda.synchronize()
    D = p.unpack_batch(sC).cpu().numpy()
    tau = sC.dA()[:, :m].cpu().numpy()
    assert tau[5, 0] == 0.0 and tau[6, 40] == 0.0 and tau[7, 63] == 0.0
    worst = 0.0
    for b in range(batch):
        Dr, taur = oracle.dgelqf(A[b])
        assert np.array_equal(tau[b] == 0.0, taur == 0.0), b
        worst = max(worst, rel(D[b], Dr), rel(tau[b], taur))
    print(f"gelqf 2048 x 64x64: worst rel Frobenius error {worst:.3e}")
    assert worst <= TOL * n
    for b in (0, 5, 6, 7, 2047):
        Q = oracle.lq_q(D[b], tau[b])
        assert np.abs(np.tril(D[b]) @ Q - A[b]).max() <= 1e-13 * n, b


@pytest.mark.parametrize("m,n", [(65, 65), (100, 100), (128, 128), (256, 256), (200, 130), (130, 200),
                                 (17, 200), (256, 20), (97, 250)])
@pytest.mark.parametrize("off", [(0, 0, 0, 0), (3, 5, 7, 2)])
def test_dgelqf_blocked(m, n, off):
    """Orders above 64 (the blocked kernel: panel reflectors, T from the
    reflectors' Gram matrix, MFMA block update of the rows below) against
    the oracle: reflectors, L and tau within the parity bound; the GPU's own
    factors reproduce A; sentinels outside D untouched."""
    note("gelqf blocked", m, n, off)
    ci, cj, di, dj = off
    A = np.random.default_rng(m * 11 + n).standard_normal((m, n))
    sC, sD = sentinel_mat(ci + m, cj + n), sentinel_mat(di + m, dj + n)
    p.pack(dev(A), sC, ci, cj)
    p.blasfeo_dgelqf(m, n, sC, ci, cj, sD, di, dj)
    p.check_last()
    Dfull = host(sD)
    D = Dfull[di:, dj:]
    k = min(m, n)
    tau = sD.dA()[:k].cpu().numpy()
    Dr, taur = oracle.dgelqf(A)
    assert_parity(D, Dr, max(m, n), "gelqf blocked")
    assert_parity(tau, taur, max(m, n), "tau")
    Q = oracle.lq_q(D, tau)
    assert np.abs(np.tril(D)[:, :k] @ Q[:k] - A).max() <= 1e-13 * max(m, n)
    mask = np.ones_like(Dfull, dtype=bool)
    mask[di:, dj:] = False
    assert np.all(Dfull[mask] == SENT)


def test_dgelqf_blocked_batched_zero_row_in_place():
    """Blocked kernel: a batch with an identity reflector (a zero row right
    of the diagonal), every instance against the oracle; in place."""
    note("gelqf blocked batched")
    rng = np.random.default_rng(92)
    batch, m, n = 200, 90, 120
    A = rng.standard_normal((batch, m, n))
    A[5, 0, 1:] = 0.0
    A[6, 40, 41:] = 0.0
    sC = p.pack_batch(dev(A))
    p.blasfeo_hip_dgelqf_batched(batch, m, n, sC, 0, 0, sC, 0, 0)
    torch.cuda.synchronize()
    D = p.unpack_batch(sC).cpu().numpy()
    tau = sC.dA()[:, :m].cpu().numpy()
    assert tau[5, 0] == 0.0
    for b in range(batch):
        Dr, taur = oracle.dgelqf(A[b])
        assert_parity(D[b], Dr, n, f"gelqf blocked b={b}")
        assert_parity(tau[b], taur, n, f"tau b={b}")


# ------------------------------------------------------------------ potrf_l_mn (stacking)

def stacked(m, n, seed):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n))
    H = G @ G.T + n * np.eye(n)
    A = rng.standard_normal((m - n, n))
    return np.vstack([H, A])


@pytest.mark.parametrize("m,n", [(46, 40), (20, 16), (64, 33), (100, 64), (17, 1), (130, 100), (5, 5), (33, 31)])
@pytest.mark.parametrize("off", [(0, 0, 0, 0), (3, 5, 7, 2)])
def test_dpotrf_l_mn(m, n, off):
    """[H; A] -> [L; A L^-T] element by element against the oracle, with the
    stacked rows sharing the last diagonal tile when n is not a multiple of
    16 (46 x 40: rows 40..45 sit in the tile of columns 32..39); only the
    lower part of H is read; the strictly upper part of the top block of D
    and everything outside D keep their sentinels."""
    note("potrf_l_mn", m, n, off)
    ci, cj, di, dj = off
    C = stacked(m, n, m * 7 + n)
    Cp = C.copy()
    Cp[:n][np.triu_indices(n, 1)] = np.nan
    sC, sD = sentinel_mat(ci + m, cj + n), sentinel_mat(di + m, dj + n)
    p.pack(dev(Cp), sC, ci, cj)
    p.blasfeo_dpotrf_l_mn(m, n, sC, ci, cj, sD, di, dj)
    Dfull = host(sD)
    D = Dfull[di:, dj:]
    Dr, dAr, inf = oracle.dpotrf_l_mn(C, n)
    assert inf == 0
    low = np.tril(np.ones((m, n), bool))
    assert_parity(np.where(low, D, 0.0), Dr, n, "potrf_l_mn")
    assert np.all(D[~low] == SENT)
    assert np.all(Dfull[:di] == SENT) and np.all(Dfull[:, :dj] == SENT)
    assert_parity(sD.dA()[:n].cpu().numpy(), dAr, n, "dA")


def test_dpotrf_l_mn_exact_and_failure():
    note("potrf_l_mn exact")
    for m, n, seed in ((46, 40, 60), (70, 33, 61)):
        L, LL = synth.small_integer_factor(n, seed=seed)
        Y = np.random.default_rng(seed).integers(-3, 4, (m - n, n)).astype(float)
        sC, sD = mat(np.vstack([LL, Y @ L.T])), p.DMat(m, n)
        p.blasfeo_dpotrf_l_mn(m, n, sC, 0, 0, sD, 0, 0)
        assert np.array_equal(np.tril(host(sD)), np.vstack([L, Y]))
    # a non-positive pivot in the last block column (which holds stacked rows)
    C = stacked(46, 40, 62)
    C[37, 37] = -1.0
    batch = 3
    sC = p.pack_batch(dev(np.stack([stacked(46, 40, 63), C, stacked(46, 40, 64)])))
    sD = p.DMatBatch(batch, 46, 40)
    info = torch.full((batch,), -1, dtype=torch.int32, device=DEV)
    p.blasfeo_hip_dpotrf_l_mn_batched(batch, 46, 40, sC, 0, 0, sD, 0, 0, info)
    torch.cuda.synchronize()
    assert info.cpu().numpy().tolist() == [0, oracle.dpotrf_l_mn(C, 40)[2], 0] == [0, 38, 0]
    with pytest.raises(p.HipError):
        p.blasfeo_hip_dpotrf_l_mn_batched(batch, 39, 40, sC, 0, 0, sD, 0, 0, info)


def test_range_space_chain_batched():
    """The two fused calls of the range-space method on a uniform batch:
    potrf_l_mn([H; A]) = [L; Y] (n = 40, 8 constraints: 48 stacked rows fill
    three panels, one fewer than H and A apart), then chol(Y Y^T) by the fused
    syrk+potrf kernel; every instance's factors against the oracle chain."""
    note("range-space chain batched")
    batch, n, ma = 512, 40, 8
    C = np.stack([stacked(n + ma, n, 100 + b) for b in range(batch)])
    sC, sD = p.pack_batch(dev(C)), p.DMatBatch(batch, n + ma, n)
    info = torch.full((batch,), -1, dtype=torch.int32, device=DEV)
    p.blasfeo_hip_dpotrf_l_mn_batched(batch, n + ma, n, sC, 0, 0, sD, 0, 0, info)
    torch.cuda.synchronize()
    assert int((info != 0).sum()) == 0
    D = p.unpack_batch(sD).cpu().numpy()
    Y = D[:, n:, :]
    sY, sZ = p.pack_batch(dev(Y)), p.pack_batch(dev(np.zeros((batch, ma, ma))))
    sS = p.DMatBatch(batch, ma, ma, fill=0.0)
    info2 = torch.full((batch,), -1, dtype=torch.int32, device=DEV)
    p.blasfeo_hip_dsyrk_dpotrf_trsm_batched(batch, ma, n, 0, sY, sZ, None, sS, None, info2)
    torch.cuda.synchronize()
    assert int((info2 != 0).sum()) == 0
    S = p.unpack_batch(sS).cpu().numpy()
    for b in range(0, batch, 37):
        Dr, _, _ = oracle.dpotrf_l_mn(C[b], n)
        assert_parity(np.where(np.tril(np.ones((n + ma, n), bool)), D[b], 0.0), Dr, n, f"D b={b}")
        Sr, _, _ = oracle.dsyrk_dpotrf_ln(Dr[n:], Dr[n:], np.zeros((ma, ma)))
        assert_parity(np.tril(S[b]), Sr, n, f"S b={b}")


@pytest.mark.parametrize("n", [16, 37, 64, 100, 130, 256])
def test_dpotrf_l_small_integer_exact(n):
    """A = L L^T with the closed-form L (diagonal {1, 2, 4}, off-diagonal
    integers -3..3): every partial sum, inverse-block entry and product of
    the blocked factorization is exactly representable, so L is reproduced
    bit for bit."""
    note("potrf exact", n)
    L, A = synth.small_integer_factor(n, seed=n)
    sC, sD = mat(A), p.DMat(n, n)
    p.blasfeo_dpotrf_l(n, sC, 0, 0, sD, 0, 0)
    assert np.array_equal(np.tril(host(sD)), L)
    assert np.array_equal(sD.dA()[:n].cpu().numpy(), 1.0 / np.diag(L))


def test_dpotrf_l_in_place_identity_diagonal():
    note("potrf identity/diag in place")
    d = np.linspace(0.5, 9.0, 40)
    s = mat(np.diag(d))
    p.blasfeo_dpotrf_l(40, s, 0, 0, s, 0, 0)
    out = host(s)
    assert np.array_equal(np.diag(out), np.sqrt(d))
    assert np.count_nonzero(np.tril(out, -1)) == 0


@pytest.mark.parametrize("bad", [0, 7, 16, 39])
def test_dpotrf_l_info_first_failing_pivot(bad):
    note("potrf info", bad)
    L, A = synth.small_integer_factor(40, seed=21)
    A = A.copy()
    A[bad, bad] -= L[bad, bad] ** 2 + 1.0  # pivot of column `bad` becomes -1
    Lr, _, inf = oracle.dpotrf_l(A)
    assert inf == bad + 1
    sC, sD = mat(A), p.DMat(40, 40)
    info = torch.zeros(1, dtype=torch.int32, device=DEV)
    p.blasfeo_hip_dpotrf_l_info(40, sC, 0, 0, sD, 0, 0, info)
    torch.cuda.synchronize()
    assert int(info.item()) == bad + 1
    assert np.array_equal(np.tril(host(sD))[:, :bad], L[:, :bad])


@pytest.mark.parametrize("m,k", [(64, 64), (40, 32), (17, 3), (100, 50)])
def test_dsyrk_dpotrf_ln(m, k):
    note("syrk_potrf", m, k)
    rng = np.random.default_rng(m + k)
    A, B = rng.standard_normal((m, k)) / 4, rng.standard_normal((m, k)) / 4
    G = rng.standard_normal((m, m))
    M0 = G @ G.T + m * np.eye(m)
    C = M0 - A @ B.T  # the lower part of C + A B^T is that of the SPD matrix M0
    sA, sB, sC, sD = mat(A), mat(B), mat(C), p.DMat(m, m)
    info = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    p.blasfeo_hip_dsyrk_dpotrf_ln_info(m, k, sA, 0, 0, sB, 0, 0, sC, 0, 0, sD, 0, 0, info)
    Lr, dAr, inf = oracle.dsyrk_dpotrf_ln(A, B, C)
    D = host(sD)
    assert inf == 0 and int(info.item()) == 0
    assert_parity(np.tril(D), Lr, m, "syrk_potrf")


# ------------------------------------------------------------------ uniform batches (generic kernels)

def test_batched_generic_routines():
    note("batched generic")
    batch, m, n, k = 33, 20, 36, 12
    rng = np.random.default_rng(9)
    A, B, C = rng.uniform(-1, 1, (batch, m, k)), rng.uniform(-1, 1, (batch, n, k)), rng.uniform(-1, 1, (batch, m, n))
    sA, sB, sC = p.pack_batch(dev(A)), p.pack_batch(dev(B)), p.pack_batch(dev(C))
    sD = p.DMatBatch(batch, m, n)
    p.blasfeo_hip_dgemm_nt_batched(batch, m, n, k, 1.0, sA, 0, 0, sB, 0, 0, -1.0, sC, 0, 0, sD, 0, 0)
    torch.cuda.synchronize()
    D = p.unpack_batch(sD).cpu().numpy()
    for b in range(batch):
        assert_parity(D[b], oracle.dgemm_nt(A[b], B[b], C[b], 1.0, -1.0), k, f"gemm b={b}")
    G = rng.standard_normal((batch, m, m))
    S = G @ np.swapaxes(G, 1, 2) + m * np.eye(m)
    sS, sL = p.pack_batch(dev(S)), p.DMatBatch(batch, m, m, fill=0.0)
    info = torch.full((batch,), -1, dtype=torch.int32, device=DEV)
    p.blasfeo_hip_dpotrf_l_batched(batch, m, sS, 0, 0, sL, 0, 0, info)
    torch.cuda.synchronize()
    L = p.unpack_batch(sL).cpu().numpy()
    dA = sL.dA()[:, :m].cpu().numpy()
    assert np.all(info.cpu().numpy() == 0)
    for b in range(batch):
        Lr, dAr, _ = oracle.dpotrf_l(S[b])
        assert_parity(np.tril(L[b]), Lr, m, f"potrf b={b}")
        assert_parity(dA[b], dAr, m, f"dA b={b}")
    X = rng.standard_normal((batch, 5, m))
    sX, sY = p.pack_batch(dev(X)), p.DMatBatch(batch, 5, m)
    p.blasfeo_hip_dtrsm_rltn_batched(batch, 5, m, 2.0, sL, 0, 0, sX, 0, 0, sY, 0, 0)
    torch.cuda.synchronize()
    Y = p.unpack_batch(sY).cpu().numpy()
    for b in range(batch):
        assert_parity(Y[b], oracle.dtrsm_rltn(np.tril(L[b]), X[b], 2.0), m, f"trsm b={b}")
