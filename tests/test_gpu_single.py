"""GPU parity of the single-precision routines (struct blasfeo_smat, 32-float
panels) against the CPU oracle's single-precision routines, through the C ABI.

Tolerances follow from FP32 rounding (u = 2^-24): a k-term dot product
computed in two different orders differs by at most 2*gamma_k times the sum
of the magnitudes of its terms, so gemm/syrk are checked element by element
against (2k + 4) u (|alpha| |A||B|^T + |beta| |C|); the Cholesky factor of a
well-conditioned matrix (condition number below 10 here) is checked by the
relative Frobenius error 4 n u against the oracle and by the backward error
|L L^T - S| / |S| <= 4 n u.  Integer data whose factorization is exact in
binary32 must match bit for bit."""
import numpy as np
import pytest

import oracle
import synth
from _util import note
from oracle import panel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1704_02457_amd as p  # noqa: E402

DEV = torch.device("cuda:0")
SENT = 7.25
U32 = 2.0 ** -24


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device=DEV)


def smat(A):
    return p.spack(dev(A))


def host(sA):
    torch.cuda.synchronize()
    return p.sunpack(sA).cpu().numpy()


def sentinel(m, n):
    return smat(np.full((m, n), SENT, dtype=np.float32))


def spd(n, seed):
    """S = M M^T / n + I with M ~ U[-1, 1]: eigenvalues in [1, ~4]."""
    rng = np.random.default_rng(seed)
    M = rng.uniform(-1, 1, (n, n))
    S = M @ M.T / max(n, 1) + np.eye(n)
    return (0.5 * (S + S.T)).astype(np.float32)


def gemm_bound(A, B, C, alpha, beta):
    k = A.shape[1]
    mag = abs(alpha) * (np.abs(A.astype(np.float64)) @ np.abs(B.astype(np.float64)).T) + abs(beta) * np.abs(C)
    return (2 * k + 4) * U32 * mag + 1e-30


# ------------------------------------------------------------------ pack / unpack

@pytest.mark.parametrize("m,n", [(1, 1), (32, 32), (33, 5), (64, 64), (130, 37)])
def test_spack_matches_independent_decoder(m, n):
    note("spack", m, n)
    rng = np.random.default_rng(m * 100 + n)
    A = rng.standard_normal((m, n)).astype(np.float32)
    s = smat(A)
    torch.cuda.synchronize()
    raw = s.buf[: s.s.pm * 32 * s.s.cn].cpu().numpy()
    assert s.s.cn == (n + 3) // 4 * 4 and s.s.pm == (m + 31) // 32
    assert np.array_equal(panel.unpack(raw, m, n, s.s.cn, 32), A)
    assert np.array_equal(host(s), A)
    big = sentinel(m + 37, n + 3)
    p.spack(dev(A), out=big, bi=37, bj=3)
    full = host(big)
    assert np.array_equal(full[37:, 3:], A)
    mask = np.ones_like(full, dtype=bool)
    mask[37:, 3:] = False
    assert np.all(full[mask] == np.float32(SENT))


def test_smat_memsize_and_create():
    L = p.lib()
    assert L.blasfeo_memsize_smat(0, 0) == 0
    assert L.blasfeo_memsize_smat(-1, 3) == -1
    for m, n in [(1, 1), (33, 5), (64, 64), (100, 7)]:
        ms = L.blasfeo_memsize_smat(m, n)
        pm, cn = (m + 31) // 32, (n + 3) // 4 * 4
        assert ms % 256 == 0 and ms >= 4 * (pm * 32 * cn + max(m, n))
        s = p.SMat(m, n)
        assert (s.s.m, s.s.n, s.s.pm, s.s.cn, s.s.memsize) == (m, n, pm, cn, ms)
        assert s.s.dA - s.s.pA == 4 * pm * 32 * cn


# ------------------------------------------------------------------ gemm_nt / syrk_ln

SGEMM_CASES = [(64, 64, 64), (1, 1, 1), (17, 33, 5), (63, 65, 31), (100, 40, 130), (16, 16, 0)]
OFFS = [(0,) * 8, (3, 5, 33, 2, 1, 7, 40, 11)]


@pytest.mark.parametrize("m,n,k", SGEMM_CASES)
@pytest.mark.parametrize("offs", OFFS)
def test_sgemm_nt(m, n, k, offs):
    note("sgemm_nt", m, n, k, offs)
    ai, aj, bi, bj, ci, cj, di, dj = offs
    rng = np.random.default_rng(m + 3 * n + 7 * k)
    A, B, C = (rng.uniform(-1, 1, s).astype(np.float32) for s in ((m, k), (n, k), (m, n)))
    alpha, beta = 1.5, -0.75
    sA, sB, sC = sentinel(ai + m, aj + k), sentinel(bi + n, bj + k), sentinel(ci + m, cj + n)
    p.spack(dev(A), out=sA, bi=ai, bj=aj)
    p.spack(dev(B), out=sB, bi=bi, bj=bj)
    p.spack(dev(C), out=sC, bi=ci, bj=cj)
    sD = sentinel(di + m, dj + n)
    p.blasfeo_sgemm_nt(m, n, k, alpha, sA, ai, aj, sB, bi, bj, beta, sC, ci, cj, sD, di, dj)
    D = host(sD)
    ref = oracle.sgemm_nt(A, B, C, alpha, beta)
    err = np.abs(D[di:, dj:].astype(np.float64) - ref)
    assert np.all(err <= gemm_bound(A, B, C, alpha, beta)), err.max()
    mask = np.ones_like(D, dtype=bool)
    mask[di:, dj:] = False
    assert np.all(D[mask] == np.float32(SENT))


@pytest.mark.parametrize("k", [5, 7, 30])
def test_sgemm_nt_nonfinite_origin_stays_in_its_row(k):
    """k not a multiple of 4 and an infinite A(ai, aj): only row 0 of D is
    non-finite, as in the oracle; every other row matches it."""
    note("sgemm_nt inf origin", k)
    m, n, ai, aj = 40, 33, 3, 5
    rng = np.random.default_rng(k)
    A, B, C = (rng.uniform(-1, 1, s).astype(np.float32) for s in ((m, k), (n, k), (m, n)))
    A[0, 0] = np.inf
    sA = sentinel(ai + m, aj + k)
    p.spack(dev(A), out=sA, bi=ai, bj=aj)
    sB, sC, sD = smat(B), smat(C), sentinel(m, n)
    p.blasfeo_sgemm_nt(m, n, k, 1.0, sA, ai, aj, sB, 0, 0, 1.0, sC, 0, 0, sD, 0, 0)
    D = host(sD)
    ref = oracle.sgemm_nt(A, B, C, 1.0, 1.0)
    assert np.all(np.isfinite(D[1:])) and np.all(~np.isfinite(ref[0]))
    assert np.array_equal(np.isinf(D[0]) & (np.sign(D[0]) == np.sign(ref[0])), np.isinf(ref[0]))
    err = np.abs(D[1:].astype(np.float64) - ref[1:])
    assert np.all(err <= gemm_bound(A[1:], B, C[1:], 1.0, 1.0)), err.max()


def test_sgemm_nt_integer_exact_and_in_place():
    """Small integers: every product and partial sum is exact in binary32."""
    note("sgemm_nt exact")
    rng = np.random.default_rng(5)
    A, B, C = (rng.integers(-8, 9, s).astype(np.float32) for s in ((77, 45), (50, 45), (77, 50)))
    ref = oracle.sgemm_nt(A, B, C, 2.0, -1.0)
    sC = smat(C)
    p.blasfeo_sgemm_nt(77, 50, 45, 2.0, smat(A), 0, 0, smat(B), 0, 0, -1.0, sC, 0, 0, sC, 0, 0)
    assert np.array_equal(host(sC), ref)


@pytest.mark.parametrize("m,k", [(64, 64), (1, 3), (17, 5), (40, 0), (97, 33)])
@pytest.mark.parametrize("off", [0, 9])
def test_ssyrk_ln(m, k, off):
    note("ssyrk_ln", m, k, off)
    rng = np.random.default_rng(7 * m + k)
    A, B = (rng.uniform(-1, 1, (m, k)).astype(np.float32) for _ in range(2))
    C = rng.uniform(-1, 1, (m, m)).astype(np.float32)
    sD = sentinel(off + m, off + m)
    p.blasfeo_ssyrk_ln(m, k, 0.5, smat(A), 0, 0, smat(B), 0, 0, 2.0, smat(C), 0, 0, sD, off, off)
    D = host(sD)[off:, off:].astype(np.float64)
    ref = oracle.ssyrk_ln(A, B, C, 0.5, 2.0)
    lo = np.tril(np.ones((m, m), dtype=bool))
    assert np.all(np.abs(D - ref)[lo] <= gemm_bound(A, B, C, 0.5, 2.0)[lo])
    assert np.all(D[~lo] == SENT)


# ------------------------------------------------------------------ potrf_l

def check_factor(L, S, ref, n, what):
    L64 = np.tril(L.astype(np.float64))
    nr = np.linalg.norm(ref)
    e = np.linalg.norm(L64 - ref) / (nr if nr > 0 else 1.0)
    assert e <= 4 * n * U32, f"{what}: rel error vs oracle {e:.3e}"
    ns = np.linalg.norm(S.astype(np.float64))
    b = np.linalg.norm(L64 @ L64.T - S) / (ns if ns > 0 else 1.0)
    assert b <= 4 * n * U32, f"{what}: backward error {b:.3e}"


@pytest.mark.parametrize("m", [1, 5, 16, 17, 33, 64, 100, 129])
@pytest.mark.parametrize("off", [(0, 0, 0, 0), (3, 2, 35, 1)])
def test_spotrf_l(m, off):
    note("spotrf_l", m, off)
    ci, cj, di, dj = off
    S = spd(m, m)
    sC = sentinel(ci + m, cj + m)
    p.spack(dev(S), out=sC, bi=ci, bj=cj)
    sD = sentinel(di + m, dj + m)
    p.blasfeo_spotrf_l(m, sC, ci, cj, sD, di, dj)
    D = host(sD)
    L = D[di:, dj:]
    ref, info = oracle.spotrf_l(S)
    assert info == 0
    check_factor(L, S, ref.astype(np.float64), m, f"spotrf m={m}")
    assert np.all(L[np.triu_indices(m, 1)] == np.float32(SENT))
    mask = np.ones_like(D, dtype=bool)
    mask[di:, dj:] = False
    assert np.all(D[mask] == np.float32(SENT))
    if (di, dj) == (0, 0):
        dA = sD.dA()[:m].cpu().numpy().astype(np.float64)
        want = 1.0 / np.diag(L).astype(np.float64)
        assert np.all(np.abs(dA - want) <= 2 * U32 * np.abs(want))
        assert sD.s.use_dA == 1


@pytest.mark.parametrize("m", [24, 64, 112])
def test_spotrf_l_exact_structured(m):
    """A factor whose blocked FP32 factorization is exact (power-of-two
    diagonal, bidiagonal +-1 diagonal blocks, entries -1, 0, 1 below): the
    result must equal it bit for bit, as must the oracle's."""
    note("spotrf exact", m)
    L, S = synth.structured_integer_factor(m, seed=m)
    ref, info = oracle.spotrf_l(S.astype(np.float32))
    assert info == 0 and np.array_equal(ref.astype(np.float64), L)
    sD = p.SMat(m, m)
    p.blasfeo_spotrf_l(m, smat(S), 0, 0, sD, 0, 0)
    assert np.array_equal(np.tril(host(sD)).astype(np.float64), L)


@pytest.mark.parametrize("batch,m", [(7, 40), (300, 64), (33, 100), (5, 1)])
def test_spotrf_l_batched(batch, m):
    note("spotrf_l batched", batch, m)
    S = np.stack([spd(m, 1000 + b) for b in range(batch)])
    sC = p.spack_batch(dev(S))
    sD = p.SMatBatch(batch, m, m)
    info = torch.full((batch,), -5, dtype=torch.int32, device=DEV)
    p.blasfeo_hip_spotrf_l_batched(batch, m, sC, 0, 0, sD, 0, 0, info)
    torch.cuda.synchronize()
    L = p.sunpack_batch(sD).cpu().numpy()
    assert np.all(info.cpu().numpy() == 0)
    for b in sorted({0, batch // 2, batch - 1}):
        ref, _ = oracle.spotrf_l(S[b])
        check_factor(L[b], S[b], ref.astype(np.float64), m, f"instance {b}")
        dA = sD.dA()[b, :m].cpu().numpy().astype(np.float64)
        want = 1.0 / np.diag(L[b]).astype(np.float64)
        assert np.all(np.abs(dA - want) <= 2 * U32 * np.abs(want))


def test_spotrf_l_batched_info():
    """info[b] is the 1-based first pivot that is not positive."""
    note("spotrf info")
    m = 50
    S = np.stack([spd(m, 5) for _ in range(4)])
    S[1, 20, 20] = -1.0
    S[2, 0, 0] = 0.0
    S[3, 49, 49] = -100.0
    sD = p.SMatBatch(4, m, m)
    info = torch.full((4,), -5, dtype=torch.int32, device=DEV)
    p.blasfeo_hip_spotrf_l_batched(4, m, p.spack_batch(dev(S)), 0, 0, sD, 0, 0, info)
    torch.cuda.synchronize()
    got = info.cpu().numpy().tolist()
    want = [oracle.spotrf_l(S[b])[1] for b in range(4)]
    assert want == [0, 21, 1, 50] and got == want


def test_sgemm_ssyrk_batched():
    note("sgemm/ssyrk batched")
    rng = np.random.default_rng(17)
    batch, m, n, k = 500, 40, 24, 40
    A = rng.uniform(-1, 1, (batch, m, k)).astype(np.float32)
    B = rng.uniform(-1, 1, (batch, n, k)).astype(np.float32)
    C = rng.uniform(-1, 1, (batch, m, n)).astype(np.float32)
    sD = p.SMatBatch(batch, m, n)
    p.blasfeo_hip_sgemm_nt_batched(batch, m, n, k, 1.0, p.spack_batch(dev(A)), 0, 0, p.spack_batch(dev(B)), 0, 0,
                                   1.0, p.spack_batch(dev(C)), 0, 0, sD, 0, 0)
    torch.cuda.synchronize()
    D = p.sunpack_batch(sD).cpu().numpy().astype(np.float64)
    for b in (0, 251, batch - 1):
        ref = oracle.sgemm_nt(A[b], B[b], C[b])
        assert np.all(np.abs(D[b] - ref) <= gemm_bound(A[b], B[b], C[b], 1.0, 1.0))
    Q = rng.uniform(-1, 1, (batch, m, m)).astype(np.float32)
    sY = p.SMatBatch(batch, m, m)
    sA = p.spack_batch(dev(A))
    p.blasfeo_hip_ssyrk_ln_batched(batch, m, k, 1.0, sA, 0, 0, sA, 0, 0, 1.0, p.spack_batch(dev(Q)), 0, 0, sY, 0, 0)
    torch.cuda.synchronize()
    Y = p.sunpack_batch(sY).cpu().numpy().astype(np.float64)
    lo = np.tril(np.ones((m, m), dtype=bool))
    for b in (0, 377, batch - 1):
        ref = oracle.ssyrk_ln(A[b], A[b], Q[b])
        assert np.all(np.abs(Y[b] - ref)[lo] <= gemm_bound(A[b], A[b], Q[b], 1.0, 1.0)[lo])


def test_single_argument_errors_and_empty():
    note("single errors")
    s = p.SMat(8, 8)
    with pytest.raises(p.HipError):
        p.blasfeo_sgemm_nt(8, 8, 8, 1.0, s, 1, 0, s, 0, 0, 1.0, s, 0, 0, s, 0, 0)
    with pytest.raises(p.HipError):
        p.blasfeo_spotrf_l(9, s, 0, 0, s, 0, 0)
    with pytest.raises(p.HipError):
        p.blasfeo_ssyrk_ln(8, 8, 1.0, s, 0, 0, s, 0, 1, 1.0, s, 0, 0, s, 0, 0)
    L = p.lib()
    assert L.blasfeo_hip_spotrf_l_batched(70000, 8, s.ref, 0, 0, s.ref, 0, 0, None, None) == -1
    assert L.blasfeo_hip_sgemm_nt_batched(2, 8, 8, 8, 1.0, s.ref, 0, 0, s.ref, 0, 2, 1.0, s.ref, 0, 0, s.ref,
                                          0, 0, None) == -9
    # empty problems launch nothing and succeed
    p.blasfeo_spotrf_l(0, s, 0, 0, s, 0, 0)
    p.blasfeo_sgemm_nt(0, 8, 8, 1.0, s, 0, 0, s, 0, 0, 1.0, s, 0, 0, s, 0, 0)
    info = torch.full((3,), 9, dtype=torch.int32, device=DEV)
    p.blasfeo_hip_spotrf_l_batched(3, 0, s, 0, 0, s, 0, 0, info)
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0, 0, 0]
