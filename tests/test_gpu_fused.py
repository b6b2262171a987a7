"""GPU parity of the fused, wave-per-instance syrk_ln + potrf_l + trsm_rltn
batch kernel (the uniform-batch workload) against the CPU oracle."""
import numpy as np
import pytest

import oracle
import synth
from _util import TOL, assert_parity, note

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1704_02457_amd as p  # noqa: E402

DEV = torch.device("cuda:0")


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def run_fused(Q, B, R, poison=True):
    batch, m, k = B.shape
    nrhs = R.shape[1] if R is not None else 0
    sA = p.pack_batch(dev(B)) if k > 0 else None
    sQ = p.pack_batch(dev(Q))
    sE = p.pack_batch(dev(R)) if nrhs > 0 else None
    sL = p.DMatBatch(batch, m, m, fill=np.nan if poison else 0.0)
    sX = p.DMatBatch(batch, nrhs, m, fill=np.nan) if nrhs > 0 else None
    info = torch.full((batch,), -3, dtype=torch.int32, device=DEV)
    p.blasfeo_hip_dsyrk_dpotrf_trsm_batched(batch, m, k, nrhs, sA, sQ, sE, sL, sX, info)
    torch.cuda.synchronize()
    L = p.unpack_batch(sL).cpu().numpy()
    X = p.unpack_batch(sX).cpu().numpy() if nrhs else None
    dA = sL.dA()[:, :m].cpu().numpy()
    return L, X, dA, info.cpu().numpy()


CASES = [(64, 64, 16), (40, 32, 8), (1, 1, 1), (17, 5, 3), (33, 64, 16), (64, 0, 0), (48, 7, 16), (16, 16, 16)]


@pytest.mark.parametrize("m,k,nrhs", CASES)
@pytest.mark.parametrize("batch", [1, 7, 130])
def test_fused_batch_parity(m, k, nrhs, batch):
    note("fused", m, k, nrhs, batch)
    d = synth.uniform_batch(batch, seed=1, n=m, k=max(k, 1), nrhs=max(nrhs, 1))
    B = d["B"][:, :, :k]
    R = d["RHS"][:, :nrhs, :] if nrhs else None
    L, X, dA, info = run_fused(d["Q"], B, R)
    assert np.all(info == 0)
    for b in range(batch):
        M = d["Q"][b] + B[b] @ B[b].T
        Lr, dAr, inf = oracle.dsyrk_dpotrf_ln(B[b], B[b], d["Q"][b]) if k else oracle.dpotrf_l(d["Q"][b])
        assert inf == 0
        assert_parity(np.tril(L[b]), Lr, m, f"L b={b}")
        # strictly upper part of each diagonal block was never written (NaN poison kept)
        assert np.all(np.isnan(L[b][np.triu_indices(m, 1)]))
        assert_parity(dA[b], dAr, m, f"dA b={b}")
        if nrhs:
            assert_parity(X[b], oracle.dtrsm_rltn(Lr, R[b]), m, f"X b={b}")
        del M


def test_fused_exact_small_integer():
    note("fused exact")
    batch, m, k = 5, 64, 12
    Ls, Bs, Qs, Xs = [], [], [], []
    rng = np.random.default_rng(17)
    for b in range(batch):
        L, LL = synth.small_integer_factor(m, seed=100 + b)
        A = rng.integers(-2, 3, (m, k)).astype(float)
        Ls.append(L)
        Bs.append(A)
        Qs.append(LL - A @ A.T)
        Xs.append(rng.integers(-3, 4, (16, m)).astype(float))
    Q, B, X = np.array(Qs), np.array(Bs), np.array(Xs)
    R = np.einsum("bij,bkj->bik", X, np.array(Ls))  # R = X L^T, exact integers
    L, Xg, dA, info = run_fused(Q, B, R)
    assert np.all(info == 0)
    for b in range(batch):
        assert np.array_equal(np.tril(L[b]), Ls[b])
        assert np.array_equal(dA[b], 1.0 / np.diag(Ls[b]))
        assert np.array_equal(Xg[b], X[b])


def test_fused_failure_is_per_instance():
    note("fused failure")
    batch, m = 9, 64
    d = synth.uniform_batch(batch, seed=2, n=m, k=64, nrhs=16)
    Q = d["Q"].copy()
    Q[4, 37, 37] = -1e6  # instance 4 fails at column 37
    Q[7, 0, 0] = np.nan  # instance 7: NaN pivot at column 0
    L, X, dA, info = run_fused(Q, d["B"], d["RHS"])
    for b in range(batch):
        Lr, dAr, inf = oracle.dsyrk_dpotrf_ln(d["B"][b], d["B"][b], Q[b])
        assert info[b] == inf, (b, info[b], inf)
        if inf == 0:
            assert_parity(np.tril(L[b]), Lr, m, f"L b={b}")
            assert_parity(X[b], oracle.dtrsm_rltn(Lr, d["RHS"][b]), m, f"X b={b}")
    assert info[4] == 38 and info[7] == 1


def test_fused_deterministic():
    note("fused determinism")
    d = synth.uniform_batch(64, seed=5)
    a = run_fused(d["Q"], d["B"], d["RHS"], poison=False)
    b = run_fused(d["Q"], d["B"], d["RHS"], poison=False)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_fused_full_size_all_instances():
    """The full uniform-batch workload (16384 instances, n = 64, k = 64, 16
    right-hand sides) in the launch configuration the benchmark times: every
    instance's L (lower triangle), dA and X against the oracle, in chunks of
    4096 run by the oracle's OpenMP driver, each within 1e-13 n."""
    note("fused full size, all instances")
    from oracle import parity
    batch, n, chunk = 16384, 64, 4096
    d = synth.uniform_batch_device(batch, seed=1)
    sA, sQ, sE = p.pack_batch(d["B"]), p.pack_batch(d["Q"]), p.pack_batch(d["RHS"])
    sL = p.DMatBatch(batch, n, n, fill=0.0)
    sX = p.DMatBatch(batch, 16, n, fill=0.0)
    info = torch.full((batch,), -3, dtype=torch.int32, device=DEV)
    p.blasfeo_hip_dsyrk_dpotrf_trsm_batched(batch, n, 64, 16, sA, sQ, sE, sL, sX, info)
    torch.cuda.synchronize()
    assert int((info != 0).sum().item()) == 0
    Lall, Xall = p.unpack_batch(sL), p.unpack_batch(sX)
    # dA of instance b: after its pm*16*cn = 4*16*64 doubles of panels
    base = torch.arange(batch, device=DEV, dtype=torch.int64)[:, None] * sL.stride + 4 * 16 * n
    dAall = sL.buf[base + torch.arange(n, device=DEV)[None, :]]
    w = parity.Worst()
    for c0 in range(0, batch, chunk):
        sl = slice(c0, c0 + chunk)
        parity.fused_chunk(w, d["Q"][sl].cpu().numpy(), d["B"][sl].cpu().numpy(), d["RHS"][sl].cpu().numpy(),
                           Lall[sl].cpu().numpy(), Xall[sl].cpu().numpy(), dAall[sl].cpu().numpy())
    print("[parity] uniform batch", w.as_dict(), flush=True)
    assert w.instances == batch
    for k in ("L", "X", "dA"):
        assert w[k] <= TOL * n, (k, w[k])


def test_fused_bitwise_deterministic():
    """Two launches on the same data give bit-identical factors and solutions
    (every sum has a fixed order: MFMA chains, no atomics)."""
    note("fused determinism")
    d = synth.uniform_batch(257, seed=5, n=64, k=64, nrhs=16)
    out1 = run_fused(d["Q"], d["B"], d["RHS"])
    out2 = run_fused(d["Q"], d["B"], d["RHS"])
    for a, b in zip(out1, out2):
        assert np.array_equal(np.nan_to_num(a, nan=7.0), np.nan_to_num(b, nan=7.0))
