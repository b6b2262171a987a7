"""The no-allocation plan execution (blasfeo_hip_dposv_vbatched_noalloc):
its workspace is the library's fixed per-GPU device array.  Checked against
blasfeo_hip_dposv_vbatched (caller's workspace) bit for bit and against the
oracle within 1e-13 n, on two calls in a row, the second with a smaller
batch; the calls allocate no device memory; a plan whose workspace exceeds
the array is rejected before anything is launched."""
import ctypes

import numpy as np
import pytest

import oracle
from _util import assert_parity, note

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1704_02457_amd as p  # noqa: E402

DEV = torch.device("cuda:0")
LIMIT = 32 << 20  # BLASFEO_HIP_NOALLOC_SCRATCH_BYTES


def _batch(ns, nrhs, seed):
    rng = np.random.default_rng(seed)
    plan = p.VbPlan(ns, nrhs)
    A, B = plan.mat_arena(fill=np.nan), plan.vec_arena()
    mats, rhs = [], []
    for i, n in enumerate(ns):
        G = rng.standard_normal((n, n))
        M = G @ G.T + n * np.eye(n)
        M = 0.5 * (M + M.T)
        mats.append(M)
        rhs.append(rng.standard_normal((n, nrhs)))
        Ai = np.tril(M) + np.triu(np.full((n, n), np.nan), 1)  # only the lower part may be read
        p.pack(torch.as_tensor(Ai, device=DEV), out=plan.dmat(A, i))
        plan.rhs(B, i).copy_(torch.as_tensor(rhs[i], device=DEV))
    return plan, mats, rhs, A, B


def _run_pair(ns, nrhs, seed):
    plan, mats, rhs, A, B = _batch(ns, nrhs, seed)
    assert 0 < plan.ws64_bytes <= LIMIT
    b = len(ns)
    L0, X0 = plan.mat_arena(fill=np.nan), plan.vec_arena(fill=np.nan)
    L1, X1 = plan.mat_arena(fill=np.nan), plan.vec_arena(fill=np.nan)
    i0 = torch.full((b,), -5, dtype=torch.int32, device=DEV)
    i1 = torch.full((b,), -5, dtype=torch.int32, device=DEV)
    plan.set_graph(False)
    plan.solve(A, L0, B, X0, i0, work=plan.workspace())
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    plan.solve_noalloc(A, L1, B, X1, i1)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free0 == free1, (free0, free1)
    nan3 = lambda t: torch.nan_to_num(t, nan=3.0)
    assert torch.equal(nan3(L1), nan3(L0)) and torch.equal(nan3(X1), nan3(X0))
    assert torch.equal(i1, i0) and int((i1 != 0).sum()) == 0
    for i, n in enumerate(ns):
        Lr, dAr, ir = oracle.dpotrf_l(mats[i])
        assert ir == 0
        assert_parity(np.tril(p.unpack(plan.dmat(L1, i)).cpu().numpy()), Lr, n, f"noalloc L {i} n={n}")
        assert_parity(plan.dmat(L1, i).dA()[:n].cpu().numpy(), dAr, n, f"noalloc dA {i}")
        assert_parity(plan.rhs(X1, i).cpu().numpy(), oracle.dpotrs_l(Lr, rhs[i]), n, f"noalloc X {i}")


def test_noalloc_matches_workspace_execution_twice():
    note("noalloc: two calls, the second smaller")
    assert p.lib().blasfeo_hip_noalloc_init() == 0
    # orders on both sides of 64 (the scratch holds the n > 64 inverses)
    _run_pair([300, 17, 130, 64, 200, 65, 96, 256, 40, 129], 3, seed=41)
    _run_pair([80, 9, 150], 1, seed=42)


def test_noalloc_rejects_plans_beyond_the_array():
    note("noalloc: size limit")
    ns = [256] * 1100  # 1100 x 16 blocks x 2 KiB > 32 MiB
    plan = p.VbPlan(ns, 1)
    assert plan.ws64_bytes > LIMIT
    A, L = plan.mat_arena(fill=0.0), plan.mat_arena(fill=0.0)
    B, X = plan.vec_arena(), plan.vec_arena(fill=7.0)
    info = torch.full((len(ns),), -5, dtype=torch.int32, device=DEV)
    rc = p.lib().blasfeo_hip_dposv_vbatched_noalloc(plan.handle, ctypes.c_void_p(A.data_ptr()),
                                                    ctypes.c_void_p(L.data_ptr()), ctypes.c_void_p(B.data_ptr()),
                                                    ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(info.data_ptr()),
                                                    None)
    torch.cuda.synchronize()
    assert rc == -1
    assert torch.all(info == -5) and torch.all(X == 7.0)  # nothing launched
    assert p.lib().blasfeo_hip_dposv_vbatched_noalloc(None, None, None, None, None, None, None) == -1
