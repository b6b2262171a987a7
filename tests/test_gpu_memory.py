"""GPU checks of the memory half of the boundary (Appendix A.1.2 and the
packing routines of Appendix A.3): hipMalloc-backed allocate/free of matrices
and vectors, vector creation over caller memory, vector pack/unpack with
offsets, and the statement of the header that compute calls allocate nothing
(the plan executions and the mixed-precision solver run on the caller's
workspace, also inside a captured stream)."""
import ctypes

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


@pytest.mark.parametrize("m,n", [(1, 1), (17, 5), (64, 64), (130, 37)])
def test_allocate_dmat_pack_unpack_free(m, n):
    note("allocate_dmat", m, n)
    L = p.lib()
    L.blasfeo_hip_get_last_error()
    s = p.blasfeo_dmat()
    L.blasfeo_allocate_dmat(m, n, ctypes.byref(s))
    assert L.blasfeo_hip_get_last_error() == 0
    assert s.pA and s.pA % 256 == 0
    assert (s.m, s.n, s.memsize) == (m, n, L.blasfeo_memsize_dmat(m, n))
    assert s.dA == s.pA + s.pm * 16 * s.cn * 8
    A = np.random.default_rng(m + n).standard_normal((m, n))
    At = torch.as_tensor(np.asfortranarray(A).ravel(order="F"), device=DEV)
    L.blasfeo_pack_dmat(m, n, At.data_ptr(), m, ctypes.byref(s), 0, 0)
    back = torch.full((n, m), np.nan, dtype=torch.float64, device=DEV)
    L.blasfeo_unpack_dmat(m, n, ctypes.byref(s), 0, 0, back.data_ptr(), m)
    torch.cuda.synchronize()
    assert L.blasfeo_hip_get_last_error() == 0
    assert np.array_equal(back.t().cpu().numpy(), A)
    L.blasfeo_free_dmat(ctypes.byref(s))
    assert L.blasfeo_hip_get_last_error() == 0
    assert not s.pA and not s.dA
    L.blasfeo_free_dmat(ctypes.byref(s))  # freeing twice is a no-op
    assert L.blasfeo_hip_get_last_error() == 0


@pytest.mark.parametrize("m", [1, 16, 33, 300])
def test_allocate_dvec_pack_unpack_free(m):
    note("allocate_dvec", m)
    L = p.lib()
    L.blasfeo_hip_get_last_error()
    v = p.blasfeo_dvec()
    L.blasfeo_allocate_dvec(m, ctypes.byref(v))
    assert L.blasfeo_hip_get_last_error() == 0
    assert v.pa and v.pa % 256 == 0 and v.m == m and v.memsize == L.blasfeo_memsize_dvec(m)
    x = torch.as_tensor(np.arange(1, m + 1, dtype=np.float64), device=DEV)
    L.blasfeo_pack_dvec(m, x.data_ptr(), ctypes.byref(v), 0)
    y = torch.full((m,), np.nan, dtype=torch.float64, device=DEV)
    L.blasfeo_unpack_dvec(m, ctypes.byref(v), 0, y.data_ptr())
    torch.cuda.synchronize()
    assert L.blasfeo_hip_get_last_error() == 0
    assert torch.equal(x, y)
    L.blasfeo_free_dvec(ctypes.byref(v))
    assert L.blasfeo_hip_get_last_error() == 0 and not v.pa


def test_create_dvec_over_caller_memory_with_offsets():
    """create_dvec records the caller's memory; pack at yi writes exactly
    elements yi..yi+m-1; unpack at xi reads them back; out-of-range
    sub-vectors are rejected before any copy."""
    note("create_dvec offsets")
    L = p.lib()
    L.blasfeo_hip_get_last_error()
    n = 40
    mem = torch.full((L.blasfeo_memsize_dvec(n) // 8,), 7.25, dtype=torch.float64, device=DEV)
    v = p.blasfeo_dvec()
    L.blasfeo_create_dvec(n, ctypes.byref(v), ctypes.c_void_p(mem.data_ptr()))
    assert v.pa == mem.data_ptr() and v.m == n and v.pm == 3
    x = torch.as_tensor(np.linspace(-1.0, 1.0, 13), device=DEV)
    L.blasfeo_pack_dvec(13, x.data_ptr(), ctypes.byref(v), 21)
    torch.cuda.synchronize()
    h = mem.cpu().numpy()
    assert np.all(h[:21] == 7.25) and np.array_equal(h[21:34], x.cpu().numpy()) and np.all(h[34:n] == 7.25)
    y = torch.zeros(5, dtype=torch.float64, device=DEV)
    L.blasfeo_unpack_dvec(5, ctypes.byref(v), 23, y.data_ptr())
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy(), x.cpu().numpy()[2:7])
    assert L.blasfeo_hip_get_last_error() == 0
    L.blasfeo_pack_dvec(13, x.data_ptr(), ctypes.byref(v), 28)  # 28 + 13 > 40
    assert L.blasfeo_hip_get_last_error() == -3
    # an operand outside its vector is reported at the struct's position
    L.blasfeo_unpack_dvec(5, ctypes.byref(v), -1, y.data_ptr())
    assert L.blasfeo_hip_get_last_error() == -2
    torch.cuda.synchronize()
    assert np.array_equal(mem.cpu().numpy(), h)


def _conditioned(ns, cond, nrhs, seed):
    _, mats, rhs = synth.conditioned_batch(len(ns), cond, seed=seed, nrhs=nrhs, sizes=ns)
    plan = p.VbPlan(ns, nrhs)
    A, B = plan.mat_arena(fill=np.nan), plan.vec_arena()
    for i, n in enumerate(ns):
        p.pack(torch.as_tensor(mats[i], device=DEV), out=plan.dmat(A, i))
        plan.rhs(B, i).copy_(torch.as_tensor(rhs[i], device=DEV))
    return plan, mats, rhs, A, B


def test_compute_calls_allocate_nothing():
    """The first FP64 execution and the first mixed-precision call of a new
    plan leave the device's free memory unchanged: their scratch is the
    workspace the caller allocated beforehand (here ~100 MB for the
    mixed-precision tiles, which a first-call allocation would show)."""
    note("no allocation in compute calls")
    # load every code object first (a module's first launch may map its code)
    wp, _, _, Aw, Bw = _conditioned([40, 130], 1e2, 2, seed=30)
    Xw, Lw = wp.vec_arena(), wp.mat_arena()
    z = torch.zeros(2, dtype=torch.int32, device=DEV)
    wp.solve(Aw, Lw, Bw, Xw, z)
    wp.solve_mixed(Aw, Bw, Xw, z.clone(), torch.zeros(2, dtype=torch.float64, device=DEV), z.clone(), L=Lw)
    torch.cuda.synchronize()
    ns = [384] * 128 + [130, 77, 40]
    plan, mats, rhs, A, B = _conditioned(ns, 1e4, 2, seed=31)
    assert plan.mixed_bytes > 50e6
    X, L = plan.vec_arena(fill=np.nan), plan.mat_arena(fill=np.nan)
    w64, wmx = plan.workspace(), plan.workspace(mixed=True)
    b = len(ns)
    info, iters, fb = (torch.full((b,), -7, dtype=torch.int32, device=DEV) for _ in range(3))
    berr = torch.zeros(b, dtype=torch.float64, device=DEV)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    plan.solve(A, L, B, X, info, work=w64)
    plan.solve_mixed(A, B, X, iters, berr, fb, prec=p.FP32, L=L, info=info, work=wmx)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free0 - free1 < 8 << 20, (free0, free1)
    assert np.all(fb.cpu().numpy() == 0) and float(berr.max()) <= 1e-12  # the refinement target


def test_mixed_and_fp64_calls_in_a_captured_graph():
    """Both compute calls recorded by torch's stream capture (global mode)
    and replayed: every replay, with eager work and synchronizations in
    between, matches the eager results bit for bit."""
    note("capture of compute calls")
    ns = [20, 64, 100, 200, 17, 256]
    plan, mats, rhs, A, B = _conditioned(ns, 1e3, 2, seed=32)
    plan.set_graph(False)
    X, L = plan.vec_arena(fill=np.nan), plan.mat_arena(fill=np.nan)
    X2, L2 = plan.vec_arena(fill=np.nan), plan.mat_arena(fill=np.nan)
    w64, wmx = plan.workspace(), plan.workspace(mixed=True)
    b = len(ns)
    info, iters, fb, info2 = (torch.full((b,), -7, dtype=torch.int32, device=DEV) for _ in range(4))
    berr = torch.zeros(b, dtype=torch.float64, device=DEV)
    # eager references
    plan.solve(A, L, B, X, info, work=w64)
    torch.cuda.synchronize()
    Xe, Le = X.clone(), L.clone()
    plan.solve_mixed(A, B, X2, iters, berr, fb, prec=p.FP32, L=L2, info=info2, work=wmx)
    torch.cuda.synchronize()
    X2e, ite, be = X2.clone(), iters.clone(), berr.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan.solve(A, L, B, X, info, work=w64, stream=s)
        plan.solve_mixed(A, B, X2, iters, berr, fb, prec=p.FP32, L=L2, info=info2, work=wmx, stream=s)
    for rep in range(3):
        for t in (X, L, X2):
            t.fill_(np.nan)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        eq = lambda a, c: torch.equal(torch.nan_to_num(a, nan=3.0), torch.nan_to_num(c, nan=3.0))
        assert eq(X, Xe) and eq(L, Le) and eq(X2, X2e), rep
        assert torch.equal(iters, ite) and torch.equal(berr, be), rep
    for i, n in enumerate(ns):
        Lr = oracle.dpotrf_l(mats[i])[0]
        assert_parity(plan.rhs(X, i).cpu().numpy(), oracle.dpotrs_l(Lr, rhs[i]), n, f"x {i}")
