"""GPU parity of the mixed-precision uneven-batch solver (FP32 / FP16-operand
factor, FP64 iterative refinement, FP64 fallback) against the CPU oracle."""
import numpy as np
import pytest

import oracle
import synth
from _util import TOL as PTOL
from _util import assert_parity, note

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1704_02457_amd as p  # noqa: E402

DEV = torch.device("cuda:0")
TOL = 1e-12


def setup(mats, rhs, nrhs):
    ns = [m.shape[0] for m in mats]
    plan = p.VbPlan(ns, nrhs)
    A = plan.mat_arena(fill=np.nan)
    B = plan.vec_arena()
    X = plan.vec_arena(fill=np.nan)
    for i, n in enumerate(ns):
        # only the lower triangle of A may be read
        Ai = np.tril(mats[i]) + np.triu(np.full((n, n), np.nan), 1)
        p.pack(torch.as_tensor(Ai, device=DEV), out=plan.dmat(A, i))
        plan.rhs(B, i).copy_(torch.as_tensor(np.asarray(rhs[i]).reshape(n, nrhs), device=DEV))
    return plan, A, B, X


def run(plan, A, B, X, prec, max_iter=10, L=None):
    b = len(plan.ns)
    iters = torch.full((b,), -7, dtype=torch.int32, device=DEV)
    fb = torch.full((b,), -7, dtype=torch.int32, device=DEV)
    berr = torch.full((b,), np.nan, dtype=torch.float64, device=DEV)
    info = torch.full((b,), -7, dtype=torch.int32, device=DEV)
    plan.solve_mixed(A, B, X, iters, berr, fb, prec=prec, tol=TOL, max_iter=max_iter, L=L, info=info)
    torch.cuda.synchronize()
    return iters.cpu().numpy(), berr.cpu().numpy(), fb.cpu().numpy(), info.cpu().numpy()


@pytest.mark.parametrize("prec", [p.FP32, p.FP16_SCALED])
def test_mixed_exact_integer(prec):
    """A = L L^T with a small-integer L and b = A x with integer x: every
    step is exact, so the GPU factor is S L bit for bit, x0 = x and no
    correction is needed."""
    note("mixed exact", prec)
    ns = [1, 7, 16, 40, 64, 100, 130]
    mats, rhs, facs, xs = [], [], [], []
    rng = np.random.default_rng(5)
    for k, n in enumerate(ns):
        L, A = synth.structured_integer_factor(n, seed=k, diag=(1.0,))
        x = rng.integers(-3, 4, (n, 2)).astype(float)
        mats.append(A)
        rhs.append(A @ x)
        facs.append(L)
        xs.append(x)
    plan, A, B, X = setup(mats, rhs, 2)
    it, be, fb, info = run(plan, A, B, X, prec)
    assert list(fb) == [0] * len(ns) and list(it) == [0] * len(ns) and list(info) == [0] * len(ns)
    assert np.all(be == 0.0)
    for i, n in enumerate(ns):
        s = oracle.mixed_scale(mats[i])
        L32 = plan.mixed_factor(i).cpu().numpy().astype(np.float64)
        assert np.array_equal(L32, s[:, None] * facs[i]), f"factor n={n}"
        L32o, so, info_o = oracle.mixed_factor(mats[i], prec)
        assert info_o == 0 and np.array_equal(L32o.astype(np.float64), L32)
        assert np.array_equal(plan.rhs(X, i).cpu().numpy(), xs[i]), f"x n={n}"


SIZES = [1, 5, 16, 17, 33, 64, 65, 100, 130, 200, 256, 300, 384]


@pytest.mark.parametrize("prec,cond", [(p.FP32, 1e2), (p.FP32, 1e4), (p.FP32, 1e6), (p.FP16_SCALED, 1e2)])
def test_mixed_parity(prec, cond):
    """Per instance and right-hand side: the GPU's reported backward error is
    the oracle's backward error of the GPU's x and meets the tolerance; x
    agrees with the oracle's mixed and FP64 solutions within the bound the
    tolerance implies; the correction counts agree with the oracle's within
    one (FP32; FP16: at most one more); the FP32 factor has a backward error
    at the FP32 level."""
    note("mixed parity", prec, cond)
    nrhs = 3
    ns, mats, rhs = synth.conditioned_batch(len(SIZES), cond, seed=4, nrhs=nrhs, sizes=SIZES)
    plan, A, B, X = setup(mats, rhs, nrhs)
    it, be, fb, info = run(plan, A, B, X, prec)
    Xo, ito, etao, _ = oracle.batch_dposv_mixed(mats, rhs, tol=TOL, max_iter=10, prec=prec, nthreads=8)
    assert list(fb) == [0] * len(SIZES), (fb, ito)
    assert np.all(ito >= 0)
    if prec == p.FP32:
        assert np.all(np.abs(it - ito) <= 1), (it, ito)
    else:
        # the oracle rounds every downdate operand to binary16; the GPU only
        # those of the block (matrix-core) downdates, so it never needs more
        assert np.all(it <= ito + 1), (it, ito)
    for i, n in enumerate(SIZES):
        A_ = mats[i]
        Xg = plan.rhs(X, i).cpu().numpy()
        worst = 0.0
        for c in range(nrhs):
            e = oracle.berr(A_, Xg[:, c], rhs[i][:, c])
            worst = max(worst, e)
            assert e <= TOL + n * 2.0 ** -52, (n, c, e)
        assert abs(worst - be[i]) <= n * 2.0 ** -52 + 1e-3 * worst, (n, worst, be[i])
        bound = 2.0 * n * cond * TOL * 4
        for ref in (Xo[i], oracle.dpotrs_l(oracle.dpotrf_l(A_)[0], rhs[i])):
            err = np.abs(Xg - ref).max() / np.abs(ref).max()
            assert err <= bound, (n, err, bound)
        if prec == p.FP32:
            s = oracle.mixed_scale(A_)
            L32 = plan.mixed_factor(i).cpu().numpy().astype(np.float64)
            As = s[:, None] * A_ * s[None, :]
            res = np.linalg.norm(L32 @ L32.T - As) / np.linalg.norm(As)
            assert res <= 4 * n * 2.0 ** -24, (n, res)
            assert np.all(np.triu(L32, 1) == 0)


def test_mixed_fallback_paths():
    """Fallback 1 (factorization breaks down: not SPD, NaN, FP16 at cond 1e6),
    fallback 2 (max_iter = 0 on a system that needs a correction); with an L
    arena those instances are re-solved in FP64 (parity with the FP64
    oracle, info from the FP64 factorization)."""
    note("mixed fallback")
    nrhs = 2
    ns = [40, 90, 130, 64, 100, 33]
    _, mats, rhs = synth.conditioned_batch(len(ns), 1e2, seed=4, nrhs=nrhs, sizes=ns)
    mats[1] = mats[1].copy()
    mats[1][50, 50] = -1.0                       # not SPD: FP64 info 51 (or earlier)
    mats[3] = mats[3].copy()
    mats[3][20, 3] = np.nan                      # NaN below the diagonal
    _, m6, _ = synth.conditioned_batch(1, 1e6, seed=9, nrhs=nrhs, sizes=[130])
    mats[2] = m6[0]                              # FP16 breaks down at cond 1e6
    plan, A, B, X = setup(mats, rhs, nrhs)
    L = plan.mat_arena(fill=0.0)
    it, be, fb, info = run(plan, A, B, X, p.FP16_SCALED, L=L)
    for i in (0, 4, 5):
        assert fb[i] == 0 and info[i] == 0
    assert fb[1] == 1 and fb[2] != 0 and fb[3] != 0
    assert np.isinf(be[1]) and (fb[2] == 2 or np.isinf(be[2]))
    _, _, inf1 = oracle.dpotrf_l(mats[1])
    assert info[1] == inf1 > 0
    Lr, _, inf2 = oracle.dpotrf_l(mats[2])
    assert info[2] == inf2 == 0
    assert_parity(plan.rhs(X, 2).cpu().numpy(), oracle.dpotrs_l(Lr, rhs[2]), 130, "fallback x")
    # max_iter = 0: every instance that needs a correction gives up (fallback 2)
    _, mats, rhs = synth.conditioned_batch(3, 1e4, seed=4, nrhs=1, sizes=[64, 100, 200])
    plan, A, B, X = setup(mats, rhs, 1)
    L = plan.mat_arena(fill=0.0)
    it, be, fb, info = run(plan, A, B, X, p.FP32, max_iter=0, L=L)
    Xo, ito, etao, _ = oracle.batch_dposv_mixed(mats, rhs, max_iter=0, nthreads=3)
    assert list(fb == 2) == list(ito == -2) and np.all(fb == 2)
    assert np.all(info == 0) and np.all(it == 0) and np.all(be > TOL)
    for i in range(3):
        Lr = oracle.dpotrf_l(mats[i])[0]
        assert_parity(plan.rhs(X, i).cpu().numpy(), oracle.dpotrs_l(Lr, rhs[i]), mats[i].shape[0], "fb2 x")
    # without an L arena: the flags alone, X keeps the last iterate
    X.fill_(0.0)
    it, be, fb, info = run(plan, A, B, X, p.FP32, max_iter=0, L=None)
    assert np.all(fb == 2) and np.all(info == 0)
    for i in range(3):
        xg = plan.rhs(X, i).cpu().numpy()[:, 0]
        assert abs(oracle.berr(mats[i], xg, rhs[i][:, 0]) - be[i]) <= 1e-3 * be[i]


def test_mixed_repeat_and_errors():
    """Two calls in a row give identical results (deterministic order of
    every sum); bad arguments are rejected before any launch."""
    note("mixed repeat")
    ns, mats, rhs = synth.conditioned_batch(6, 1e3, seed=4, nrhs=4, sizes=[20, 50, 128, 77, 300, 16])
    plan, A, B, X = setup(mats, rhs, 4)
    r1 = run(plan, A, B, X, p.FP32)
    X1 = X.clone()
    r2 = run(plan, A, B, X, p.FP32)
    # (the arena's padding rows stay NaN)
    assert torch.equal(torch.nan_to_num(X, nan=7.0), torch.nan_to_num(X1, nan=7.0))
    for a, b in zip(r1, r2):
        assert np.array_equal(a, b)
    z = torch.zeros(6, dtype=torch.int32, device=DEV)
    zd = torch.zeros(6, dtype=torch.float64, device=DEV)
    with pytest.raises(p.HipError):
        plan.solve_mixed(A, B, X, z, zd, z, prec=3)
    with pytest.raises(p.HipError):
        plan.solve_mixed(A, B, X, z, zd, z, max_iter=-1)
    with pytest.raises(p.HipError):
        plan.solve_mixed(A, B, X, None, zd, z)
    assert plan.mixed_bytes > plan.ws64_bytes > 0
    plan0 = p.VbPlan([10, 20], 0)
    assert plan0.mixed_bytes == 0
    with pytest.raises(p.HipError):
        plan0.solve_mixed(A, B, X, z, zd, z, work=plan.workspace(mixed=True))
    # a workspace that is not 256-byte aligned is rejected
    w = plan.workspace(mixed=True)
    with pytest.raises(p.HipError):
        plan.solve_mixed(A, B, X, z, zd, z, work=w.data_ptr() + 8)


def x_bound(n, cond, eta_g, eta_o):
    """Per-instance bound on the relative Frobenius difference of two FP64
    solutions X of A X = B, A = U diag(sigma) U^T with sigma_max = 1 and
    kappa_2 = cond.  Where the FP64 forward-error floor cond * u stays below
    the parity tolerance 1e-13 n, that tolerance applies.  Above it no two
    FP64 solvers with different summation orders agree to 1e-13 n, and the
    bound is the first-order perturbation bound of two solutions whose
    normwise backward errors are eta_g and eta_o (each widened by the FP64
    residual's own rounding (n+1) u): for each column,
      ||x_g - x_o||_2 <= ||A^-1||_2 (||r_g||_2 + ||r_o||_2)
                      <= cond sqrt(n) (eta_g + eta_o + 2 (n+1) u) (||A||_inf ||x||_inf + ||b||_inf)
    with ||A||_inf <= sqrt(n), ||x||_inf <= ||x||_2 and ||b||_inf <= ||x||_2."""
    u = 2.0 ** -53
    if cond * u <= PTOL * n:
        return np.full(np.shape(eta_g), PTOL * n)
    return cond * (n + np.sqrt(n)) * (np.asarray(eta_g) + np.asarray(eta_o) + 2 * (n + 1) * u)


def assert_solution_parity(det, n, cond):
    b = x_bound(n, cond, det["eta"], det["eta_orc"])
    bad = np.nonzero(~(det["X"] <= b))[0]
    assert bad.size == 0, (n, cond, bad[:4], det["X"][bad[:4]], b[bad[:4]])


@pytest.mark.parametrize("cond", [1e2, 1e4, 1e6])
def test_conditioned_full_size_all_instances(cond):
    """The conditioned workload at full size (16384 systems, n ~ U{128..384},
    4 rhs) in the benchmark's launch configuration, every system checked:
      * the FP64 plan (autotuned, captured graph replayed): L (lower) and dA
        against the oracle within 1e-13 n, X within x_bound (1e-13 n up to
        cond 1e4, the perturbation bound at cond 1e6), and the oracle's
        backward error of every X within (3n+1) u;
      * the mixed-precision solve (FP32 factor; also FP16 operands at cond
        <= 1e3): no fallback, and the oracle's backward error of every
        solution column within tol (plus the residual's own rounding n u)."""
    note("conditioned full size, all instances", cond)
    from oracle import parity
    batch, nrhs = 16384, 4
    ns = synth.conditioned_sizes(batch, seed=4)
    plan = p.VbPlan(ns, nrhs)
    A, L, B, X = plan.mat_arena(), plan.mat_arena(fill=0.0), plan.vec_arena(), plan.vec_arena()
    orth = synth.orthogonal_batch_device(ns, seed=4, nrhs=nrhs)
    mats = {}
    for n, (idx, U, Bn) in orth.items():
        mats[n] = synth.conditioned_from_orthogonal(U, cond)
        plan.pack_class(n, idx, mats[n], A)
        plan.scatter_rhs(n, idx, Bn, B)
    del orth
    info = torch.full((batch,), -5, dtype=torch.int32, device=DEV)
    plan.autotune(A, L, B, X, info)
    plan.capture(A, L, B, X, info)
    L.fill_(np.nan)
    X.fill_(np.nan)
    info.fill_(-5)
    plan.solve(A, L, B, X, info)
    torch.cuda.synchronize()
    assert int((info != 0).sum().item()) == 0
    host = {}
    w = parity.Worst()
    for n in sorted(mats):
        idx = np.nonzero(ns == n)[0]
        Ah = mats[n].cpu().numpy()
        Bh = plan.gather_rhs(n, idx, B).cpu().numpy()
        host[n] = (idx, Ah, Bh)
        det = {}
        wc = parity.dposv_chunk(parity.Worst(), Ah, Bh, plan.unpack_class(n, idx, L).cpu().numpy(),
                                plan.dA_class(n, idx, L).cpu().numpy(), plan.gather_rhs(n, idx, X).cpu().numpy(),
                                detail=det)
        for k in ("L", "dA"):
            assert wc[k] <= PTOL * n, (n, k, wc[k])
        assert_solution_parity(det, n, cond)
        assert wc["eta"] <= (3 * n + 1) * 2.0 ** -53, (n, wc["eta"])
        w.merge(wc)
    print(f"[parity] conditioned {cond:.0e} FP64 plan", w.as_dict(), flush=True)
    assert w.instances == batch
    X64 = X.clone()
    precs = [p.FP32] + ([p.FP16_SCALED] if cond <= 1e3 else [])
    for prec in precs:
        X.fill_(np.nan)
        L2 = plan.mat_arena(fill=0.0)
        it, be, fb, inf2 = run(plan, A, B, X, prec, L=L2)
        assert np.all(fb == 0) and np.all(inf2 == 0)
        assert float(be.max()) <= TOL
        wm = parity.Worst()
        for n in sorted(host):
            idx, Ah, Bh = host[n]
            Xg = plan.gather_rhs(n, idx, X).cpu().numpy()
            eta = parity.eta_chunk(wm, Ah, Bh, Xg)
            assert eta.max() <= TOL + n * 2.0 ** -52, (prec, n, eta.max())
            # the GPU's own stopping test agrees with the oracle's backward error
            assert np.all(np.abs(eta - be[idx]) <= 1e-3 * eta + n * 2.0 ** -52), (prec, n)
            # x against the FP64 plan's solution (both backward stable)
            X64n = plan.gather_rhs(n, idx, X64).cpu().numpy()
            d = parity.rel_err(Xg, X64n)
            assert d.max() <= 8.0 * n * cond * TOL, (prec, n, d.max())
        print(f"[parity] conditioned {cond:.0e} mixed prec {prec}", wm.as_dict(),
              "iters", np.bincount(it).tolist(), flush=True)
        assert wm.instances == batch
