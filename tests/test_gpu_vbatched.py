"""GPU parity of the uneven-batch plan (potrf_l + forward/back substitution,
size-bucketed kernels, captured hipGraph) against the CPU oracle."""
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

SIZES = [1, 5, 8, 15, 16, 17, 31, 32, 33, 47, 48, 49, 63, 64, 65, 80, 100, 127, 128, 129, 200, 256, 300]


def build(ns, nrhs, seed=3):
    rng = np.random.default_rng(seed)
    mats, rhs = [], []
    for n in ns:
        G = rng.standard_normal((n, n))
        A = G @ G.T + n * np.eye(n)
        mats.append(0.5 * (A + A.T))
        rhs.append(rng.standard_normal((n, max(nrhs, 1)))[:, :nrhs])
    plan = p.VbPlan(ns, nrhs)
    A = plan.mat_arena(fill=np.nan)
    L = plan.mat_arena(fill=np.nan)
    B = plan.vec_arena()
    X = plan.vec_arena(fill=np.nan)
    for i, n in enumerate(ns):
        # only the lower triangle of A may be read
        Ai = np.tril(mats[i]) + np.triu(np.full((n, n), np.nan), 1)
        p.pack(torch.as_tensor(Ai, device=DEV), out=plan.dmat(A, i))
        if nrhs:
            plan.rhs(B, i).copy_(torch.as_tensor(rhs[i], device=DEV))
    info = torch.full((len(ns),), -5, dtype=torch.int32, device=DEV)
    return plan, mats, rhs, A, L, B, X, info


def check_all(plan, mats, rhs, L, X, info, nrhs, what):
    torch.cuda.synchronize()
    inf = info.cpu().numpy()
    for i, n in enumerate(plan.ns):
        n = int(n)
        Lr, dAr, ir = oracle.dpotrf_l(mats[i])
        assert ir == 0 and inf[i] == 0, (what, i, inf[i])
        Lg = p.unpack(plan.dmat(L, i)).cpu().numpy()
        assert_parity(np.tril(Lg), Lr, n, f"{what} L n={n}")
        assert np.all(np.isnan(Lg[np.triu_indices(n, 1)])), f"{what}: upper part written (n={n})"
        assert_parity(plan.dmat(L, i).dA()[:n].cpu().numpy(), dAr, n, f"{what} dA n={n}")
        if nrhs:
            Xr = oracle.dpotrs_l(Lr, rhs[i])
            Xg = plan.rhs(X, i).cpu().numpy()
            assert_parity(Xg, Xr, n, f"{what} X n={n}")


@pytest.mark.parametrize("nrhs", [1, 4, 0])
def test_vbatched_mixed_sizes(nrhs):
    note("vbatched", nrhs)
    plan, mats, rhs, A, L, B, X, info = build(SIZES, nrhs)
    plan.set_graph(False)
    plan.solve(A, L, B, X, info)
    check_all(plan, mats, rhs, L, X, info, nrhs, "eager")


def test_vbatched_graph_replay_and_autotune():
    note("vbatched graph")
    ns = [7, 16, 40, 64, 70, 130, 33, 90]
    plan, mats, rhs, A, L, B, X, info = build(ns, 2, seed=8)
    plan.capture(A, L, B, X, info)  # records and instantiates; launches nothing
    torch.cuda.synchronize()
    assert torch.all(torch.isnan(X)) and torch.all(info == -5)
    plan.solve(A, L, B, X, info)  # replays the graph
    check_all(plan, mats, rhs, L, X, info, 2, "graph first")
    X0 = X.clone()
    for rep in range(3):  # replays, with eager work and syncs in between
        X.fill_(np.nan)
        L.fill_(np.nan)
        torch.cuda.synchronize()
        plan.solve(A, L, B, X, info)
        torch.cuda.synchronize()
        assert torch.equal(torch.nan_to_num(X, nan=123.0), torch.nan_to_num(X0, nan=123.0)), rep
    # new data through the same pointers: the replayed graph must see it
    rng = np.random.default_rng(99)
    for i, n in enumerate(ns):
        G = rng.standard_normal((n, n))
        mats[i] = G @ G.T + n * np.eye(n)
        p.pack(torch.as_tensor(mats[i], device=DEV), out=plan.dmat(A, i))
    plan.solve(A, L, B, X, info)
    check_all(plan, mats, rhs, L, X, info, 2, "graph new data")
    plan.autotune(A, L, B, X, info)
    assert len(plan.config()) == 6
    plan.solve(A, L, B, X, info)  # the graph was dropped: direct launches
    check_all(plan, mats, rhs, L, X, info, 2, "after autotune")
    plan.capture(A, L, B, X, info)
    L.fill_(np.nan)
    plan.solve(A, L, B, X, info)
    check_all(plan, mats, rhs, L, X, info, 2, "after autotune, graph")


def test_vbatched_autotune_cache(tmp_path):
    """A plan over the same orders takes every class's configuration from
    the tuning cache (saved to a file and loaded back) without running
    anything, and solves correctly with it."""
    note("vbatched tune cache")
    ns = [7, 16, 40, 64, 70, 130, 33, 90, 200, 250]
    classes = 5  # n <= 16, 33..48, 49..64, 65..192, > 192
    p.tune_cache_clear()
    plan, mats, rhs, A, L, B, X, info = build(ns, 2, seed=8)
    plan.autotune(A, L, B, X, info)
    cfg = plan.config()
    assert p.tune_cache_stats() == (classes, 0, classes)
    path = str(tmp_path / "tune.txt")
    assert p.tune_cache_save(path) == classes
    p.tune_cache_clear()
    assert p.tune_cache_load(path) == classes
    plan2, mats, rhs, A, L, B, X, info = build(ns, 2, seed=9)
    plan2.autotune(A, L, B, X, info)
    torch.cuda.synchronize()
    assert p.tune_cache_stats() == (classes, classes, 0)
    assert torch.all(torch.isnan(L)) and torch.all(info == -5), "a cached autotune launched work"
    assert list(plan2.config()) == list(cfg)
    plan2.solve(A, L, B, X, info)
    check_all(plan2, mats, rhs, L, X, info, 2, "cached configuration")
    # a different batch of orders is a different key: it is timed
    plan3, mats, rhs, A, L, B, X, info = build(ns[:-1], 2, seed=9)
    plan3.autotune(A, L, B, X, info)
    assert p.tune_cache_stats()[2] >= 1
    p.tune_cache_clear()


def test_vbatched_failure_is_per_instance():
    note("vbatched failure")
    ns = [20, 64, 100, 48, 150]
    plan, mats, rhs, A, L, B, X, info = build(ns, 1, seed=4)
    bad = {1: 37, 2: 70, 4: 0}
    for i, col in bad.items():
        M = mats[i].copy()
        M[col, col] = -1.0
        mats[i] = M
        p.pack(torch.as_tensor(M, device=DEV), out=plan.dmat(A, i))
    plan.solve(A, L, B, X, info)
    torch.cuda.synchronize()
    inf = info.cpu().numpy()
    for i, n in enumerate(ns):
        Lr, _, ir = oracle.dpotrf_l(mats[i])
        assert inf[i] == ir, (i, inf[i], ir)
        if ir == 0:
            Lg = p.unpack(plan.dmat(L, i)).cpu().numpy()
            assert_parity(np.tril(Lg), Lr, n, f"L {i}")
            assert_parity(plan.rhs(X, i).cpu().numpy(), oracle.dpotrs_l(Lr, rhs[i]), n, f"X {i}")
    assert [inf[i] for i in bad] == [col + 1 for col in bad.values()]


@pytest.mark.parametrize("cfg", [2, 201, 202, 204, 211, 212])
def test_vbatched_failure_large_configs(cfg):
    """A non-positive pivot in the first or the second block column of a
    column pair, or in a trailing single block column, is reported at its
    1-based position; the other instances are unaffected."""
    note("vbatched large failure cfg", cfg)
    ns = [100, 150, 150, 129, 200]
    plan, mats, rhs, A, L, B, X, info = build(ns, 2, seed=20 + cfg)
    bad = {0: 20, 1: 70, 2: 90, 3: 128}
    for i, col in bad.items():
        M = mats[i].copy()
        M[col, col] = -1.0
        mats[i] = M
        p.pack(torch.as_tensor(M, device=DEV), out=plan.dmat(A, i))
    plan.set_config([2, 2, 2, 2, cfg, cfg])
    plan.solve(A, L, B, X, info)
    torch.cuda.synchronize()
    inf = info.cpu().numpy()
    for i, n in enumerate(ns):
        Lr, _, ir = oracle.dpotrf_l(mats[i])
        assert inf[i] == ir, (cfg, i, inf[i], ir)
        if ir == 0:
            Lg = p.unpack(plan.dmat(L, i)).cpu().numpy()
            assert_parity(np.tril(Lg), Lr, n, f"L {i}")
            assert_parity(plan.rhs(X, i).cpu().numpy(), oracle.dpotrs_l(Lr, rhs[i]), n, f"X {i}")
    assert [inf[i] for i in bad] == [col + 1 for col in bad.values()]


def test_vbatched_full_size_all_instances():
    """The uneven workload at full size (65536 systems, n = 8*U{1..32}, one
    right-hand side) in the benchmark's configuration (autotuned launch
    shapes, captured graph replayed): every system's L (lower), dA and x
    against the oracle, size class by size class (OpenMP driver), each
    within 1e-13 n; every info code 0; the oracle's backward error of every
    GPU solution within (3n+1) u."""
    note("vbatched full size, all instances")
    from oracle import parity
    batch = 65536
    ns = synth.uneven_sizes(batch, seed=2)
    plan = p.VbPlan(ns, 1)
    A = plan.mat_arena()
    L = plan.mat_arena(fill=0.0)
    B = plan.vec_arena()
    X = plan.vec_arena()
    classes = synth.uneven_batch_device(ns, seed=2)
    for n, (idx, An, bn) in classes.items():
        plan.pack_class(n, idx, An, A)
        plan.scatter_rhs(n, idx, bn, B)
    info = torch.full((batch,), -5, dtype=torch.int32, device=DEV)
    plan.autotune(A, L, B, X, info)
    plan.capture(A, L, B, X, info)
    L.fill_(np.nan)
    X.fill_(np.nan)
    info.fill_(-5)
    plan.solve(A, L, B, X, info)
    torch.cuda.synchronize()
    assert int((info != 0).sum().item()) == 0
    w = parity.Worst()
    for n, (idx, An, bn) in classes.items():
        Lg = plan.unpack_class(n, idx, L).cpu().numpy()
        dAg = plan.dA_class(n, idx, L).cpu().numpy()
        Xg = plan.gather_rhs(n, idx, X).cpu().numpy()
        wc = parity.dposv_chunk(parity.Worst(), An.cpu().numpy(), bn.cpu().numpy()[:, :, None], Lg, dAg, Xg)
        for k in ("L", "dA", "X"):
            assert wc[k] <= TOL * n, (n, k, wc[k])
        assert wc["eta"] <= (3 * n + 1) * 2.0 ** -53, (n, wc["eta"])
        w.merge(wc)
    print("[parity] uneven batch", w.as_dict(), flush=True)
    assert w.instances == batch


def test_vbatched_small_integer_exact():
    """Closed form through every size class: A = L L^T with the small-integer
    L (diagonal {1, 2, 4}, off-diagonal -3..3) and b = A x with integer x;
    the factor and the solution come out bit for bit (eager and graph)."""
    note("vbatched exact")
    ns = [8, 16, 23, 33, 48, 64, 65, 100, 130, 200, 256]
    rng = np.random.default_rng(44)
    facs, mats, xs = [], [], []
    for i, n in enumerate(ns):
        Lf, Af = synth.small_integer_factor(n, seed=500 + i)
        facs.append(Lf)
        mats.append(Af)
        xs.append(rng.integers(-4, 5, (n, 2)).astype(float))
    plan = p.VbPlan(ns, 2)
    A, L, B, X = plan.mat_arena(fill=np.nan), plan.mat_arena(fill=np.nan), plan.vec_arena(), plan.vec_arena(fill=np.nan)
    for i, n in enumerate(ns):
        p.pack(torch.as_tensor(mats[i], device=DEV), out=plan.dmat(A, i))
        plan.rhs(B, i).copy_(torch.as_tensor(mats[i] @ xs[i], device=DEV))
    info = torch.full((len(ns),), -5, dtype=torch.int32, device=DEV)
    for cfg in ([2, 2, 2, 2, 211, 211], [1, 1, 1, 1, 4, 8], [4, 4, 4, 4, 104, 204]):
        plan.set_config(cfg)
        L.fill_(np.nan)
        X.fill_(np.nan)
        plan.solve(A, L, B, X, info)
        torch.cuda.synchronize()
        assert np.all(info.cpu().numpy() == 0)
        for i, n in enumerate(ns):
            assert np.array_equal(np.tril(p.unpack(plan.dmat(L, i)).cpu().numpy()), facs[i]), (cfg, n)
            assert np.array_equal(plan.rhs(X, i).cpu().numpy(), xs[i]), (cfg, n)


@pytest.mark.parametrize("cfg", [4, 8, 16, 104, 108, 116, 201, 202, 204, 211, 212, 214])
def test_vbatched_large_kernel_configs(cfg):
    """Every launch configuration of the n > 64 class, with and without
    right-hand sides, ragged orders up to the largest supported one."""
    note("vbatched large cfg", cfg)
    ns = [65, 80, 100, 127, 128, 129, 200, 256, 300, 383, 512]
    for nrhs in (3, 0):
        plan, mats, rhs, A, L, B, X, info = build(ns, nrhs, seed=cfg)
        plan.set_config([2, 2, 2, 2, cfg, cfg])
        assert list(plan.config()) == [2, 2, 2, 2, cfg, cfg]
        plan.solve(A, L, B, X, info)
        check_all(plan, mats, rhs, L, X, info, nrhs, f"cfg {cfg} nrhs {nrhs}")


def test_vbatched_bitwise_deterministic():
    """Two eager executions of a plan give bit-identical factors and
    solutions in every size class."""
    note("vbatched determinism")
    ns = [3, 16, 30, 48, 64, 100, 180, 250, 320]
    plan, mats, rhs, A, L, B, X, info = build(ns, 2, seed=12)
    plan.set_graph(False)
    plan.solve(A, L, B, X, info)
    torch.cuda.synchronize()
    L1, X1 = L.clone(), X.clone()
    L.fill_(np.nan)
    X.fill_(np.nan)
    plan.solve(A, L, B, X, info)
    torch.cuda.synchronize()
    assert torch.equal(torch.nan_to_num(L, nan=7.0), torch.nan_to_num(L1, nan=7.0))
    assert torch.equal(torch.nan_to_num(X, nan=7.0), torch.nan_to_num(X1, nan=7.0))
