#!/usr/bin/env python3
"""Benchmark of the panel-major FP64 routines on one MI355X.

Workload timed as `value` (one "step"): the uniform batch -- 16384 independent
instances of L = chol(Q + B B^T) (n = 64, k = 64) followed by X = E L^{-T}
with 16 right-hand sides, all in one fused wave-per-instance kernel, inputs
already resident in HBM in panel-major layout; a step is one replay of a
hipGraph holding that call.  Metric: algorithmic GFLOP/s
(LAPACK Working Note 41 counts) and the fraction of the FP64 peak.

Also reported (under "extra"): the single-instance gemm_nt 64^3 and potrf_l 64
latencies.  The JSON line carries the roofline of the dominant kernel (HBM
bound: algorithmic bytes / average kernel time, HIP events on the launch
stream) and the CPU oracle timed on the host cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


def kernel_source_sha():
    """Hash of the code of the timed kernel's sources, comments and white
    space removed (the counter-based traffic in profiles/ is used only while
    it still matches, so any change to the code invalidates it)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("fused.hip", "blocks.hpp", "common.hpp"):
        with open(os.path.join(ROOT, "paper_1704_02457_amd", "csrc", f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()[:16]


def measured_traffic():
    """Per-launch HBM bytes of the fused kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE runs, or None if absent or stale."""
    path = os.path.join(ROOT, "profiles", "traffic_fused_uniform16384.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_sha") != kernel_source_sha():
        return None
    return t.get("bytes_per_launch")


# The paper's own CPU measurements of these routines (single-threaded, one
# matrix, its BLASFEO HP implementation), quoted with their hardware.  They
# are context for the oracle baseline, not targets: no GPU figure is in the
# paper.
PAPER_CPU = [
    {"routine": "dpotrf_l, n = 24", "value": "> 10", "unit": "GFLOP/s", "precision": "FP64",
     "hardware": "Intel Core i7-4800MQ (Haswell) 3.3 GHz, 1 core, AVX2/FMA, peak 52.8 GFLOP/s",
     "passage": "§5.2 (choice of alternative approaches, Intel Haswell)"},
    {"routine": "dgemm_nt, n <= 256", "value": "close to peak (52.8)", "unit": "GFLOP/s", "precision": "FP64",
     "hardware": "Intel Core i7-4800MQ (Haswell) 3.3 GHz, 1 core", "passage": "§1, §5.2 (Intel Haswell)"},
    {"routine": "dgemm_nt", "value": "up to 95 % of peak (about 27.4 of 28.8)", "unit": "GFLOP/s",
     "precision": "FP64", "hardware": "Intel Core i7-3520M (Ivy Bridge) 3.6 GHz, 1 core, AVX, peak 28.8 GFLOP/s",
     "passage": "§5.2 (Intel Ivy-Bridge)"},
    {"routine": "dgemm_nt", "value": "90 % of peak (about 7.7 of 8.6)", "unit": "GFLOP/s", "precision": "FP64",
     "hardware": "ARM Cortex A57 (NVIDIA Tegra TX1) 2.15 GHz, 1 core, peak 8.6 GFLOP/s",
     "passage": "§5.2 (ARM Cortex A57)"},
    {"routine": "plain C triple loop (the oracle's style), runtime sizes", "value": "about 20 % of peak",
     "unit": "fraction", "precision": "FP64", "hardware": "Intel Ivy Bridge i3-3420 and Haswell, 1 core",
     "passage": "Appendix B (numerical experiments)"},
]


def measure_peaks(p, torch, reps=10):
    """Attainable FP64 matrix-core rate and HBM copy rate on this GPU, with the
    library's probe kernels (HIP events on the launch stream)."""
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    sink = torch.zeros(1024, dtype=torch.float64, device=dev)
    fl = {}

    def mfma():
        fl["f"] = p.lib().blasfeo_hip_probe_dmfma(1024, 2000, sink.data_ptr(), stream.cuda_stream)

    _, pm = time_events(mfma, reps, 2, stream)
    nbytes = 1 << 30
    src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)

    def copy():
        p.check(p.lib().blasfeo_hip_probe_copy(src.data_ptr(), dst.data_ptr(), nbytes, stream.cuda_stream))

    _, pc = time_events(copy, reps, 2, stream)
    del src, dst
    torch.cuda.empty_cache()
    if fl["f"] <= 0:
        raise RuntimeError(f"probe_dmfma failed: {fl['f']}")
    return {"fp64_mfma_tflops": round(fl["f"] / (np.median(pm) * 1e-3) / 1e12, 2),
            "hbm_copy_gbs": round(2 * nbytes / (np.median(pc) * 1e-3) / 1e9, 1),
            "probe": "k_probe_dmfma: 4096 waves x 2000 x 4 independent 16x16x4 FP64 MFMA; "
                     "k_probe_copy: 1 GiB -> 1 GiB, 16-byte accesses (read + write bytes counted)"}


def flops_syrk(n, k):
    return n * (n + 1) * k


def flops_potrf(n):
    return n ** 3 / 3.0 + n ** 2 / 2.0 + n / 6.0


def flops_trsm(m, n):
    return m * n * n


def uniform_counts(n=64, k=64, nrhs=16):
    flops = flops_syrk(n, k) + flops_potrf(n) + flops_trsm(nrhs, n)
    lower = n * (n + 1) // 2
    # Q lower, B, E in; L lower, X, dA out (8 bytes each)
    byts = 8 * (lower + n * k + nrhs * n + lower + nrhs * n + n)
    return flops, byts


def uneven_counts(ns):
    """Algorithmic flops (potrf + potrs, 1 rhs) and bytes (A lower in, L lower
    out, b in, x out, dA out) of the uneven batch."""
    n = np.asarray(ns, dtype=np.float64)
    flops = float(np.sum(flops_potrf(n) + 2 * n * n))
    byts = float(np.sum(8 * (n * (n + 1) + 3 * n)))
    return flops, byts


def roofline_pair(flops, byts, ms):
    """Achieved rates of a whole-workload time against both published peaks."""
    tf = flops / (ms * 1e-3) / 1e12
    gbs = byts / (ms * 1e-3) / 1e9
    return {"tflops": round(tf, 2), "frac_fp64_peak": round(tf / FP64_PEAK_TFLOPS, 4),
            "gbs_algorithmic": round(gbs, 1), "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}


def cpu_threads():
    return len(os.sched_getaffinity(0))


def cpu_uneven(p, plan, ns, A, L, B, X, per_class=128):
    """Oracle (potrf + potrs) on a stratified subset of the uneven batch: the
    first `per_class` instances of every order, timed on the host cores and
    extrapolated to the whole batch by flops; the GPU's factors and solutions
    of the subset are compared with the oracle's."""
    from oracle import parity
    w = parity.Worst()
    fl_sub = 0.0
    for n in sorted(set(int(x) for x in ns)):
        idx = np.nonzero(ns == n)[0][:per_class]
        Ah = plan.unpack_class(n, idx, A).cpu().numpy()
        Bh = plan.gather_rhs(n, idx, B).cpu().numpy()
        parity.dposv_chunk(w, Ah, Bh, plan.unpack_class(n, idx, L).cpu().numpy(),
                           plan.dA_class(n, idx, L).cpu().numpy(), plan.gather_rhs(n, idx, X).cpu().numpy(),
                           nthreads=cpu_threads())
        fl_sub += len(idx) * (flops_potrf(n) + 2.0 * n * n)
    fl_all, _ = uneven_counts(ns)
    # the parity helper also ran the oracle's backward error: time only the
    # factor + solve with a second pass over the same subset
    import oracle
    t = 0.0
    for n in sorted(set(int(x) for x in ns)):
        idx = np.nonzero(ns == n)[0][:per_class]
        Ah = plan.unpack_class(n, idx, A).cpu().numpy()
        Bh = plan.gather_rhs(n, idx, B).cpu().numpy()
        t0 = time.perf_counter()
        oracle.batch_dposv_uniform(Ah, Bh, nthreads=cpu_threads())
        t += time.perf_counter() - t0
    gf = fl_sub / t / 1e9
    return {"value": round(gf, 3), "unit": "GFLOP/s", "cores": int(w.threads), "kind": "oracle",
            "solves_per_s_extrapolated": round(len(ns) / (fl_all / (gf * 1e9)), 1),
            "sample": f"{w.instances} systems: the first {per_class} of each of the {len(set(ns.tolist()))} orders, "
                      f"{t:.2f} s, extrapolated to the batch by flops",
            "parity_subset": {"max_rel_err_L": w["L"], "max_rel_err_X": w["X"], "max_eta": w["eta"],
                              "instances": w.instances}}


def bench_uneven(p, synth, torch, batch=65536, reps=5, cpu=True):
    """The uneven workload: 65536 SPD solves, n = 8*U{1..32}, 1 rhs, through
    a plan (size classes, autotuned launch shapes, captured hipGraph)."""
    ns = synth.uneven_sizes(batch, seed=2)
    plan = p.VbPlan(ns, 1)
    A, L = plan.mat_arena(), plan.mat_arena(fill=0.0)
    B, X = plan.vec_arena(), plan.vec_arena()
    classes = synth.uneven_batch_device(ns, seed=2)
    for n, (idx, An, bn) in classes.items():
        plan.pack_class(n, idx, An, A)
        plan.scatter_rhs(n, idx, bn, B)
    del classes
    torch.cuda.empty_cache()
    info = torch.zeros(batch, dtype=torch.int32, device="cuda")
    plan.autotune(A, L, B, X, info)
    plan.capture(A, L, B, X, info)  # the timed executions replay this graph
    stream = torch.cuda.current_stream()
    _, per = time_events(lambda: plan.solve(A, L, B, X, info), reps, 2, stream)
    ms = float(np.median(per))
    fl, by = uneven_counts(ns)
    bad = int((info != 0).sum().item())
    out = {"uneven_ms": round(ms, 3), "uneven_gflops": round(fl / ms / 1e6, 1),
           "uneven_solves_per_s": round(batch / ms * 1e3, 1), "uneven_gbs": round(by / ms / 1e6, 1),
           "uneven_failed": bad, "uneven_config": [int(x) for x in plan.config()],
           "uneven_roofline": roofline_pair(fl, by, ms)}
    if cpu:
        out["uneven_cpu"] = cpu_uneven(p, plan, ns, A, L, B, X)
    del A, L, B, X, plan
    torch.cuda.empty_cache()
    return out


def riccati_stage_flops(nx, nu):
    """Per stage: trmm C = X Lc (X (nu+nx)-by-nx, Lc lower), syrk C C^T,
    potrf of order nu+nx (LAPACK Working Note 41 counts)."""
    nm = nx + nu
    return nm * nx * nx + nm * (nm + 1) * nx + flops_potrf(nm)


def bench_riccati(p, synth, torch, batch=4096, nx=32, nu=8, N=20, reps=10, cpu=True):
    """The Riccati workload: 4096 backward recursions, nx=32, nu=8, N=20."""
    d = synth.riccati_batch(batch, seed=3, nx=nx, nu=nu)
    dev = torch.device("cuda:0")
    sA, sB = p.pack_batch(torch.as_tensor(d["A"], device=dev)), p.pack_batch(torch.as_tensor(d["B"], device=dev))
    sQ, sR = p.pack_batch(torch.as_tensor(d["Q"], device=dev)), p.pack_batch(torch.as_tensor(d["R"], device=dev))
    sP = p.pack_batch(torch.as_tensor(d["PN"], device=dev))
    sF = p.DMatBatch(batch * N, nx + nu, nx + nu, fill=0.0)
    info = torch.zeros(batch, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    _, per = time_events(lambda: p.blasfeo_hip_dric_trf_batched(batch, nx, nu, N, sA, sB, sQ, sR, sP, sF, info,
                                                                stream), reps, 2, stream)
    ms = float(np.median(per))
    fl = batch * N * riccati_stage_flops(nx, nu)
    nm = nx + nu
    # A, B, Q, R, P_N in; N lower (nu+nx)^2 stage factors out
    by = 8.0 * batch * (2 * nx * nx + nx * nu + nu * nu + nx * nx + N * nm * (nm + 1) / 2)
    out = {"riccati_ms": round(ms, 3), "riccati_gflops": round(fl / ms / 1e6, 1),
           "riccati_recursions_per_s": round(batch / ms * 1e3, 1),
           "riccati_failed": int((info != 0).sum().item()),
           "riccati_roofline": roofline_pair(fl, by, ms)}
    if cpu:
        from oracle import parity
        w = parity.Worst()
        Fg = p.unpack_batch(sF).cpu().numpy().reshape(batch, N, nm, nm)
        parity.riccati_chunk(w, d, N, Fg, nthreads=cpu_threads())
        import oracle
        t0 = time.perf_counter()
        oracle.batch_ric_trf(d["A"], d["B"], d["Q"], d["R"], d["PN"], N, nthreads=cpu_threads())
        t = time.perf_counter() - t0
        out["riccati_cpu"] = {"value": round(fl / t / 1e9, 3), "unit": "GFLOP/s", "cores": int(w.threads),
                              "kind": "oracle", "recursions_per_s": round(batch / t, 1),
                              "sample": f"all {batch} recursions, {t:.2f} s",
                              "parity": {"max_rel_err_F": w["F"], "instances": w.instances}}
    # the solve of the linear-quadratic problem on those factors
    rng = np.random.default_rng(5)
    vb, vr = (torch.as_tensor(rng.standard_normal((batch, N, k)), device=dev) for k in (nx, nu))
    vq, vx0 = torch.as_tensor(rng.standard_normal((batch, N + 1, nx)), device=dev), \
        torch.as_tensor(rng.standard_normal((batch, nx)), device=dev)
    vu = torch.empty((batch, N, nu), dtype=torch.float64, device=dev)
    vx = torch.empty((batch, N + 1, nx), dtype=torch.float64, device=dev)
    _, ps = time_events(lambda: p.blasfeo_hip_dric_trs_batched(batch, nx, nu, N, sA, sB, sP, sF, vb, vr, vq, vx0,
                                                               vu, vx, stream), reps, 2, stream)
    out.update({"riccati_solve_ms": round(float(np.median(ps)), 3),
                "riccati_solves_per_s": round(batch / float(np.median(ps)) * 1e3, 1)})
    del sF
    # the C step of one stage as a separate batched trmm_rlnn: C = [B^T; A^T] L,
    # (nu + nx) x nx times an nx x nx lower factor, m n^2 flops per instance
    m = nu + nx
    rng = np.random.default_rng(3)
    sX = p.pack_batch(torch.as_tensor(rng.uniform(-1, 1, (batch, m, nx)), device=dev))
    sLc = p.pack_batch(torch.as_tensor(np.tril(rng.uniform(-1, 1, (batch, nx, nx))), device=dev))
    sC = p.DMatBatch(batch, m, nx)
    _, pt = time_events(lambda: p.blasfeo_hip_dtrmm_rlnn_batched(batch, m, nx, 1.0, sLc, 0, 0, sX, 0, 0, sC, 0, 0,
                                                                 stream), reps, 2, stream)
    tms = float(np.median(pt))
    out.update({"trmm_rlnn_batch_ms": round(tms, 4),
                "trmm_rlnn_batch_gflops": round(batch * m * nx * nx / tms / 1e6, 1),
                "trmm_rlnn_batch_config": f"{batch} x (B {m}x{nx}, A {nx}x{nx} lower)"})
    del sX, sLc, sC
    torch.cuda.empty_cache()
    return out


def bench_stacking(p, torch, batch=16384, n=40, ma=8, reps=10):
    """The range-space method of the stacking passage on a uniform batch:
    potrf_l_mn of [H; A] (H 40x40, 8 constraints: 48 stacked rows fill three
    panels), then chol(Y Y^T) of the 8x40 block Y = A L^-T by the fused
    syrk+potrf kernel."""
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(12)
    G = rng.standard_normal((batch, n, n))
    H = G @ np.swapaxes(G, 1, 2) + n * np.eye(n)
    C = np.concatenate([H, rng.standard_normal((batch, ma, n))], axis=1)
    sC, sD = p.pack_batch(torch.as_tensor(C, device=dev)), p.DMatBatch(batch, n + ma, n)
    info = torch.zeros(batch, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    _, t1 = time_events(lambda: p.blasfeo_hip_dpotrf_l_mn_batched(batch, n + ma, n, sC, 0, 0, sD, 0, 0, info, stream),
                        reps, 2, stream)
    Y = p.unpack_batch(sD)[:, n:, :].contiguous()
    sY, sZ = p.pack_batch(Y), p.pack_batch(torch.zeros((batch, ma, ma), dtype=torch.float64, device=dev))
    sS = p.DMatBatch(batch, ma, ma, fill=0.0)
    info2 = torch.zeros(batch, dtype=torch.int32, device=dev)
    _, t2 = time_events(lambda: p.blasfeo_hip_dsyrk_dpotrf_trsm_batched(batch, ma, n, 0, sY, sZ, None, sS, None, info2,
                                                                        stream), reps, 2, stream)
    m1, m2 = float(np.median(t1)), float(np.median(t2))
    fl1 = flops_potrf(n) + ma * n * n
    fl2 = ma * (ma + 1) * n + flops_potrf(ma)
    # LU with partial pivoting of 16384 independent 64 x 64 matrices
    nl = 64
    sG = p.pack_batch(torch.as_tensor(rng.standard_normal((batch, nl, nl)), device=dev))
    sLU = p.DMatBatch(batch, nl, nl)
    ipiv = torch.zeros((batch, nl), dtype=torch.int32, device=dev)
    info3 = torch.zeros(batch, dtype=torch.int32, device=dev)
    _, t3 = time_events(lambda: p.blasfeo_hip_dgetrf_batched(batch, nl, nl, sG, 0, 0, sLU, 0, 0, 1, ipiv, info3,
                                                             stream), reps, 2, stream)
    m3 = float(np.median(t3))
    # LQ of the same matrices
    sLQ = p.DMatBatch(batch, nl, nl)
    _, t4 = time_events(lambda: p.blasfeo_hip_dgelqf_batched(batch, nl, nl, sG, 0, 0, sLQ, 0, 0, stream), reps, 2,
                        stream)
    m4 = float(np.median(t4))
    del sG, sLU, sLQ
    # the blocked LU (orders above 64): 2048 independent 256 x 256 matrices,
    # and one 256 x 256 matrix alone (latency)
    nb, bb = 256, 2048
    gen = torch.Generator(device=dev)
    gen.manual_seed(15)
    sG = p.pack_batch(torch.randn((bb, nb, nb), dtype=torch.float64, device=dev, generator=gen))
    sLU = p.DMatBatch(bb, nb, nb)
    ipb = torch.zeros((bb, nb), dtype=torch.int32, device=dev)
    infb = torch.zeros(bb, dtype=torch.int32, device=dev)
    _, t5 = time_events(lambda: p.blasfeo_hip_dgetrf_batched(bb, nb, nb, sG, 0, 0, sLU, 0, 0, 1, ipb, infb, stream),
                        reps, 1, stream)
    m5 = float(np.median(t5))
    _, t6 = time_events(lambda: p.blasfeo_hip_dgetrf_batched(1, nb, nb, sG, 0, 0, sLU, 0, 0, 1, ipb, infb, stream),
                        reps, 2, stream)
    m6 = float(np.median(t6))
    sLQ = p.DMatBatch(bb, nb, nb)
    _, t7 = time_events(lambda: p.blasfeo_hip_dgelqf_batched(bb, nb, nb, sG, 0, 0, sLQ, 0, 0, stream), reps, 1,
                        stream)
    m7 = float(np.median(t7))
    del sG, sLU, sLQ
    return {"getrf_pivot_256_batch_ms": round(m5, 3),
            "getrf_pivot_256_batch_gflops": round(bb * (2.0 / 3.0) * nb ** 3 / m5 / 1e6, 1),
            "getrf_pivot_256_batch_config": f"{bb} x {nb}x{nb}, blocked (panels of 16, MFMA trailing update)",
            "getrf_pivot_256_single_us": round(m6 * 1e3, 1),
            "gelqf_256_batch_ms": round(m7, 3),
            "gelqf_256_batch_gflops": round(bb * (4.0 / 3.0) * nb ** 3 / m7 / 1e6, 1),
            "gelqf_64_batch_ms": round(m4, 4),
            "gelqf_64_batch_gflops": round(batch * (4.0 / 3.0) * nl ** 3 / m4 / 1e6, 1),
            "gelqf_64_batch_config": f"{batch} x {nl}x{nl}, one wave per instance (matrix in registers, "
                                     "panels of 16 rows, MFMA block update)",
            "getrf_pivot_64_batch_ms": round(m3, 4),
            "getrf_pivot_64_batch_gflops": round(batch * (2.0 / 3.0) * nl ** 3 / m3 / 1e6, 1),
            "getrf_pivot_64_batch_config": f"{batch} x {nl}x{nl}, one wave per instance (matrix in registers, "
                                           "panels of 16, MFMA trailing update)",
            "stacked_potrf_l_mn_ms": round(m1, 4), "stacked_potrf_l_mn_gflops": round(batch * fl1 / m1 / 1e6, 1),
            "range_space_schur_chol_ms": round(m2, 4),
            "range_space_chain_ms": round(m1 + m2, 4),
            "range_space_config": f"{batch} x (H {n}x{n}, A {ma}x{n})",
            "range_space_failed": int((info != 0).sum().item() + (info2 != 0).sum().item())}


def bench_single(p, torch, batch=16384, n=64, reps=10):
    """The single-precision routines on 16384 independent 64 x 64 operands:
    sgemm_nt (64x64x64) and spotrf_l of SPD matrices, FP32 panel-major."""
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(14)
    f = dict(device=dev, dtype=torch.float32, generator=g)
    A, B, C = (torch.rand((batch, n, n), **f) * 2 - 1 for _ in range(3))
    sA, sB, sC = p.spack_batch(A), p.spack_batch(B), p.spack_batch(C)
    sD = p.SMatBatch(batch, n, n)
    stream = torch.cuda.current_stream()
    _, t1 = time_events(lambda: p.blasfeo_hip_sgemm_nt_batched(batch, n, n, n, 1.0, sA, 0, 0, sB, 0, 0, 1.0, sC, 0, 0,
                                                               sD, 0, 0, stream), reps, 2, stream)
    S = torch.bmm(A, A.transpose(1, 2).contiguous()) / n + torch.eye(n, device=dev, dtype=torch.float32)
    sS, sL = p.spack_batch(S), p.SMatBatch(batch, n, n)
    info = torch.zeros(batch, dtype=torch.int32, device=dev)
    _, t2 = time_events(lambda: p.blasfeo_hip_spotrf_l_batched(batch, n, sS, 0, 0, sL, 0, 0, info, stream), reps, 2,
                        stream)
    m1, m2 = float(np.median(t1)), float(np.median(t2))
    del A, B, C, S, sA, sB, sC, sD, sS, sL
    return {"sgemm_nt_64_batch_ms": round(m1, 4), "sgemm_nt_64_batch_gflops": round(batch * 2.0 * n ** 3 / m1 / 1e6, 1),
            "spotrf_l_64_batch_ms": round(m2, 4),
            "spotrf_l_64_batch_gflops": round(batch * flops_potrf(n) / m2 / 1e6, 1),
            "spotrf_l_failed": int((info != 0).sum().item())}


def mixed_fp64_counts(ns, nrhs):
    """FP64 path per system: potrf n^3/3 + forward/back solves 2 n^2 per rhs."""
    ns = np.asarray(ns, dtype=np.float64)
    return float(np.sum(ns ** 3 / 3.0 + ns ** 2 / 2.0 + ns / 6.0 + 2.0 * nrhs * ns ** 2))


def cpu_conditioned(plan, ns, A, L, B, X, nrhs, per_order=16):
    """Oracle FP64 solves (potrf + potrs) on a stratified subset of the
    conditioned batch (the first `per_order` systems of every order), timed on
    the host cores, with the GPU's FP64-plan factors and solutions of the
    subset compared with the oracle's."""
    from oracle import parity
    import oracle
    w = parity.Worst()
    fl_sub, t = 0.0, 0.0
    for n in sorted(set(int(x) for x in ns)):
        idx = np.nonzero(ns == n)[0][:per_order]
        Ah = plan.unpack_class(n, idx, A).cpu().numpy()
        Bh = plan.gather_rhs(n, idx, B).cpu().numpy()
        parity.dposv_chunk(w, Ah, Bh, plan.unpack_class(n, idx, L).cpu().numpy(),
                           plan.dA_class(n, idx, L).cpu().numpy(), plan.gather_rhs(n, idx, X).cpu().numpy(),
                           nthreads=cpu_threads())
        t0 = time.perf_counter()
        oracle.batch_dposv_uniform(Ah, Bh, nthreads=cpu_threads())
        t += time.perf_counter() - t0
        fl_sub += len(idx) * (flops_potrf(n) + 2.0 * nrhs * n * n)
    gf = fl_sub / t / 1e9
    return {"value": round(gf, 3), "unit": "GFLOP/s", "cores": int(w.threads), "kind": "oracle",
            "solves_per_s_extrapolated": round(len(ns) / (mixed_fp64_counts(ns, nrhs) / (gf * 1e9)), 1),
            "sample": f"{w.instances} systems (the first {per_order} of every order), {t:.2f} s, "
                      "extrapolated to the batch by flops",
            "parity_subset": {"max_rel_err_L": w["L"], "max_rel_err_X": w["X"], "max_eta": w["eta"],
                              "instances": w.instances}}


def bench_mixed(p, synth, torch, batch=16384, nrhs=4, reps=3, conds=(1e2, 1e4, 1e6), fp16_max_cond=1e3, cpu=True):
    """The mixed-precision workload: 16384 SPD systems, n ~ U{128..384},
    A = U diag(sigma) U^T with cond in {1e2, 1e4, 1e6}, 4 rhs; the FP32
    (and, for cond <= 1e3, FP16-operand) factor with FP64 refinement to
    eta <= 1e-12, against the plain FP64 plan on the same data."""
    ns = synth.conditioned_sizes(batch, seed=4)
    plan = p.VbPlan(ns, nrhs)
    ws = plan.mixed_bytes
    A, L = plan.mat_arena(), plan.mat_arena(fill=0.0)
    B, X = plan.vec_arena(), plan.vec_arena()
    t0 = time.perf_counter()
    orth = synth.orthogonal_batch_device(ns, seed=4, nrhs=nrhs)
    for n, (idx, U, Bn) in orth.items():
        plan.scatter_rhs(n, idx, Bn, B)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    info = torch.zeros(batch, dtype=torch.int32, device=dev)
    iters = torch.zeros(batch, dtype=torch.int32, device=dev)
    fb = torch.zeros(batch, dtype=torch.int32, device=dev)
    berr = torch.zeros(batch, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    fl64 = mixed_fp64_counts(ns, nrhs)
    out = {"mixed_batch": batch, "mixed_nrhs": nrhs, "mixed_workspace_gb": round(ws / 1e9, 2),
           "mixed_input_gen_s": round(gen_s, 1), "mixed_fp64_gflop": round(fl64 / 1e9, 1)}
    tuned = False
    for cond in conds:
        for n, (idx, U, Bn) in orth.items():
            plan.pack_class(n, idx, synth.conditioned_from_orthogonal(U, cond), A)
        torch.cuda.synchronize()
        if not tuned:
            plan.autotune(A, L, B, X, info)
            plan.capture(A, L, B, X, info)
            tuned = True
        _, per = time_events(lambda: plan.solve(A, L, B, X, info), reps, 1, stream)
        ms64 = float(np.median(per))
        by64 = float(np.sum(8.0 * (ns * (ns + 1.0) + ns + 2.0 * nrhs * ns)))
        r = {"fp64_ms": round(ms64, 3), "fp64_solves_per_s": round(batch / ms64 * 1e3, 1),
             "fp64_gflops": round(fl64 / ms64 / 1e6, 1), "fp64_failed": int((info != 0).sum().item()),
             "fp64_roofline": roofline_pair(fl64, by64, ms64)}
        if cpu and cond == conds[0]:
            r["fp64_cpu"] = cpu_conditioned(plan, ns, A, L, B, X, nrhs)
        precs = [("fp32", p.FP32)] + ([("fp16", p.FP16_SCALED)] if cond <= fp16_max_cond else [])
        host = None  # host copies of this condition's matrices, for the oracle's backward errors
        for name, prec in precs:
            def solve():
                plan.solve_mixed(A, B, X, iters, berr, fb, prec=prec, tol=1e-12, max_iter=10, L=L, info=info)
            _, per = time_events(solve, reps, 1, stream)
            ms = float(np.median(per))
            it = iters.cpu().numpy()
            f = fb.cpu().numpy()
            be = berr.cpu().numpy()
            ok = f == 0
            if cpu:
                # the oracle's backward error of every mixed-precision solution
                from oracle import parity
                if host is None:
                    host = {n: (plan.unpack_class(n, np.nonzero(ns == n)[0], A).cpu().numpy(),
                                plan.gather_rhs(n, np.nonzero(ns == n)[0], B).cpu().numpy())
                            for n in sorted(set(int(x) for x in ns))}
                wm = parity.Worst()
                for n, (Ah, Bh) in host.items():
                    parity.eta_chunk(wm, Ah, Bh, plan.gather_rhs(n, np.nonzero(ns == n)[0], X).cpu().numpy(),
                                     nthreads=cpu_threads())
                r[f"{name}_oracle_max_berr"] = wm["eta"]
                r[f"{name}_oracle_checked"] = wm.instances
            r.update({
                f"{name}_ms": round(ms, 3),
                f"{name}_solves_per_s": round(batch / ms * 1e3, 1),
                f"{name}_speedup_vs_fp64": round(ms64 / ms, 3),
                f"{name}_iters_hist": {int(k): int(v) for k, v in zip(*np.unique(it[ok], return_counts=True))},
                f"{name}_max_berr": float(be[ok].max()) if ok.any() else None,
                f"{name}_fallback": {"factor": int((f == 1).sum()), "refine": int((f == 2).sum())},
                f"{name}_fp64_failed_after_fallback": int((info != 0).sum().item()),
            })
        out[f"mixed_cond_{cond:.0e}"] = r
    del A, L, B, X, orth, plan
    torch.cuda.empty_cache()
    return out


def warm(fn, warmup, min_ms=30.0):
    """At least `warmup` calls, and calls until the GPU has been busy for
    min_ms: its clocks settle only after tens of milliseconds under load."""
    import torch
    t0 = time.perf_counter()
    i = 0
    while i < warmup or (time.perf_counter() - t0) * 1e3 < min_ms:
        fn()
        i += 1
        if i % 4 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()


def time_steps(fn, steps, warmup, stream):
    """K steps back to back, bracketed by synchronizations: wall-clock
    seconds and the GPU milliseconds between two events on the stream
    around them (no instrumentation between the steps)."""
    import torch
    warm(fn, warmup)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, e0.elapsed_time(e1)


def time_events(fn, steps, warmup, stream):
    import torch
    warm(fn, warmup)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [a.elapsed_time(b) for a, b in evs]
    return wall, per


def cpu_baseline_uniform(Qh, Bh, Rh, flops_per, min_seconds=10.0):
    import oracle
    threads = len(os.sched_getaffinity(0))
    done, t0 = 0, time.perf_counter()
    used = threads
    while True:
        Lo, Xo, _, info, used = oracle.batch_syrk_potrf_trsm(Qh, Bh, Rh, nthreads=threads)
        done += Qh.shape[0]
        el = time.perf_counter() - t0
        if el >= min_seconds:
            break
    out = {"value": round(done * flops_per / el / 1e9, 3), "unit": "GFLOP/s", "cores": int(used),
           "kind": "oracle",
           "sample": f"{Qh.shape[0]} instances of the same workload (host copy of the device inputs), "
                     f"{done // Qh.shape[0]} pass(es), {el:.1f} s, OpenMP over instances"}
    return out, Lo, Xo


def parity_vs_oracle(Lg, Xg, Lo, Xo):
    """Largest relative Frobenius error of the GPU's L (lower) and X over the
    compared instances, with the 1e-13*n bound of the parity tests."""
    n = Lg.shape[-1]
    eL = np.linalg.norm(np.tril(Lg) - Lo, axis=(1, 2)) / np.linalg.norm(Lo, axis=(1, 2))
    eX = np.linalg.norm(Xg - Xo, axis=(1, 2)) / np.linalg.norm(Xo, axis=(1, 2))
    worst = float(max(eL.max(), eX.max()))
    return {"instances": int(Lg.shape[0]), "max_rel_frobenius_err": worst, "bound": 1e-13 * n,
            "within_bound": bool(worst <= 1e-13 * n)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    # the GPU's clocks settle only after tens of milliseconds under load (the
    # first ~50 replays after the set-up run about 8 % slower than the rest);
    # every timing also keeps warming up until the GPU has been busy 30 ms
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--batch", type=int, default=16384)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-extra", action="store_true", help="time only the uniform-batch workload")
    ap.add_argument("--legs", default="uneven,riccati,stacking,single,mixed",
                    help="comma list of the further workloads to time (uneven, riccati, stacking, single, mixed)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration for rocprofv3 --pmc)")
    ap.add_argument("--tune-cache", default=os.environ.get(
                        "BLASFEO_HIP_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "blasfeo_hip",
                                                               "tune.txt")),
                    help="tuning-cache file of the plans' autotuner: loaded before the legs, saved after them "
                         "('' for none)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU only (asked for --gpus {args.gpus}); "
              "the instances are independent and would shard by contiguous chunks of the batch, "
              "one chunk per GPU, with no collective on the hot path", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1704_02457_amd as p
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    B, n, k, nrhs = args.batch, 64, 64, 16
    print(f"[bench] generating uniform batch {B} x (n={n}, k={k}, nrhs={nrhs})", file=sys.stderr, flush=True)
    d = synth.uniform_batch_device(B, seed=1, n=n, k=k, nrhs=nrhs)
    sA, sQ, sE = p.pack_batch(d["B"]), p.pack_batch(d["Q"]), p.pack_batch(d["RHS"])
    sL = p.DMatBatch(B, n, n, fill=0.0)
    sX = p.DMatBatch(B, nrhs, n, fill=0.0)
    info = torch.zeros(B, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()

    # one step = one replay of a hipGraph holding the fused batched call
    gstream = torch.cuda.Stream()
    gstream.wait_stream(stream)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=gstream):
        p.blasfeo_hip_dsyrk_dpotrf_trsm_batched(B, n, k, nrhs, sA, sQ, sE, sL, sX, info, gstream)
    torch.cuda.synchronize()

    def step():
        graph.replay()

    print("[bench] timing fused syrk+potrf+trsm (graph replays)", file=sys.stderr, flush=True)
    wall, gpu_ms = time_steps(step, args.steps, args.warmup, stream)
    # per-replay distribution, in a separate pass (an event pair per replay)
    _, per = time_events(step, min(args.steps, 50), 2, stream)
    bad = int((info != 0).sum().item())
    if bad:
        print(f"[bench] WARNING: {bad} instances reported a failed factorization", file=sys.stderr)
    fl, by = uniform_counts(n, k, nrhs)
    kern_ms = gpu_ms / args.steps  # one kernel per step: its average duration in the timed region
    ms_step = wall * 1e3 / args.steps
    gflops = B * fl / (ms_step * 1e-3) / 1e9
    achieved_gbs = B * by / (kern_ms * 1e-3) / 1e9

    # single-instance latencies (gemm_nt 64^3, potrf_l 64)
    s = synth.single(seed=0, n=64)
    A1, B1, C1 = (p.pack(torch.as_tensor(s[x], device=dev)) for x in "ABC")
    D1 = p.DMat(64, 64)
    S1, L1 = p.pack(torch.as_tensor(s["S"], device=dev)), p.DMat(64, 64)

    def gemm1():
        p.blasfeo_dgemm_nt(64, 64, 64, 1.0, A1, 0, 0, B1, 0, 0, 1.0, C1, 0, 0, D1, 0, 0)

    def potrf1():
        p.blasfeo_dpotrf_l(64, S1, 0, 0, L1, 0, 0)

    _, pg = time_events(gemm1, 50, 5, stream)
    _, pp = time_events(potrf1, 50, 5, stream)

    # the other single-instance routines of the path at the same sizes:
    # syrk_ln 64x64 (k = 64) and trsm_rltn of a 16x64 right-hand side
    Y1 = p.DMat(64, 64)
    E1, X1 = p.pack(torch.as_tensor(s["A"][:16], device=dev)), p.DMat(16, 64)
    p.blasfeo_dpotrf_l(64, S1, 0, 0, L1, 0, 0)

    def syrk1():
        p.blasfeo_dsyrk_ln(64, 64, 1.0, A1, 0, 0, B1, 0, 0, 1.0, C1, 0, 0, Y1, 0, 0)

    def trsm1():
        p.blasfeo_dtrsm_rltn(16, 64, 1.0, L1, 0, 0, E1, 0, 0, X1, 0, 0)

    _, ps1 = time_events(syrk1, 50, 5, stream)
    _, pt1 = time_events(trsm1, 50, 5, stream)
    extra = {
        "single_gemm_nt_64_us": round(float(np.median(pg)) * 1e3, 2),
        "single_gemm_nt_64_gflops": round(2 * 64 ** 3 / (np.median(pg) * 1e-3) / 1e9, 2),
        "single_potrf_l_64_us": round(float(np.median(pp)) * 1e3, 2),
        "single_potrf_l_64_gflops": round(flops_potrf(64) / (np.median(pp) * 1e-3) / 1e9, 2),
        "single_syrk_ln_64_us": round(float(np.median(ps1)) * 1e3, 2),
        "single_trsm_rltn_16x64_us": round(float(np.median(pt1)) * 1e3, 2),
        "uniform_kernel_ms_mean": round(kern_ms, 4),
        "uniform_replay_ms_median_instrumented": round(float(np.median(per)), 4),
        "uniform_replay_ms_min_instrumented": round(float(np.min(per)), 4),
        "uniform_failed_instances": bad,
    }

    print("[bench] FP64 matrix-core and HBM copy probes", file=sys.stderr, flush=True)
    peaks = measure_peaks(p, torch)
    extra["measured_peaks"] = peaks

    legs = set() if args.no_extra else {x.strip() for x in args.legs.split(",") if x.strip()}
    cpu_legs = not args.no_cpu
    tune_loaded = p.tune_cache_load(args.tune_cache) if args.tune_cache else 0
    if "uneven" in legs:
        print("[bench] uneven batch (65536 solves)", file=sys.stderr, flush=True)
        extra.update(bench_uneven(p, synth, torch, cpu=cpu_legs))
    if "riccati" in legs:
        print("[bench] Riccati batch (4096 x N=20)", file=sys.stderr, flush=True)
        extra.update(bench_riccati(p, synth, torch, cpu=cpu_legs))
    if "stacking" in legs:
        print("[bench] stacked potrf_l_mn + range-space chain (16384 x (40 + 8) x 40)", file=sys.stderr, flush=True)
        extra.update(bench_stacking(p, torch))
    if "single" in legs:
        print("[bench] single precision sgemm_nt / spotrf_l (16384 x 64)", file=sys.stderr, flush=True)
        extra.update(bench_single(p, torch))
    if "mixed" in legs:
        print("[bench] mixed precision vs FP64 (16384 x n in [128,384], 4 rhs)", file=sys.stderr, flush=True)
        extra.update(bench_mixed(p, synth, torch, cpu=cpu_legs))

    if args.tune_cache and ({"uneven", "mixed"} & legs):
        os.makedirs(os.path.dirname(os.path.abspath(args.tune_cache)), exist_ok=True)
        p.tune_cache_save(args.tune_cache)
    ent, hits, miss = p.tune_cache_stats()
    extra["tuning_cache"] = {"path": args.tune_cache or None, "entries_loaded": tune_loaded,
                             "entries": ent, "classes_from_cache": hits, "classes_timed": miss}

    if args.calib_copy:
        x = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y

    cpu = None
    if not args.no_cpu:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        ns = min(B, 16384)
        cpu, Lo, Xo = cpu_baseline_uniform(d["Q"][:ns].cpu().numpy(), d["B"][:ns].cpu().numpy(),
                                           d["RHS"][:ns].cpu().numpy(), fl, args.cpu_seconds)
        # the oracle's outputs of this leg against the GPU's, every instance
        Lg = p.unpack_batch(sL).cpu().numpy()[:ns]
        Xg = p.unpack_batch(sX).cpu().numpy()[:ns]
        cpu["parity"] = parity_vs_oracle(Lg, Xg, Lo, Xo)
        del Lg, Xg, Lo, Xo

    out = {
        "metric": "batched dpotrf+dgemm GFLOP/s & % FP64 peak; mixed vs FP64 solves/s @1e-12",
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "pct_fp64_peak": round(100 * gflops / 1e3 / FP64_PEAK_TFLOPS, 2),
        "config": {"workload": f"uniform batch: {B} x [L = chol(Q + B B^T), n=64, k=64; X = E L^-T, 16 rhs], "
                               "fused syrk_ln+potrf_l+trsm_rltn, panel-major, HBM resident",
                   "batch": B, "n": n, "k": k, "nrhs": nrhs, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved_gbs / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                     "kernel": "k_syrk_potrf_trsm<4>", "bytes_per_instance": by,
                     "frac_of_measured_copy": round(achieved_gbs / peaks["hbm_copy_gbs"], 4)},
        "cpu_baseline": cpu,
        "paper_cpu": PAPER_CPU,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
