"""Chunked comparison of full-size batches with the oracle.

TEST INFRASTRUCTURE ONLY (the parity tests and the CPU leg of the benchmark).
Every function takes host numpy arrays (C-order stacks of instances), runs the
oracle's OpenMP drivers on them and returns the largest per-instance errors,
so that every instance of a workload can be checked chunk by chunk.  The
parity metric is the relative Frobenius error ||G - R||_F / ||R||_F of each
instance (the factor's lower triangle, the solution block).
"""
import time

import numpy as np

from . import batch_berr_uniform, batch_dposv_uniform, batch_ric_trf, batch_syrk_potrf_trsm


def rel_err(G, R):
    """Per-instance relative Frobenius error over the last two axes."""
    G = np.asarray(G, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    num = np.linalg.norm((G - R).reshape(G.shape[0], -1), axis=1)
    den = np.linalg.norm(R.reshape(R.shape[0], -1), axis=1)
    return num / np.where(den > 0, den, 1.0)


class Worst:
    """Running maxima (NaN-propagating) of named error measures, plus the
    instance count and the oracle's own time and thread count."""

    def __init__(self):
        self.v = {}
        self.instances = 0
        self.oracle_s = 0.0
        self.threads = 0

    def add(self, name, errs):
        e = float(np.max(errs)) if np.size(errs) else 0.0
        if np.isnan(errs).any():
            e = float("nan")
        old = self.v.get(name, 0.0)
        self.v[name] = e if (np.isnan(e) or e > old) else old

    def merge(self, other):
        """Fold another Worst (e.g. of one size class) into this one."""
        for k, v in other.v.items():
            self.add(k, np.asarray([v]))
        self.instances += other.instances
        self.oracle_s += other.oracle_s
        self.threads = max(self.threads, other.threads)

    def __getitem__(self, k):
        return self.v[k]

    def as_dict(self):
        d = {k: float(v) for k, v in self.v.items()}
        d["instances"] = int(self.instances)
        return d


def dposv_chunk(w, A, B, Lg, dAg, Xg, nthreads=0, gpu_info=None, detail=None):
    """One chunk of Cholesky solves of a single order n: A (b,n,n), B, Xg
    (b,n,nrhs), Lg (b,n,n) lower, dAg (b,n).  Records L, dA, X errors against
    the oracle and the oracle's backward error of the GPU's X ("eta").  With
    a dict `detail`, also stores the per-instance X errors ("X"), the GPU's
    and the oracle's own backward errors ("eta", "eta_orc")."""
    t0 = time.perf_counter()
    Lr, Xr, dAr, infr, used = batch_dposv_uniform(A, B, nthreads=nthreads)
    eta, _ = batch_berr_uniform(A, Xg, B, nthreads=nthreads)
    if detail is not None:
        detail["eta"] = eta
        detail["eta_orc"] = batch_berr_uniform(A, Xr, B, nthreads=nthreads)[0]
        detail["X"] = rel_err(Xg, Xr)
    w.oracle_s += time.perf_counter() - t0
    w.threads = max(w.threads, used)
    assert np.all(infr == 0), "oracle: non-SPD instance in a chunk"
    if gpu_info is not None:
        assert np.array_equal(np.asarray(gpu_info), infr), "info codes differ"
    w.add("L", rel_err(np.tril(Lg), Lr))
    w.add("dA", rel_err(dAg[:, None, :], dAr[:, None, :]))
    w.add("X", rel_err(Xg, Xr))
    w.add("eta", eta)
    w.instances += A.shape[0]
    return w


def eta_chunk(w, A, B, Xg, name="eta", nthreads=0):
    """Oracle backward error of the GPU's solutions Xg (b,n,nrhs)."""
    t0 = time.perf_counter()
    eta, used = batch_berr_uniform(A, Xg, B, nthreads=nthreads)
    w.oracle_s += time.perf_counter() - t0
    w.threads = max(w.threads, used)
    w.add(name, eta)
    w.instances += A.shape[0]
    return eta


def fused_chunk(w, Q, Bk, E, Lg, Xg, dAg, nthreads=0):
    """One chunk of the uniform fused workload: L = chol(Q + B B^T),
    X = E L^-T.  Returns the oracle's L and X of the chunk."""
    t0 = time.perf_counter()
    Lr, Xr, dAr, infr, used = batch_syrk_potrf_trsm(Q, Bk, E, nthreads=nthreads)
    w.oracle_s += time.perf_counter() - t0
    w.threads = max(w.threads, used)
    assert np.all(infr == 0)
    w.add("L", rel_err(np.tril(Lg), Lr))
    w.add("X", rel_err(Xg, Xr))
    w.add("dA", rel_err(dAg[:, None, :], dAr[:, None, :]))
    w.instances += Q.shape[0]
    return Lr, Xr


def riccati_chunk(w, d, N, Fg, nthreads=0):
    """Chunk of Riccati recursions: d holds A, B, Q, R, PN stacks; Fg
    (b,N,nm,nm) the GPU's stage factors.  Records the worst stage error."""
    t0 = time.perf_counter()
    Fr, infr, used = batch_ric_trf(d["A"], d["B"], d["Q"], d["R"], d["PN"], N, nthreads=nthreads)
    w.oracle_s += time.perf_counter() - t0
    w.threads = max(w.threads, used)
    assert np.all(infr == 0)
    b = Fg.shape[0]
    nm = Fg.shape[-1]
    w.add("F", rel_err(np.tril(Fg).reshape(b * N, nm, nm), Fr.reshape(b * N, nm, nm)))
    w.instances += b
    return Fr
