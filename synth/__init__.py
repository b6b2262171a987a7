"""Seeded synthetic inputs for the five workloads of the panel-major routines.

This module only draws random numbers and assembles test matrices from them
(sums, scalings and, where a recipe asks for an SPD matrix, one product G*G^T).
It holds none of the arithmetic of the routines under test, and both the CPU
oracle and the HIP path receive exactly the arrays produced here.

Two generators are provided:

* numpy ``default_rng(seed)`` (PCG64) for the small cases used on the CPU and in
  the element-by-element parity tests; draws happen in the order the recipe
  lists the matrices, each as one vectorised draw over the whole batch;
* torch's device generator (Philox) for full-size batches that are built
  directly in device memory (``*_device`` functions).  A full-size parity test
  copies the sampled instances back to the host and hands those bytes to the
  oracle.

All matrices are returned in "C order" stacks (batch, rows, cols) of float64.
"""
import numpy as np

# --------------------------------------------------------------------------
# Workload 1: single instance, gemm_nt 64x64x64 then potrf_l of 64x64 SPD
# --------------------------------------------------------------------------

def single(seed=0, n=64):
    """A, B, C ~ U[-1,1] (n x n); then M ~ U[-1,1] and S = M M^T + n I."""
    rng = np.random.default_rng(seed)
    A = rng.uniform(-1.0, 1.0, (n, n))
    B = rng.uniform(-1.0, 1.0, (n, n))
    C = rng.uniform(-1.0, 1.0, (n, n))
    M = rng.uniform(-1.0, 1.0, (n, n))
    S = M @ M.T + n * np.eye(n)
    S = 0.5 * (S + S.T)
    return dict(A=A, B=B, C=C, M=M, S=S)


# --------------------------------------------------------------------------
# Workload 2: uniform batch, L = chol(Q + B B^T), X = RHS L^-T
# --------------------------------------------------------------------------

def uniform_batch(batch, seed=1, n=64, k=64, nrhs=16):
    """Q = diag(U[1,2]) + 0.01 sym(G), B = randn(n,k)/8, RHS = randn(nrhs,n)."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(1.0, 2.0, (batch, n))
    G = rng.standard_normal((batch, n, n))
    B = rng.standard_normal((batch, n, k)) / 8.0
    R = rng.standard_normal((batch, nrhs, n))
    Q = 0.01 * 0.5 * (G + np.swapaxes(G, 1, 2))
    idx = np.arange(n)
    Q[:, idx, idx] += d
    return dict(Q=Q, B=B, RHS=R)


def uniform_batch_device(batch, seed=1, n=64, k=64, nrhs=16, device="cuda"):
    """Same recipe as :func:`uniform_batch`, drawn on the device."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    f = dict(device=device, dtype=torch.float64, generator=g)
    d = torch.rand((batch, n), **f) + 1.0
    G = torch.randn((batch, n, n), **f)
    B = torch.randn((batch, n, k), **f) / 8.0
    R = torch.randn((batch, nrhs, n), **f)
    Q = 0.005 * (G + G.transpose(1, 2))
    del G
    Q.diagonal(dim1=1, dim2=2).add_(d)
    return dict(Q=Q, B=B, RHS=R)


# --------------------------------------------------------------------------
# Workload 3: uneven batch of SPD solves, n in {8, 16, ..., 256}
# --------------------------------------------------------------------------

def uneven_sizes(batch, seed=2, step=8, nmax=256):
    rng = np.random.default_rng(seed)
    return (step * rng.integers(1, nmax // step + 1, batch)).astype(np.int32)


def uneven_batch(batch, seed=2, step=8, nmax=256, sizes=None):
    """n = 8*U{1..32}; A = G G^T + n I with G randn(n,n); b = randn(n).

    After the sizes, G and b are drawn instance by instance in batch order.
    """
    rng = np.random.default_rng(seed)
    ns = (step * rng.integers(1, nmax // step + 1, batch)).astype(np.int32) if sizes is None else np.asarray(sizes, np.int32)
    mats, rhs = [], []
    for n in ns:
        G = rng.standard_normal((n, n))
        b = rng.standard_normal(n)
        A = G @ G.T + n * np.eye(n)
        mats.append(0.5 * (A + A.T))
        rhs.append(b)
    return ns, mats, rhs


def uneven_batch_device(ns, seed=2, device="cuda"):
    """Device version: for each size class (ascending n) draw G (count,n,n)
    then b (count,n), and form A = G G^T + n I.  Returns a dict n -> (idx, A, b)
    where idx are the batch positions of that size class."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    ns = np.asarray(ns)
    out = {}
    for n in np.unique(ns):
        idx = np.nonzero(ns == n)[0]
        cnt = len(idx)
        G = torch.randn((cnt, int(n), int(n)), device=device, dtype=torch.float64, generator=g)
        b = torch.randn((cnt, int(n)), device=device, dtype=torch.float64, generator=g)
        A = torch.bmm(G, G.transpose(1, 2).contiguous())
        del G
        A = 0.5 * (A + A.transpose(1, 2))
        A.diagonal(dim1=1, dim2=2).add_(float(n))
        out[int(n)] = (idx, A, b)
    return out


# --------------------------------------------------------------------------
# Workload 4: batch of backward Riccati recursions
# --------------------------------------------------------------------------

def riccati_batch(batch, seed=3, nx=32, nu=8):
    """A = I + 0.05 randn(nx,nx), B = randn(nx,nu)/4, Q = I, R = 0.1 I, P_N = I."""
    rng = np.random.default_rng(seed)
    A = np.eye(nx)[None] + 0.05 * rng.standard_normal((batch, nx, nx))
    B = rng.standard_normal((batch, nx, nu)) / 4.0
    Q = np.broadcast_to(np.eye(nx), (batch, nx, nx)).copy()
    R = np.broadcast_to(0.1 * np.eye(nu), (batch, nu, nu)).copy()
    PN = np.broadcast_to(np.eye(nx), (batch, nx, nx)).copy()
    return dict(A=A, B=B, Q=Q, R=R, PN=PN)


# --------------------------------------------------------------------------
# Workload 5: SPD systems with prescribed condition number, 4 right-hand sides
# --------------------------------------------------------------------------

def spectrum(n, cond):
    """sigma_i = cond^(-i/(n-1)), i = 0..n-1 (geometric, sigma_0 = 1)."""
    if n == 1:
        return np.ones(1)
    return cond ** (-np.arange(n) / (n - 1.0))


def conditioned_batch(batch, cond, seed=4, nmin=128, nmax=384, nrhs=4, sizes=None):
    """n ~ U{nmin..nmax}; A = U diag(sigma) U^T with U from QR(randn(n,n));
    B = randn(n, nrhs).  Sizes first, then per instance G then B."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(nmin, nmax + 1, batch).astype(np.int32) if sizes is None else np.asarray(sizes, np.int32)
    mats, rhs = [], []
    for n in ns:
        G = rng.standard_normal((n, n))
        b = rng.standard_normal((n, nrhs))
        U, _ = np.linalg.qr(G)
        A = (U * spectrum(n, cond)) @ U.T
        mats.append(0.5 * (A + A.T))
        rhs.append(b)
    return ns, mats, rhs


def conditioned_sizes(batch, seed=4, nmin=128, nmax=384):
    """n ~ U{nmin..nmax} (the sizes of conditioned_batch)."""
    return np.random.default_rng(seed).integers(nmin, nmax + 1, batch).astype(np.int32)


def orthogonal_batch_device(ns, seed=4, nrhs=4, device="cuda"):
    """Per size class (ascending n): G (count,n,n) randn, then B (count,n,nrhs)
    randn; U = the orthogonal factor of G = U R.  U is computed by two passes
    of Cholesky QR (G <- G R^-1 with R^T R = G^T G), which gives the Q of a
    Householder QR up to the signs of its columns -- signs that cancel in
    U diag(sigma) U^T.  Classes whose Gram matrix is too ill-conditioned for
    Cholesky QR use Householder QR.  Returns n -> (idx, U, B)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    ns = np.asarray(ns)
    out = {}
    for n in np.unique(ns):
        idx = np.nonzero(ns == n)[0]
        cnt, n = len(idx), int(n)
        G = torch.randn((cnt, n, n), device=device, dtype=torch.float64, generator=g)
        B = torch.randn((cnt, n, nrhs), device=device, dtype=torch.float64, generator=g)
        U = G
        ok = True
        for _ in range(2):
            gram = torch.bmm(U.transpose(1, 2).contiguous(), U)
            Lg, info = torch.linalg.cholesky_ex(gram)
            if bool((info != 0).any()):
                ok = False
                break
            U = torch.linalg.solve_triangular(Lg.transpose(1, 2).contiguous(), U, upper=True, left=False)
        if not ok:
            U, _ = torch.linalg.qr(G)
        out[n] = (idx, U, B)
    return out


def conditioned_from_orthogonal(U, cond):
    """A = U diag(sigma) U^T (symmetrized) for a (count,n,n) orthogonal U."""
    import torch
    n = U.shape[-1]
    s = torch.as_tensor(spectrum(n, cond), device=U.device, dtype=U.dtype)
    A = torch.bmm(U * s[None, None, :], U.transpose(1, 2).contiguous())
    return 0.5 * (A + A.transpose(1, 2))


def conditioned_batch_device(ns, cond, seed=4, nrhs=4, device="cuda"):
    """Device version of conditioned_batch: n -> (idx, A, B) per size class
    (ascending n), A = U diag(sigma) U^T with U from orthogonal_batch_device."""
    out = {}
    for n, (idx, U, B) in orthogonal_batch_device(ns, seed, nrhs, device).items():
        out[n] = (idx, conditioned_from_orthogonal(U, cond), B)
    return out


# --------------------------------------------------------------------------
# Closed-form test matrices
# --------------------------------------------------------------------------

def small_integer_factor(n, seed=11, diag=(1.0, 2.0, 4.0), off=3):
    """Lower triangular L with diagonal drawn from ``diag`` and integer
    off-diagonal entries in [-off, off]; returns (L, A = L L^T).

    With power-of-two diagonals every product, partial sum and reciprocal in
    the Cholesky factorization of A is exact in FP64 (for moderate n), so any
    correctly rounded implementation must reproduce L bit for bit."""
    rng = np.random.default_rng(seed)
    L = np.tril(rng.integers(-off, off + 1, (n, n)).astype(np.float64), -1)
    L[np.arange(n), np.arange(n)] = rng.choice(np.asarray(diag, dtype=np.float64), n)
    return L, L @ L.T


def structured_integer_factor(n, seed=0, diag=(1.0, 2.0)):
    """Lower L with power-of-two diagonal, 16x16 diagonal blocks bidiagonal
    (+-1 on the subdiagonal), entries of -1, 0, 1 below the diagonal blocks.
    The inverse of every diagonal block then has entries of magnitude <= 1
    times powers of two, so blocked and unblocked Cholesky in binary32 and
    binary16 arithmetic all reproduce L exactly."""
    rng = np.random.default_rng(seed)
    L = np.tril(rng.integers(-1, 2, (n, n)).astype(np.float64), -1)
    for b0 in range(0, n, 16):
        b1 = min(n, b0 + 16)
        L[b0:b1, b0:b1] = 0.0
        for i in range(b0 + 1, b1):
            L[i, i - 1] = rng.choice([-1.0, 1.0])
    L[np.arange(n), np.arange(n)] = rng.choice(np.asarray(diag), n)
    return L, L @ L.T
