"""Shared helpers of the GPU tests (host side only)."""
import sys

import numpy as np

TOL = 1e-13  # relative Frobenius error allowed per unit of the order n


def note(*args):
    """Print the case about to run on the GPU (flushed, so a crash names it)."""
    print("[case]", *args, flush=True)
    sys.stdout.flush()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def assert_parity(gpu, ref, n, what=""):
    e = rel(gpu, ref)
    assert e <= TOL * max(n, 1), f"{what}: rel Frobenius error {e:.3e} > {TOL * max(n, 1):.1e}"
    return e
