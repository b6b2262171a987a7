"""Independent decoder of the panel-major matrix format (§4.3 of the paper).

TEST INFRASTRUCTURE ONLY.  The tests use it to read raw device buffers written
by the library and to check the library's own pack/unpack kernels.

Panel-major storage (§4.3, "Panel-major matrix format"): rows are grouped in
horizontal panels of ``ps`` rows (a power of two).  Inside a panel the storage
is column-major with leading dimension ``ps``; consecutive panels are ``ps*sda``
elements apart, where ``sda`` (the structure member ``cn``) is the panel
length, at least the number of columns.  The element (i, j) therefore sits at

    (i - i % ps) * sda + j * ps + i % ps

which is the paper's first-element formula for the sub-matrix at (ai, aj).
"""
import numpy as np


def offset(i, j, sda, ps):
    """Element offset of (i, j) in a panel-major buffer (§4.3)."""
    air = i & (ps - 1)
    return (i - air) * sda + j * ps + air


def n_panels(m, ps):
    return (m + ps - 1) // ps


def pack(A, sda, ps, fill=0.0, out=None):
    """Column-major (m, n) array -> flat panel-major buffer of pm*ps*sda elements.

    Padding rows of the last panel and padding columns get ``fill``.
    """
    A = np.asarray(A)
    m, n = A.shape
    assert sda >= n
    pm = n_panels(m, ps)
    buf = np.full(pm * ps * sda, fill, dtype=A.dtype) if out is None else out
    for i in range(m):
        base = offset(i, 0, sda, ps)
        buf[base: base + n * ps: ps] = A[i, :]
    return buf


def unpack(buf, m, n, sda, ps):
    """Flat panel-major buffer -> (m, n) array."""
    buf = np.asarray(buf)
    out = np.empty((m, n), dtype=buf.dtype)
    for i in range(m):
        base = offset(i, 0, sda, ps)
        out[i, :] = buf[base: base + n * ps: ps]
    return out
