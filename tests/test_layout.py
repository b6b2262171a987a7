"""The independent panel-major decoder (oracle/panel.py) against the address
formula of §4.3 evaluated by hand and by brute-force enumeration.  CPU only."""
import os

import numpy as np
import pytest

from oracle import panel

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_golden_offsets_5x3_ps4():
    rows = []
    ps = sda = None
    with open(os.path.join(GOLD, "panel_5x3_ps4.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, *v = line.split()
            if k == "ps":
                ps = int(v[0])
            elif k == "sda":
                sda = int(v[0])
            else:
                rows.append([int(x) for x in v])
    for i, r in enumerate(rows):
        for j, o in enumerate(r):
            assert panel.offset(i, j, sda, ps) == o
    A = np.arange(15.0).reshape(5, 3)
    buf = panel.pack(A, sda, ps, fill=-1.0)
    assert buf.size == 2 * ps * sda
    for i in range(5):
        for j in range(3):
            assert buf[rows[i][j]] == A[i, j]


@pytest.mark.parametrize("ps", [4, 16, 32])
@pytest.mark.parametrize("m,n", [(1, 1), (5, 3), (17, 9), (40, 33)])
def test_offsets_brute_force(ps, m, n):
    """Enumerate the storage order: panel by panel, column by column inside a
    panel, ps consecutive rows per column (the memory walk of the figure in
    §4.3), and compare with the closed formula."""
    sda = n + 3
    expect = {}
    pos = 0
    for p in range((m + ps - 1) // ps):
        for j in range(sda):
            for r in range(ps):
                i = p * ps + r
                if i < m and j < n:
                    expect[(i, j)] = pos
                pos += 1
    for (i, j), o in expect.items():
        assert panel.offset(i, j, sda, ps) == o


def test_pack_unpack_round_trip_and_submatrix():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((37, 21))
    buf = panel.pack(A, 24, 16)
    assert np.array_equal(panel.unpack(buf, 37, 21, 24, 16), A)
    # sub-matrix at (ai, aj) = (5, 3): first element sits at offset(5, 3)
    ai, aj = 5, 3
    assert buf[panel.offset(ai, aj, 24, 16)] == A[ai, aj]
