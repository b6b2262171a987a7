"""Input generators: determinism per seed and the structure each workload
recipe promises (SPD, condition number, size ranges).  CPU only."""
import numpy as np

import synth


def test_determinism_per_seed():
    a = synth.uniform_batch(3, seed=1, n=20, k=8, nrhs=2)
    b = synth.uniform_batch(3, seed=1, n=20, k=8, nrhs=2)
    c = synth.uniform_batch(3, seed=2, n=20, k=8, nrhs=2)
    for key in a:
        assert np.array_equal(a[key], b[key])
    assert not np.array_equal(a["Q"], c["Q"])
    ns1, m1, r1 = synth.conditioned_batch(2, 1e3, seed=4, sizes=[30, 40])
    ns2, m2, r2 = synth.conditioned_batch(2, 1e3, seed=4, sizes=[30, 40])
    assert all(np.array_equal(x, y) for x, y in zip(m1, m2))
    assert np.array_equal(synth.uneven_sizes(100, seed=2), synth.uneven_sizes(100, seed=2))


def test_uniform_batch_is_spd():
    d = synth.uniform_batch(4, seed=1, n=64, k=64, nrhs=16)
    M = d["Q"] + np.einsum("bik,bjk->bij", d["B"], d["B"])
    assert np.all(np.linalg.eigvalsh(M) > 0)
    assert np.allclose(d["Q"], np.swapaxes(d["Q"], 1, 2))


def test_uneven_sizes_and_spd():
    ns = synth.uneven_sizes(4000, seed=2)
    assert set(np.unique(ns)) <= set(range(8, 257, 8)) and ns.min() == 8 and ns.max() == 256
    out = synth.uneven_batch(3, seed=2, sizes=[8, 40, 96])
    mats = out[1]
    for A, n in zip(mats, [8, 40, 96]):
        assert A.shape == (n, n) and np.allclose(A, A.T)
        assert np.linalg.eigvalsh(A).min() >= n - 1e-9  # G G^T + n I


def test_conditioned_batch_hits_target_condition():
    for cond in (1e2, 1e4, 1e6):
        ns, mats, rhs = synth.conditioned_batch(2, cond, seed=4, sizes=[50, 128])
        for A in mats:
            ev = np.linalg.eigvalsh(A)
            assert ev.min() > 0
            assert abs(np.log10(ev.max() / ev.min()) - np.log10(cond)) < 0.01
            assert np.allclose(A, A.T)
    ns = synth.conditioned_sizes(5000, seed=4)
    assert ns.min() >= 128 and ns.max() <= 384


def test_structured_integer_factor_inverse_blocks():
    """The 16x16 diagonal blocks of the structured factor have inverses with
    entries of magnitude <= 1 (times powers of two), as its docstring says."""
    L, A = synth.structured_integer_factor(48, seed=1)
    for b0 in range(0, 48, 16):
        blk = L[b0:b0 + 16, b0:b0 + 16]
        inv = np.linalg.inv(blk)
        scaled = inv * np.diag(blk)[None, :]
        assert np.all(np.abs(scaled) <= 1.0 + 1e-12)
    assert np.array_equal(A, L @ L.T)
