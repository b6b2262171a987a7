"""CPU-side checks of the C ABI: the library loads, exports every function the
header declares, and its host-only logic (memsize, create, argument checks)
behaves as documented.  No kernel is launched."""
import ctypes
import os
import re

import pytest

import paper_1704_02457_amd as p

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "blasfeo_hip.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(blasfeo_\w+)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = p.lib()
    declared = _declared_functions()
    assert len(declared) >= 30
    for name in declared:
        assert hasattr(L, name), name
    # and the binding declares a signature for each of them
    assert set(declared) <= set(p.exported_symbols())


def _mk(m, n, addr=0x100000):
    s = p.blasfeo_dmat()
    p.lib().blasfeo_create_dmat(m, n, ctypes.byref(s), ctypes.c_void_p(addr))
    return s


@pytest.mark.parametrize("m,n", [(0, 0), (1, 1), (16, 16), (17, 3), (64, 64), (40, 40), (300, 7)])
def test_memsize_and_create(m, n):
    L = p.lib()
    ms = L.blasfeo_memsize_dmat(m, n)
    cn = (n + 3) // 4 * 4
    pm = (m + 15) // 16
    expect = pm * 16 * cn * 8 + max(m, n) * 8
    expect = (expect + 255) // 256 * 256
    assert ms == expect and ms % 256 == 0
    s = _mk(m, n, 0x200000)
    assert (s.m, s.n, s.cn, s.pm, s.memsize, s.use_dA) == (m, n, cn, pm, ms, 0)
    assert s.pA == 0x200000
    if pm * cn:
        assert s.dA == 0x200000 + pm * 16 * cn * 8


def test_memsize_errors_and_dvec():
    L = p.lib()
    assert L.blasfeo_memsize_dmat(-1, 3) == -1
    assert L.blasfeo_memsize_dvec(-2) == -1
    assert L.blasfeo_memsize_dvec(17) == 256
    assert L.blasfeo_memsize_dvec(33) == 512


def test_create_does_not_touch_memory():
    # a pointer that is not mapped anywhere: create must only record it
    s = _mk(32, 32, addr=0x10)
    assert s.pA == 0x10


def test_batched_argument_errors_before_launch():
    L = p.lib()
    A = _mk(64, 64)
    X = _mk(16, 64)
    small = _mk(8, 8)
    r = lambda s: ctypes.byref(s)
    f = L.blasfeo_hip_dsyrk_dpotrf_trsm_batched
    assert f(-1, 64, 64, 16, r(A), r(A), r(X), r(A), r(X), None, None) == -1
    assert f(1, 65, 64, 16, r(A), r(A), r(X), r(A), r(X), None, None) == -2
    assert f(1, 64, -1, 16, r(A), r(A), r(X), r(A), r(X), None, None) == -3
    assert f(1, 64, 64, 17, r(A), r(A), r(X), r(A), r(X), None, None) == -4
    assert f(1, 64, 64, 16, r(small), r(A), r(X), r(A), r(X), None, None) == -5
    assert f(1, 64, 64, 16, r(A), r(small), r(X), r(A), r(X), None, None) == -6
    assert f(1, 64, 64, 16, r(A), r(A), r(small), r(A), r(X), None, None) == -7
    assert f(1, 64, 64, 16, r(A), r(A), r(X), r(small), r(X), None, None) == -8
    g = L.blasfeo_hip_dgemm_nt_batched
    # B operand (n x k) out of bounds of its matrix
    assert g(1, 64, 64, 64, 1.0, r(A), 0, 0, r(A), 1, 0, 1.0, r(A), 0, 0, r(A), 0, 0, None) == -9
    assert g(1, 64, 64, 64, 1.0, r(A), 0, 0, r(A), 0, 0, 1.0, r(A), 0, 0, r(small), 0, 0, None) == -16
    assert L.blasfeo_hip_dpotrf_l_batched(1, 9, r(small), 0, 0, r(small), 0, 0, None, None) == -3
    # plan entry points without a plan
    assert L.blasfeo_hip_plan_workspace(None, None, None) == -1
    assert L.blasfeo_hip_dposv_mixed_vbatched(None, 1, 1e-12, 10, None, None, None, None, None,
                                              None, None, None, None, None) == -1
    assert L.blasfeo_hip_plan_mixed_factor(None, 0, None, None, 1, None) == -1
    assert L.blasfeo_hip_dposv_vbatched(None, None, None, None, None, None, None, None) == -1
    assert L.blasfeo_hip_plan_capture(None, None, None, None, None, None, None) == -1


def test_single_routine_errors_recorded():
    L = p.lib()
    A = _mk(16, 16)
    L.blasfeo_hip_get_last_error()
    L.blasfeo_dgemm_nt(16, 16, 17, 1.0, ctypes.byref(A), 0, 0, ctypes.byref(A), 0, 0, 1.0,
                       ctypes.byref(A), 0, 0, ctypes.byref(A), 0, 0)
    assert L.blasfeo_hip_get_last_error() == -5
    assert L.blasfeo_hip_get_last_error() == 0
    L.blasfeo_dpotrf_l(-1, ctypes.byref(A), 0, 0, ctypes.byref(A), 0, 0)
    assert L.blasfeo_hip_get_last_error() == -1
    assert L.blasfeo_hip_strerror(-5) == b"invalid argument 5"


def test_header_compiles_as_c_and_cxx(tmp_path):
    """The boundary header is plain C: it compiles on its own with a C and a
    C++ compiler (no HIP or torch types in the signatures)."""
    import shutil
    import subprocess
    inc = os.path.join(ROOT, "include")
    src = tmp_path / "use.c"
    src.write_text('#include "blasfeo_hip.h"\nint main(void) { struct blasfeo_dmat m; (void)m; '
                   'return blasfeo_memsize_dmat(4, 4) > 0 ? 0 : 1; }\n')
    for cc, std in (("gcc", "-std=c99"), ("g++", "-std=c++17")):
        if shutil.which(cc) is None:
            pytest.skip(f"{cc} not available")
        r = subprocess.run([cc, std, "-Wall", "-Werror", "-fsyntax-only", "-I", inc,
                            "-x", "c" if cc == "gcc" else "c++", str(src)], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr


@pytest.mark.parametrize("m,n", [(0, 0), (1, 1), (32, 32), (33, 5), (64, 64), (100, 7)])
def test_smat_memsize_and_create(m, n):
    """Single precision: 32-float panels, cn = round_up(n, 4), dA after the
    panels, memsize a multiple of 256 bytes."""
    L = p.lib()
    ms = L.blasfeo_memsize_smat(m, n)
    cn, pm = (n + 3) // 4 * 4, (m + 31) // 32
    expect = (pm * 32 * cn * 4 + max(m, n) * 4 + 255) // 256 * 256
    assert ms == expect
    s = p.blasfeo_smat()
    L.blasfeo_create_smat(m, n, ctypes.byref(s), ctypes.c_void_p(0x300000))
    assert (s.m, s.n, s.cn, s.pm, s.memsize, s.use_dA) == (m, n, cn, pm, ms, 0)
    assert s.pA == 0x300000
    if pm * cn:
        assert s.dA == 0x300000 + pm * 32 * cn * 4
    assert L.blasfeo_memsize_smat(-1, 2) == -1


def test_single_batched_argument_errors_before_launch():
    L = p.lib()
    s = p.blasfeo_smat()
    L.blasfeo_create_smat(8, 8, ctypes.byref(s), ctypes.c_void_p(0x100000))
    r = ctypes.byref(s)
    g = L.blasfeo_hip_sgemm_nt_batched
    assert g(-1, 8, 8, 8, 1.0, r, 0, 0, r, 0, 0, 1.0, r, 0, 0, r, 0, 0, None) == -1
    assert g(1, 9, 8, 8, 1.0, r, 0, 0, r, 0, 0, 1.0, r, 0, 0, r, 0, 0, None) == -6
    assert g(1, 8, 8, 8, 1.0, r, 0, 0, r, 1, 0, 1.0, r, 0, 0, r, 0, 0, None) == -9
    assert g(1, 8, 8, 8, 1.0, r, 0, 0, r, 0, 0, 1.0, r, 0, 1, r, 0, 0, None) == -13
    assert g(1, 8, 8, 8, 1.0, r, 0, 0, r, 0, 0, 1.0, r, 0, 0, None, 0, 0, None) == -16
    y = L.blasfeo_hip_ssyrk_ln_batched
    assert y(1, 8, 9, 1.0, r, 0, 0, r, 0, 0, 1.0, r, 0, 0, r, 0, 0, None) == -5
    assert y(1, 8, 8, 1.0, r, 0, 0, r, 0, 0, 1.0, r, 1, 0, r, 0, 0, None) == -12
    f = L.blasfeo_hip_spotrf_l_batched
    assert f(70000, 8, r, 0, 0, r, 0, 0, None, None) == -1
    assert f(1, -1, r, 0, 0, r, 0, 0, None, None) == -2
    assert f(1, 8, r, 1, 0, r, 0, 0, None, None) == -3
    assert f(1, 8, r, 0, 0, r, 0, 1, None, None) == -6
    assert f(0, 8, r, 0, 0, r, 0, 0, None, None) == 0


def test_tune_cache_file_round_trip(tmp_path):
    """The tuning cache's file format: load merges, save writes every entry
    (one line each, sorted), malformed lines and invalid configurations are
    rejected without merging anything, a missing file is an empty cache."""
    p.tune_cache_clear()
    assert p.tune_cache_stats() == (0, 0, 0)
    assert p.tune_cache_load(str(tmp_path / "none.txt")) == 0
    src = tmp_path / "in.txt"
    src.write_text("# comment\n"
                   "gfx950:sramecc+:xnack- 256 0 4 8192 193 384 2359296 202 7.5000\n"
                   "\n"
                   "  gfx950:sramecc+:xnack- 256 2 1 900 17 32 22000 4 0.0500\n"
                   "gfx950:sramecc+:xnack- 256 0 4 8192 128 192 1310720 211 3.2500")
    assert p.tune_cache_load(str(src)) == 3
    assert p.tune_cache_stats()[0] == 3
    out = tmp_path / "out.txt"
    assert p.tune_cache_save(str(out)) == 3
    lines = out.read_text().splitlines()
    assert lines[0].startswith("#") and len(lines) == 4
    assert sorted(lines[1:]) == sorted([
        "gfx950:sramecc+:xnack- 256 0 4 8192 193 384 2359296 202 7.5000",
        "gfx950:sramecc+:xnack- 256 2 1 900 17 32 22000 4 0.0500",
        "gfx950:sramecc+:xnack- 256 0 4 8192 128 192 1310720 211 3.2500"])
    # the same key again replaces its value; a new key adds one
    upd = tmp_path / "upd.txt"
    upd.write_text("gfx950:sramecc+:xnack- 256 2 1 900 17 32 22000 2 0.0400\n"
                   "gfx942 304 1 1 10 8 16 120 1 0.0100\n")
    assert p.tune_cache_load(str(upd)) == 2
    assert p.tune_cache_save(str(out)) == 4
    assert "gfx950:sramecc+:xnack- 256 2 1 900 17 32 22000 2 0.0400" in out.read_text()
    # rejected files leave the table as it was
    for bad in ["gfx950 256 0 4 10 100 200 1500 3 1.0\n",      # cfg 3 invalid for n > 64
                "gfx950 256 2 1 10 17 32 250 8 1.0\n",         # cfg 8 invalid for a small class
                "gfx950 256 7 1 10 17 32 250 1 1.0\n",         # no class kind 7
                "gfx950 256 0 4 10 100\n",                     # too few fields
                "gfx950 256 0 4 10 100 200 1500 202 1.0 9\n",  # trailing field
                "gfx950 256 0 4 10 200 100 1500 202 1.0\n",    # nmax < nmin
                "gfx950 256 0 4 0 100 200 1500 202 1.0\n",     # no instances
                "x" * 600 + "\n"]:                            # longer than a line may be
        f = tmp_path / "bad.txt"
        f.write_text("gfx9 1 1 0 1 1 1 1 1 0.1\n" + bad)
        with pytest.raises(p.HipError):
            p.tune_cache_load(str(f))
        assert p.tune_cache_stats()[0] == 4
    with pytest.raises(p.HipError):
        p.tune_cache_save(str(tmp_path / "no_such_dir" / "x.txt"))
    p.tune_cache_clear()
    assert p.tune_cache_stats() == (0, 0, 0)
