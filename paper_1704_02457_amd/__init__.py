"""Python binding of libblasfeo_hip.so, an MI355X (gfx950) library of panel-major
dense linear algebra routines after BLASFEO (arXiv 1704.02457).

This layer only marshals arguments: every computation runs in the HIP kernels
of the shared library, reached through its C ABI (include/blasfeo_hip.h).
PyTorch is used for device memory (``torch.empty(..., device="cuda")``) and
streams.  If the library is not built, or no GPU is present, the compute
functions raise; there is no CPU fallback.

Function names are those of the C ABI.  A ``DMat`` carries a device buffer and
the ``struct blasfeo_dmat`` describing it; a ``DMatBatch`` is a uniform batch
(instance b starts ``memsize`` bytes after instance b-1) whose struct describes
instance 0, as the batched entry points expect.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libblasfeo_hip.so")
PS = 16

_lib = None


class blasfeo_dmat(ctypes.Structure):
    _fields_ = [("pA", ctypes.c_void_p), ("dA", ctypes.c_void_p), ("m", ctypes.c_int),
                ("n", ctypes.c_int), ("pm", ctypes.c_int), ("cn", ctypes.c_int),
                ("use_dA", ctypes.c_int), ("memsize", ctypes.c_int)]


class blasfeo_dvec(ctypes.Structure):
    _fields_ = [("pa", ctypes.c_void_p), ("m", ctypes.c_int), ("pm", ctypes.c_int),
                ("memsize", ctypes.c_int)]


class blasfeo_smat(ctypes.Structure):
    _fields_ = [("pA", ctypes.c_void_p), ("dA", ctypes.c_void_p), ("m", ctypes.c_int),
                ("n", ctypes.c_int), ("pm", ctypes.c_int), ("cn", ctypes.c_int),
                ("use_dA", ctypes.c_int), ("memsize", ctypes.c_int)]


_M = ctypes.POINTER(blasfeo_dmat)
_S = ctypes.POINTER(blasfeo_smat)
_V = ctypes.POINTER(blasfeo_dvec)
_i, _d, _p, _ll = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_longlong
_f = ctypes.c_float

# name -> (restype, argtypes)
_SIGS = {
    "blasfeo_memsize_dmat": (_i, [_i, _i]),
    "blasfeo_memsize_dvec": (_i, [_i]),
    "blasfeo_create_dmat": (None, [_i, _i, _M, _p]),
    "blasfeo_create_dvec": (None, [_i, _V, _p]),
    "blasfeo_allocate_dmat": (None, [_i, _i, _M]),
    "blasfeo_free_dmat": (None, [_M]),
    "blasfeo_allocate_dvec": (None, [_i, _V]),
    "blasfeo_free_dvec": (None, [_V]),
    "blasfeo_pack_dmat": (None, [_i, _i, _p, _i, _M, _i, _i]),
    "blasfeo_unpack_dmat": (None, [_i, _i, _M, _i, _i, _p, _i]),
    "blasfeo_pack_dvec": (None, [_i, _p, _V, _i]),
    "blasfeo_unpack_dvec": (None, [_i, _V, _i, _p]),
    "blasfeo_dgemm_nt": (None, [_i, _i, _i, _d, _M, _i, _i, _M, _i, _i, _d, _M, _i, _i, _M, _i, _i]),
    "blasfeo_dgemm_nn": (None, [_i, _i, _i, _d, _M, _i, _i, _M, _i, _i, _d, _M, _i, _i, _M, _i, _i]),
    "blasfeo_dsyrk_ln": (None, [_i, _i, _d, _M, _i, _i, _M, _i, _i, _d, _M, _i, _i, _M, _i, _i]),
    "blasfeo_dtrsm_rltn": (None, [_i, _i, _d, _M, _i, _i, _M, _i, _i, _M, _i, _i]),
    "blasfeo_dtrmm_rlnn": (None, [_i, _i, _d, _M, _i, _i, _M, _i, _i, _M, _i, _i]),
    "blasfeo_dpotrf_l": (None, [_i, _M, _i, _i, _M, _i, _i]),
    "blasfeo_dpotrf_l_mn": (None, [_i, _i, _M, _i, _i, _M, _i, _i]),
    "blasfeo_dgetrf_pivot": (None, [_i, _i, _M, _i, _i, _M, _i, _i, _p]),
    "blasfeo_dgetrf_nopivot": (None, [_i, _i, _M, _i, _i, _M, _i, _i]),
    "blasfeo_dgelqf": (None, [_i, _i, _M, _i, _i, _M, _i, _i]),
    "blasfeo_dsyrk_dpotrf_ln": (None, [_i, _i, _M, _i, _i, _M, _i, _i, _M, _i, _i, _M, _i, _i]),
    "blasfeo_hip_dpotrf_l_info": (None, [_i, _M, _i, _i, _M, _i, _i, _p]),
    "blasfeo_hip_dsyrk_dpotrf_ln_info": (None, [_i, _i, _M, _i, _i, _M, _i, _i, _M, _i, _i, _M, _i, _i, _p]),
    "blasfeo_hip_set_stream": (None, [_p]),
    "blasfeo_hip_get_stream": (_p, []),
    "blasfeo_hip_get_last_error": (_i, []),
    "blasfeo_hip_strerror": (ctypes.c_char_p, [_i]),
    "blasfeo_hip_version": (_i, []),
    "blasfeo_hip_pack_dmat_batched": (_i, [_i, _i, _i, _p, _i, _ll, _M, _i, _i, _p]),
    "blasfeo_hip_unpack_dmat_batched": (_i, [_i, _i, _i, _M, _i, _i, _p, _i, _ll, _p]),
    "blasfeo_hip_dgemm_nt_batched": (_i, [_i, _i, _i, _i, _d, _M, _i, _i, _M, _i, _i, _d, _M, _i, _i, _M, _i, _i, _p]),
    "blasfeo_hip_dgemm_nn_batched": (_i, [_i, _i, _i, _i, _d, _M, _i, _i, _M, _i, _i, _d, _M, _i, _i, _M, _i, _i, _p]),
    "blasfeo_hip_dsyrk_ln_batched": (_i, [_i, _i, _i, _d, _M, _i, _i, _M, _i, _i, _d, _M, _i, _i, _M, _i, _i, _p]),
    "blasfeo_hip_dtrsm_rltn_batched": (_i, [_i, _i, _i, _d, _M, _i, _i, _M, _i, _i, _M, _i, _i, _p]),
    "blasfeo_hip_dtrmm_rlnn_batched": (_i, [_i, _i, _i, _d, _M, _i, _i, _M, _i, _i, _M, _i, _i, _p]),
    "blasfeo_hip_dpotrf_l_batched": (_i, [_i, _i, _M, _i, _i, _M, _i, _i, _p, _p]),
    "blasfeo_hip_dpotrf_l_mn_batched": (_i, [_i, _i, _i, _M, _i, _i, _M, _i, _i, _p, _p]),
    "blasfeo_hip_dgetrf_batched": (_i, [_i, _i, _i, _M, _i, _i, _M, _i, _i, _i, _p, _p, _p]),
    "blasfeo_hip_dgelqf_batched": (_i, [_i, _i, _i, _M, _i, _i, _M, _i, _i, _p]),
    "blasfeo_hip_dsyrk_dpotrf_trsm_batched": (_i, [_i, _i, _i, _i, _M, _M, _M, _M, _M, _p, _p]),
    "blasfeo_hip_dric_trf_batched": (_i, [_i, _i, _i, _i, _M, _M, _M, _M, _M, _M, _p, _p]),
    "blasfeo_hip_dric_trs_batched": (_i, [_i, _i, _i, _i, _M, _M, _M, _M, _p, _p, _p, _p, _p, _p, _p]),
    "blasfeo_hip_pack_dmat_indexed": (_i, [_i, _i, _i, _p, _i, _ll, _p, _p, _i, _p]),
    "blasfeo_hip_dposv_vbatched_plan": (_i, [_i, _p, _i, ctypes.POINTER(_p), ctypes.POINTER(_ll)]),
    "blasfeo_hip_plan_workspace": (_i, [_p, ctypes.POINTER(_ll), ctypes.POINTER(_ll)]),
    "blasfeo_hip_plan_layout": (_i, [_p, _p, _p, ctypes.POINTER(_ll), ctypes.POINTER(_ll)]),
    "blasfeo_hip_dposv_vbatched": (_i, [_p, _p, _p, _p, _p, _p, _p, _p]),
    "blasfeo_hip_plan_capture": (_i, [_p, _p, _p, _p, _p, _p, _p]),
    "blasfeo_hip_noalloc_init": (_i, []),
    "blasfeo_hip_probe_dmfma": (ctypes.c_longlong, [_i, _i, _p, _p]),
    "blasfeo_hip_probe_copy": (_i, [_p, _p, ctypes.c_longlong, _p]),
    "blasfeo_hip_dposv_vbatched_noalloc": (_i, [_p, _p, _p, _p, _p, _p, _p]),
    "blasfeo_hip_plan_autotune": (_i, [_p, _p, _p, _p, _p, _p, _p, _p]),
    "blasfeo_hip_plan_set_graph": (_i, [_p, _i]),
    "blasfeo_hip_tune_cache_load": (_i, [ctypes.c_char_p]),
    "blasfeo_hip_tune_cache_save": (_i, [ctypes.c_char_p]),
    "blasfeo_hip_tune_cache_clear": (_i, []),
    "blasfeo_hip_tune_cache_stats": (_i, [ctypes.POINTER(_ll), ctypes.POINTER(_ll), ctypes.POINTER(_ll)]),
    "blasfeo_hip_plan_config": (_i, [_p, _p]),
    "blasfeo_hip_plan_set_config": (_i, [_p, _p, _i]),
    "blasfeo_hip_plan_destroy": (None, [_p]),
    "blasfeo_memsize_smat": (_i, [_i, _i]),
    "blasfeo_create_smat": (None, [_i, _i, _S, _p]),
    "blasfeo_allocate_smat": (None, [_i, _i, _S]),
    "blasfeo_free_smat": (None, [_S]),
    "blasfeo_pack_smat": (None, [_i, _i, _p, _i, _S, _i, _i]),
    "blasfeo_unpack_smat": (None, [_i, _i, _S, _i, _i, _p, _i]),
    "blasfeo_hip_pack_smat_batched": (_i, [_i, _i, _i, _p, _i, _ll, _S, _i, _i, _p]),
    "blasfeo_hip_unpack_smat_batched": (_i, [_i, _i, _i, _S, _i, _i, _p, _i, _ll, _p]),
    "blasfeo_sgemm_nt": (None, [_i, _i, _i, _f, _S, _i, _i, _S, _i, _i, _f, _S, _i, _i, _S, _i, _i]),
    "blasfeo_ssyrk_ln": (None, [_i, _i, _f, _S, _i, _i, _S, _i, _i, _f, _S, _i, _i, _S, _i, _i]),
    "blasfeo_spotrf_l": (None, [_i, _S, _i, _i, _S, _i, _i]),
    "blasfeo_hip_sgemm_nt_batched": (_i, [_i, _i, _i, _i, _f, _S, _i, _i, _S, _i, _i, _f, _S, _i, _i, _S, _i, _i, _p]),
    "blasfeo_hip_ssyrk_ln_batched": (_i, [_i, _i, _i, _f, _S, _i, _i, _S, _i, _i, _f, _S, _i, _i, _S, _i, _i, _p]),
    "blasfeo_hip_spotrf_l_batched": (_i, [_i, _i, _S, _i, _i, _S, _i, _i, _p, _p]),
    "blasfeo_hip_dposv_mixed_vbatched": (_i, [_p, _i, _d, _i, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p]),
    "blasfeo_hip_plan_mixed_factor": (_i, [_p, _i, _p, _p, _i, _p]),
}

FP32, FP16_SCALED = 1, 2


def lib():
    """Load libblasfeo_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1704_02457_amd.build` "
                               "or __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


class HipError(RuntimeError):
    pass


def check(code):
    """Raise HipError for a nonzero return code of a batched entry point."""
    if code != 0:
        raise HipError(f"blasfeo_hip error {code}: {lib().blasfeo_hip_strerror(code).decode()}")
    return code


def tune_cache_load(path):
    """Merge a tuning-cache file into the library's table; returns the
    number of entries read (0 if the file does not exist)."""
    r = lib().blasfeo_hip_tune_cache_load(os.fsencode(path))
    if r < 0:
        raise HipError(f"tuning cache {path}: malformed (code {r})")
    return r


def tune_cache_save(path):
    """Write the library's tuning table to `path`; returns the entry count."""
    r = lib().blasfeo_hip_tune_cache_save(os.fsencode(path))
    if r < 0:
        raise HipError(f"tuning cache {path}: cannot write (code {r})")
    return r


def tune_cache_clear():
    lib().blasfeo_hip_tune_cache_clear()


def tune_cache_stats():
    """(entries, hits, misses) of the library's tuning table."""
    e, h, m = _ll(0), _ll(0), _ll(0)
    lib().blasfeo_hip_tune_cache_stats(ctypes.byref(e), ctypes.byref(h), ctypes.byref(m))
    return e.value, h.value, m.value


def check_last():
    """Raise HipError if a single-instance routine recorded an error."""
    check(lib().blasfeo_hip_get_last_error())


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("paper_1704_02457_amd needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream=None):
    if stream is None:
        return _torch().cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def memsize_dmat(m, n):
    return lib().blasfeo_memsize_dmat(m, n)


class DMat:
    """A device panel-major matrix: torch storage + struct blasfeo_dmat."""

    def __init__(self, m, n, device="cuda", storage=None, offset_bytes=0):
        torch = _torch()
        self.s = blasfeo_dmat()
        ms = lib().blasfeo_memsize_dmat(m, n)
        if ms < 0:
            raise ValueError("bad size")
        if storage is None:
            storage = torch.empty(max(ms, 256) // 8, dtype=torch.float64, device=device)
        self.buf = storage
        self.off = offset_bytes // 8
        lib().blasfeo_create_dmat(m, n, ctypes.byref(self.s), ctypes.c_void_p(storage.data_ptr() + offset_bytes))
        self.m, self.n = m, n

    @property
    def ref(self):
        return ctypes.byref(self.s)

    @property
    def memsize(self):
        return self.s.memsize

    def panels(self):
        """The panel storage as a flat float64 tensor view (pm*16*cn)."""
        return self.buf[self.off: self.off + self.s.pm * PS * self.s.cn]

    def dA(self):
        off = self.off + self.s.pm * PS * self.s.cn
        return self.buf[off: off + max(self.m, self.n)]


class DMatBatch:
    """`batch` consecutive DMat chunks of memsize bytes; .s describes instance 0."""

    def __init__(self, batch, m, n, device="cuda", fill=None):
        torch = _torch()
        self.batch, self.m, self.n = batch, m, n
        ms = lib().blasfeo_memsize_dmat(m, n)
        self.stride = ms // 8
        if fill is None:
            self.buf = torch.empty(max(batch * self.stride, 32), dtype=torch.float64, device=device)
        else:
            self.buf = torch.full((max(batch * self.stride, 32),), fill, dtype=torch.float64, device=device)
        self.s = blasfeo_dmat()
        lib().blasfeo_create_dmat(m, n, ctypes.byref(self.s), ctypes.c_void_p(self.buf.data_ptr()))

    @property
    def ref(self):
        return ctypes.byref(self.s)

    def instances(self):
        """(batch, memsize/8) view of the raw chunks."""
        return self.buf[: self.batch * self.stride].view(self.batch, self.stride)

    def dA(self):
        off = self.s.pm * PS * self.s.cn
        return self.instances()[:, off: off + max(self.m, self.n)]


# ------------------------------------------------------------------ packing

def pack(A, out=None, bi=0, bj=0):
    """Column-major copy of the (m, n) tensor A (any layout, on the GPU) into a
    DMat (panel-major) through blasfeo_pack_dmat."""
    torch = _torch()
    m, n = A.shape
    At = A.t().contiguous().to(torch.float64)  # (n, m) row-major == column-major A
    if out is None:
        out = DMat(m, n, device=A.device)
    lib().blasfeo_pack_dmat(m, n, ctypes.c_void_p(At.data_ptr()), max(m, 1), out.ref, bi, bj)
    check_last()
    return out


def unpack(sA, m=None, n=None, ai=0, aj=0):
    """(m, n) tensor of the sub-matrix of DMat sA at (ai, aj)."""
    torch = _torch()
    m = sA.m - ai if m is None else m
    n = sA.n - aj if n is None else n
    out = torch.empty((n, m), dtype=torch.float64, device=sA.buf.device)
    lib().blasfeo_unpack_dmat(m, n, sA.ref, ai, aj, ctypes.c_void_p(out.data_ptr()), max(m, 1))
    check_last()
    return out.t()


def pack_batch(A, out=None):
    """(batch, m, n) tensor -> DMatBatch (panel-major) via the batched pack."""
    torch = _torch()
    batch, m, n = A.shape
    At = A.transpose(1, 2).contiguous().to(torch.float64)  # per instance column-major
    if out is None:
        out = DMatBatch(batch, m, n, device=A.device)
    check(lib().blasfeo_hip_pack_dmat_batched(batch, m, n, ctypes.c_void_p(At.data_ptr()), max(m, 1),
                                              m * n, out.ref, 0, 0, _stream()))
    return out


def unpack_batch(sA, m=None, n=None):
    torch = _torch()
    m = sA.m if m is None else m
    n = sA.n if n is None else n
    out = torch.empty((sA.batch, n, m), dtype=torch.float64, device=sA.buf.device)
    check(lib().blasfeo_hip_unpack_dmat_batched(sA.batch, m, n, sA.ref, 0, 0, ctypes.c_void_p(out.data_ptr()),
                                                max(m, 1), m * n, _stream()))
    return out.transpose(1, 2)


# ------------------------------------------------------------------ single precision

PS_S = 32


class SMat:
    """A device single-precision panel-major matrix (32-float panels) with its
    struct blasfeo_smat."""

    def __init__(self, m, n, device="cuda"):
        torch = _torch()
        self.s = blasfeo_smat()
        ms = lib().blasfeo_memsize_smat(m, n)
        if ms < 0:
            raise ValueError("bad size")
        self.buf = torch.empty(max(ms, 256) // 4, dtype=torch.float32, device=device)
        lib().blasfeo_create_smat(m, n, ctypes.byref(self.s), ctypes.c_void_p(self.buf.data_ptr()))
        self.m, self.n = m, n

    @property
    def ref(self):
        return ctypes.byref(self.s)

    def dA(self):
        off = self.s.pm * PS_S * self.s.cn
        return self.buf[off: off + max(self.m, self.n)]


class SMatBatch:
    """`batch` consecutive SMat chunks of memsize bytes; .s describes instance 0."""

    def __init__(self, batch, m, n, device="cuda"):
        torch = _torch()
        self.batch, self.m, self.n = batch, m, n
        self.stride = lib().blasfeo_memsize_smat(m, n) // 4
        self.buf = torch.empty(max(batch * self.stride, 64), dtype=torch.float32, device=device)
        self.s = blasfeo_smat()
        lib().blasfeo_create_smat(m, n, ctypes.byref(self.s), ctypes.c_void_p(self.buf.data_ptr()))

    @property
    def ref(self):
        return ctypes.byref(self.s)

    def instances(self):
        return self.buf[: self.batch * self.stride].view(self.batch, self.stride)

    def dA(self):
        off = self.s.pm * PS_S * self.s.cn
        return self.instances()[:, off: off + max(self.m, self.n)]


def spack(A, out=None, bi=0, bj=0):
    """(m, n) tensor -> SMat through blasfeo_pack_smat."""
    torch = _torch()
    m, n = A.shape
    At = A.t().contiguous().to(torch.float32)
    if out is None:
        out = SMat(m, n, device=A.device)
    _sync_stream()
    lib().blasfeo_pack_smat(m, n, ctypes.c_void_p(At.data_ptr()), max(m, 1), out.ref, bi, bj)
    check_last()
    return out


def sunpack(sA, m=None, n=None, ai=0, aj=0):
    """(m, n) float32 tensor of the sub-matrix of SMat sA at (ai, aj)."""
    torch = _torch()
    m = sA.m - ai if m is None else m
    n = sA.n - aj if n is None else n
    out = torch.empty((n, m), dtype=torch.float32, device=sA.buf.device)
    _sync_stream()
    lib().blasfeo_unpack_smat(m, n, sA.ref, ai, aj, ctypes.c_void_p(out.data_ptr()), max(m, 1))
    check_last()
    return out.t()


def spack_batch(A, out=None):
    """(batch, m, n) tensor -> SMatBatch via the batched pack."""
    torch = _torch()
    batch, m, n = A.shape
    At = A.transpose(1, 2).contiguous().to(torch.float32)
    if out is None:
        out = SMatBatch(batch, m, n, device=A.device)
    check(lib().blasfeo_hip_pack_smat_batched(batch, m, n, ctypes.c_void_p(At.data_ptr()), max(m, 1),
                                              m * n, out.ref, 0, 0, _stream()))
    return out


def sunpack_batch(sA, m=None, n=None):
    torch = _torch()
    m = sA.m if m is None else m
    n = sA.n if n is None else n
    out = torch.empty((sA.batch, n, m), dtype=torch.float32, device=sA.buf.device)
    check(lib().blasfeo_hip_unpack_smat_batched(sA.batch, m, n, sA.ref, 0, 0, ctypes.c_void_p(out.data_ptr()),
                                                max(m, 1), m * n, _stream()))
    return out.transpose(1, 2)


def blasfeo_sgemm_nt(m, n, k, alpha, sA, ai, aj, sB, bi, bj, beta, sC, ci, cj, sD, di, dj):
    _sync_stream()
    lib().blasfeo_sgemm_nt(m, n, k, alpha, sA.ref, ai, aj, sB.ref, bi, bj, beta, sC.ref, ci, cj, sD.ref, di, dj)
    check_last()


def blasfeo_ssyrk_ln(m, k, alpha, sA, ai, aj, sB, bi, bj, beta, sC, ci, cj, sD, di, dj):
    _sync_stream()
    lib().blasfeo_ssyrk_ln(m, k, alpha, sA.ref, ai, aj, sB.ref, bi, bj, beta, sC.ref, ci, cj, sD.ref, di, dj)
    check_last()


def blasfeo_spotrf_l(m, sC, ci, cj, sD, di, dj):
    _sync_stream()
    lib().blasfeo_spotrf_l(m, sC.ref, ci, cj, sD.ref, di, dj)
    check_last()


def blasfeo_hip_sgemm_nt_batched(batch, m, n, k, alpha, sA, ai, aj, sB, bi, bj, beta, sC, ci, cj, sD, di, dj,
                                 stream=None):
    return check(lib().blasfeo_hip_sgemm_nt_batched(batch, m, n, k, alpha, sA.ref, ai, aj, sB.ref, bi, bj, beta,
                                                    sC.ref, ci, cj, sD.ref, di, dj, _stream(stream)))


def blasfeo_hip_ssyrk_ln_batched(batch, m, k, alpha, sA, ai, aj, sB, bi, bj, beta, sC, ci, cj, sD, di, dj,
                                 stream=None):
    return check(lib().blasfeo_hip_ssyrk_ln_batched(batch, m, k, alpha, sA.ref, ai, aj, sB.ref, bi, bj, beta,
                                                    sC.ref, ci, cj, sD.ref, di, dj, _stream(stream)))


def blasfeo_hip_spotrf_l_batched(batch, m, sC, ci, cj, sD, di, dj, info, stream=None):
    return check(lib().blasfeo_hip_spotrf_l_batched(batch, m, sC.ref, ci, cj, sD.ref, di, dj, _ptr(info),
                                                    _stream(stream)))


# ------------------------------------------------------------------ routines (C ABI names)

def _sync_stream():
    lib().blasfeo_hip_set_stream(ctypes.c_void_p(_stream()))


def blasfeo_dgemm_nt(m, n, k, alpha, sA, ai, aj, sB, bi, bj, beta, sC, ci, cj, sD, di, dj):
    _sync_stream()
    lib().blasfeo_dgemm_nt(m, n, k, alpha, sA.ref, ai, aj, sB.ref, bi, bj, beta, sC.ref, ci, cj, sD.ref, di, dj)
    check_last()


def blasfeo_dgemm_nn(m, n, k, alpha, sA, ai, aj, sB, bi, bj, beta, sC, ci, cj, sD, di, dj):
    _sync_stream()
    lib().blasfeo_dgemm_nn(m, n, k, alpha, sA.ref, ai, aj, sB.ref, bi, bj, beta, sC.ref, ci, cj, sD.ref, di, dj)
    check_last()


def blasfeo_dsyrk_ln(m, k, alpha, sA, ai, aj, sB, bi, bj, beta, sC, ci, cj, sD, di, dj):
    _sync_stream()
    lib().blasfeo_dsyrk_ln(m, k, alpha, sA.ref, ai, aj, sB.ref, bi, bj, beta, sC.ref, ci, cj, sD.ref, di, dj)
    check_last()


def blasfeo_dtrsm_rltn(m, n, alpha, sA, ai, aj, sB, bi, bj, sD, di, dj):
    _sync_stream()
    lib().blasfeo_dtrsm_rltn(m, n, alpha, sA.ref, ai, aj, sB.ref, bi, bj, sD.ref, di, dj)
    check_last()


def blasfeo_dtrmm_rlnn(m, n, alpha, sA, ai, aj, sB, bi, bj, sD, di, dj):
    _sync_stream()
    lib().blasfeo_dtrmm_rlnn(m, n, alpha, sA.ref, ai, aj, sB.ref, bi, bj, sD.ref, di, dj)
    check_last()


def blasfeo_dpotrf_l(m, sC, ci, cj, sD, di, dj):
    _sync_stream()
    lib().blasfeo_dpotrf_l(m, sC.ref, ci, cj, sD.ref, di, dj)
    check_last()


def blasfeo_dpotrf_l_mn(m, n, sC, ci, cj, sD, di, dj):
    _sync_stream()
    lib().blasfeo_dpotrf_l_mn(m, n, sC.ref, ci, cj, sD.ref, di, dj)
    check_last()


def blasfeo_dgetrf_pivot(m, n, sC, ci, cj, sD, di, dj, ipiv):
    _sync_stream()
    lib().blasfeo_dgetrf_pivot(m, n, sC.ref, ci, cj, sD.ref, di, dj, _ptr(ipiv))
    check_last()


def blasfeo_dgetrf_nopivot(m, n, sC, ci, cj, sD, di, dj):
    _sync_stream()
    lib().blasfeo_dgetrf_nopivot(m, n, sC.ref, ci, cj, sD.ref, di, dj)
    check_last()


def blasfeo_dgelqf(m, n, sC, ci, cj, sD, di, dj):
    _sync_stream()
    lib().blasfeo_dgelqf(m, n, sC.ref, ci, cj, sD.ref, di, dj)
    check_last()


def blasfeo_dsyrk_dpotrf_ln(m, k, sA, ai, aj, sB, bi, bj, sC, ci, cj, sD, di, dj):
    _sync_stream()
    lib().blasfeo_dsyrk_dpotrf_ln(m, k, sA.ref, ai, aj, sB.ref, bi, bj, sC.ref, ci, cj, sD.ref, di, dj)
    check_last()


def blasfeo_hip_dpotrf_l_info(m, sC, ci, cj, sD, di, dj, info):
    _sync_stream()
    lib().blasfeo_hip_dpotrf_l_info(m, sC.ref, ci, cj, sD.ref, di, dj, _ptr(info))
    check_last()


def blasfeo_hip_dsyrk_dpotrf_ln_info(m, k, sA, ai, aj, sB, bi, bj, sC, ci, cj, sD, di, dj, info):
    _sync_stream()
    lib().blasfeo_hip_dsyrk_dpotrf_ln_info(m, k, sA.ref, ai, aj, sB.ref, bi, bj, sC.ref, ci, cj, sD.ref, di, dj,
                                           _ptr(info))
    check_last()


def blasfeo_hip_dgemm_nt_batched(batch, m, n, k, alpha, sA, ai, aj, sB, bi, bj, beta, sC, ci, cj, sD, di, dj,
                                 stream=None):
    return check(lib().blasfeo_hip_dgemm_nt_batched(batch, m, n, k, alpha, sA.ref, ai, aj, sB.ref, bi, bj, beta,
                                                    sC.ref, ci, cj, sD.ref, di, dj, _stream(stream)))


def blasfeo_hip_dgemm_nn_batched(batch, m, n, k, alpha, sA, ai, aj, sB, bi, bj, beta, sC, ci, cj, sD, di, dj,
                                 stream=None):
    return check(lib().blasfeo_hip_dgemm_nn_batched(batch, m, n, k, alpha, sA.ref, ai, aj, sB.ref, bi, bj, beta,
                                                    sC.ref, ci, cj, sD.ref, di, dj, _stream(stream)))


def blasfeo_hip_dsyrk_ln_batched(batch, m, k, alpha, sA, ai, aj, sB, bi, bj, beta, sC, ci, cj, sD, di, dj,
                                 stream=None):
    return check(lib().blasfeo_hip_dsyrk_ln_batched(batch, m, k, alpha, sA.ref, ai, aj, sB.ref, bi, bj, beta,
                                                    sC.ref, ci, cj, sD.ref, di, dj, _stream(stream)))


def blasfeo_hip_dtrsm_rltn_batched(batch, m, n, alpha, sA, ai, aj, sB, bi, bj, sD, di, dj, stream=None):
    return check(lib().blasfeo_hip_dtrsm_rltn_batched(batch, m, n, alpha, sA.ref, ai, aj, sB.ref, bi, bj,
                                                      sD.ref, di, dj, _stream(stream)))


def blasfeo_hip_dtrmm_rlnn_batched(batch, m, n, alpha, sA, ai, aj, sB, bi, bj, sD, di, dj, stream=None):
    return check(lib().blasfeo_hip_dtrmm_rlnn_batched(batch, m, n, alpha, sA.ref, ai, aj, sB.ref, bi, bj,
                                                      sD.ref, di, dj, _stream(stream)))


def blasfeo_hip_dpotrf_l_batched(batch, m, sC, ci, cj, sD, di, dj, info, stream=None):
    return check(lib().blasfeo_hip_dpotrf_l_batched(batch, m, sC.ref, ci, cj, sD.ref, di, dj, _ptr(info),
                                                    _stream(stream)))


def blasfeo_hip_dpotrf_l_mn_batched(batch, m, n, sC, ci, cj, sD, di, dj, info, stream=None):
    return check(lib().blasfeo_hip_dpotrf_l_mn_batched(batch, m, n, sC.ref, ci, cj, sD.ref, di, dj, _ptr(info),
                                                       _stream(stream)))


def blasfeo_hip_dgetrf_batched(batch, m, n, sC, ci, cj, sD, di, dj, pivot, ipiv, info, stream=None):
    return check(lib().blasfeo_hip_dgetrf_batched(batch, m, n, sC.ref, ci, cj, sD.ref, di, dj, int(pivot), _ptr(ipiv),
                                                  _ptr(info), _stream(stream)))


def blasfeo_hip_dgelqf_batched(batch, m, n, sC, ci, cj, sD, di, dj, stream=None):
    return check(lib().blasfeo_hip_dgelqf_batched(batch, m, n, sC.ref, ci, cj, sD.ref, di, dj, _stream(stream)))


def blasfeo_hip_dric_trs_batched(batch, nx, nu, N, sA, sB, sP, sF, b, r, q, x0, u, x, stream=None):
    return check(lib().blasfeo_hip_dric_trs_batched(batch, nx, nu, N, sA.ref, sB.ref, sP.ref, sF.ref, _ptr(b), _ptr(r),
                                                    _ptr(q), _ptr(x0), _ptr(u), _ptr(x), _stream(stream)))


def blasfeo_hip_dric_trf_batched(batch, nx, nu, N, sA, sB, sQ, sR, sP, sF, info, stream=None):
    return check(lib().blasfeo_hip_dric_trf_batched(batch, nx, nu, N, sA.ref, sB.ref, sQ.ref, sR.ref, sP.ref,
                                                    sF.ref, _ptr(info), _stream(stream)))


def blasfeo_hip_dsyrk_dpotrf_trsm_batched(batch, m, k, nrhs, sA, sQ, sE, sL, sX, info, stream=None):
    return check(lib().blasfeo_hip_dsyrk_dpotrf_trsm_batched(
        batch, m, k, nrhs, sA.ref if sA is not None else None, sQ.ref, sE.ref if sE is not None else None,
        sL.ref, sX.ref if sX is not None else None, _ptr(info), _stream(stream)))


# ------------------------------------------------------------------ uneven batches (plans)

class VbPlan:
    """Plan of an uneven batch of SPD solves (blasfeo_hip_dposv_vbatched_plan).

    Arenas are flat float64 device tensors; instance i's matrix chunk starts
    at element moff[i] of a matrix arena, its n_i x nrhs right-hand sides
    (column-major, leading dimension round_up(n_i, 16)) at element voff[i] of
    a vector arena.  The workspaces the C calls take are device tensors of
    ws64_bytes / mixed_bytes bytes; unless one is passed explicitly, the
    calls use one the object allocates (through torch) on first use.
    """

    def __init__(self, ns, nrhs):
        import numpy as np
        self.ns = np.asarray(ns, dtype=np.int32)
        self.nrhs = int(nrhs)
        self.handle = ctypes.c_void_p()
        arr = np.ascontiguousarray(self.ns)
        wb = ctypes.c_longlong()
        check(lib().blasfeo_hip_dposv_vbatched_plan(len(arr), arr.ctypes.data_as(ctypes.c_void_p), self.nrhs,
                                                    ctypes.byref(self.handle), ctypes.byref(wb)))
        self.moff = np.zeros(max(len(arr), 1), dtype=np.int64)
        self.voff = np.zeros(max(len(arr), 1), dtype=np.int64)
        mb, vb = ctypes.c_longlong(), ctypes.c_longlong()
        check(lib().blasfeo_hip_plan_layout(self.handle, self.moff.ctypes.data_as(ctypes.c_void_p),
                                            self.voff.ctypes.data_as(ctypes.c_void_p), ctypes.byref(mb),
                                            ctypes.byref(vb)))
        self.moff, self.voff = self.moff[: len(arr)] // 8, self.voff[: len(arr)] // 8
        self.mat_bytes, self.vec_bytes = mb.value, vb.value
        w64, wmx = ctypes.c_longlong(), ctypes.c_longlong()
        check(lib().blasfeo_hip_plan_workspace(self.handle, ctypes.byref(w64), ctypes.byref(wmx)))
        assert w64.value == wb.value
        self.ws64_bytes, self.mixed_bytes = w64.value, wmx.value
        self._work = None

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.blasfeo_hip_plan_destroy(h)
            self.handle = ctypes.c_void_p()

    def workspace(self, mixed=False, device="cuda"):
        """A new device workspace (uint8 tensor) for an FP64 execution or,
        with mixed=True, for a mixed-precision call."""
        torch = _torch()
        nb = self.mixed_bytes if mixed else self.ws64_bytes
        return torch.empty(max(nb, 256), dtype=torch.uint8, device=device)

    def _default_work(self, mixed):
        need = self.mixed_bytes if mixed else self.ws64_bytes
        if self._work is None or self._work.numel() < need:
            self._work = None
            self._work = self.workspace(mixed=mixed)
        return self._work

    def mat_arena(self, fill=None, device="cuda"):
        torch = _torch()
        n = max(self.mat_bytes // 8, 32)
        if fill is None:
            return torch.empty(n, dtype=torch.float64, device=device)
        return torch.full((n,), fill, dtype=torch.float64, device=device)

    def vec_arena(self, fill=0.0, device="cuda"):
        torch = _torch()
        return torch.full((max(self.vec_bytes // 8, 32),), fill, dtype=torch.float64, device=device)

    def dmat(self, arena, i):
        """DMat view of instance i inside a matrix arena."""
        n = int(self.ns[i])
        return DMat(n, n, storage=arena, offset_bytes=int(self.moff[i]) * 8)

    def rhs(self, arena, i):
        """(n_i, nrhs) view of instance i's block inside a vector arena."""
        n = int(self.ns[i])
        ld = (n + 15) // 16 * 16
        o = int(self.voff[i])
        return arena[o: o + ld * max(self.nrhs, 1)].view(max(self.nrhs, 1), ld)[:, :n].t()

    def pack_class(self, n, idx, A, arena):
        """Pack the (count, n, n) tensor A of the instances `idx` (all of order n)."""
        torch = _torch()
        At = A.transpose(1, 2).contiguous()
        off = torch.as_tensor(self.moff[idx], dtype=torch.int64, device=A.device)
        check(lib().blasfeo_hip_pack_dmat_indexed(len(idx), n, n, At.data_ptr(), n, n * n, off.data_ptr(),
                                                  arena.data_ptr(), 1, _stream()))

    def unpack_class(self, n, idx, arena):
        """(count, n, n) tensor of the matrices of instances `idx` (all of
        order n) inside a matrix arena (the indexed unpack)."""
        torch = _torch()
        out = torch.empty((len(idx), n, n), dtype=torch.float64, device=arena.device)
        off = torch.as_tensor(self.moff[idx], dtype=torch.int64, device=arena.device)
        check(lib().blasfeo_hip_pack_dmat_indexed(len(idx), n, n, out.data_ptr(), n, n * n, off.data_ptr(),
                                                  arena.data_ptr(), 0, _stream()))
        return out.transpose(1, 2)

    def dA_class(self, n, idx, arena):
        """(count, n) inverse diagonals (dA) of instances `idx` of order n."""
        torch = _torch()
        cn = (n + 3) // 4 * 4
        base = torch.as_tensor(self.moff[idx] + (n + 15) // 16 * 16 * cn, dtype=torch.int64, device=arena.device)
        return arena[base[:, None] + torch.arange(n, device=arena.device)[None, :]]

    def rhs_index(self, n, idx):
        """(count, nrhs, n) int64 element indices of the right-hand sides of
        the instances `idx` (all of order n) inside a vector arena."""
        torch = _torch()
        ld = (n + 15) // 16 * 16
        base = torch.as_tensor(self.voff[idx], dtype=torch.int64, device="cuda")
        c = torch.arange(max(self.nrhs, 1), device="cuda", dtype=torch.int64)[:, None] * ld
        r = torch.arange(n, device="cuda", dtype=torch.int64)[None, :]
        return base[:, None, None] + (c + r)[None]

    def scatter_rhs(self, n, idx, Bn, arena):
        """Write the (count, n, nrhs) right-hand sides of instances `idx`."""
        arena[self.rhs_index(n, idx)] = Bn.reshape(len(idx), n, -1).transpose(1, 2).to(arena.dtype)

    def gather_rhs(self, n, idx, arena):
        """(count, n, nrhs) blocks of instances `idx` from a vector arena."""
        return arena[self.rhs_index(n, idx)].transpose(1, 2)

    def solve(self, A, L, B, X, info=None, work=None, stream=None):
        w = self._default_work(False) if work is None else work
        return check(lib().blasfeo_hip_dposv_vbatched(self.handle, _ptr(A), _ptr(L), _ptr(B), _ptr(X),
                                                      _ptr(info), _ptr(w), _stream(stream)))

    def solve_noalloc(self, A, L, B, X, info=None, stream=None):
        """blasfeo_hip_dposv_vbatched_noalloc: the same solve with the
        workspace in the library's fixed device array."""
        return check(lib().blasfeo_hip_dposv_vbatched_noalloc(self.handle, _ptr(A), _ptr(L), _ptr(B), _ptr(X),
                                                              _ptr(info), _stream(stream)))

    def capture(self, A, L, B, X, info=None, work=None):
        """Record and instantiate the graph of an execution with these
        tensors (blasfeo_hip_plan_capture); later solve() calls with the
        same tensors replay it."""
        w = self._default_work(False) if work is None else work
        return check(lib().blasfeo_hip_plan_capture(self.handle, _ptr(A), _ptr(L), _ptr(B), _ptr(X),
                                                    _ptr(info), _ptr(w)))

    def autotune(self, A, L, B, X, info=None, work=None, stream=None):
        w = self._default_work(False) if work is None else work
        return check(lib().blasfeo_hip_plan_autotune(self.handle, _ptr(A), _ptr(L), _ptr(B), _ptr(X),
                                                     _ptr(info), _ptr(w), _stream(stream)))

    def set_graph(self, on):
        return check(lib().blasfeo_hip_plan_set_graph(self.handle, 1 if on else 0))

    def solve_mixed(self, A, B, X, iters, berr, fallback, prec=FP32, tol=1e-12, max_iter=10,
                    L=None, info=None, work=None, stream=None):
        """blasfeo_hip_dposv_mixed_vbatched: iters/fallback int32 and berr
        float64 device tensors of `batch` entries; with L (a matrix arena)
        the instances that fall back are re-solved in FP64."""
        w = self._default_work(True) if work is None else work
        return check(lib().blasfeo_hip_dposv_mixed_vbatched(
            self.handle, int(prec), float(tol), int(max_iter), _ptr(A), _ptr(B), _ptr(X), _ptr(L),
            _ptr(info), _ptr(iters), _ptr(berr), _ptr(fallback), _ptr(w), _stream(stream)))

    def mixed_factor(self, i, work=None, stream=None):
        """(n_i, n_i) float32 device tensor: the FP32 factor of S A_i S left
        in the workspace by the last mixed-precision call."""
        torch = _torch()
        n = int(self.ns[i])
        w = self._work if work is None else work
        out = torch.empty((n, n), dtype=torch.float32, device="cuda")
        check(lib().blasfeo_hip_plan_mixed_factor(self.handle, int(i), _ptr(w), out.data_ptr(), n,
                                                  _stream(stream)))
        return out.t()  # column-major storage

    def set_config(self, cfg):
        import numpy as np
        arr = np.ascontiguousarray(np.asarray(cfg, dtype=np.int32))
        return check(lib().blasfeo_hip_plan_set_config(self.handle, arr.ctypes.data_as(ctypes.c_void_p), len(arr)))

    def config(self):
        import numpy as np
        k = lib().blasfeo_hip_plan_config(self.handle, None)
        out = np.zeros(k, dtype=np.int32)
        lib().blasfeo_hip_plan_config(self.handle, out.ctypes.data_as(ctypes.c_void_p))
        return out
