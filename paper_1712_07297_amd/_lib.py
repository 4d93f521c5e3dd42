"""ctypes binding of libhs.so (include/hs.h).  Argument marshalling only: every
step of the method runs in the HIP kernels of the library.

Dense right-hand sides / solutions are torch float64 CUDA tensors of shape
(nrhs, n) (row-major, i.e. the column-major n x nrhs layout of the C ABI) or
(n,); the CSR matrix may be numpy arrays (host) or torch CUDA tensors.
"""

from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhs.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "hs.h")

HS_OK = 0
HS_ERR_ARG = -1
HS_ERR_PATTERN = -2
HS_ERR_GEOMETRY = -3
HS_ERR_BREAKDOWN = -4
HS_ERR_NOMEM = -5
HS_ERR_HIP = -6
HS_ERR_UNSUPPORTED = -7
HS_ERR_NODEVICE = -8
HS_WARN_NOT_CONVERGED = 1
HS_FP64 = 0
HS_MIXED = 1


class HsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class hs_csr(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("row_ptr", ctypes.c_void_p),
        ("col_idx", ctypes.c_void_p),
        ("val", ctypes.c_void_p),
        ("on_device", ctypes.c_int32),
    ]


class hs_geometry(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32)]


class hs_opts(ctypes.Structure):
    _fields_ = [
        ("eps", ctypes.c_double),
        ("fixed_rank", ctypes.c_int32),
        ("leaf_size", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("symmetric", ctypes.c_int32),
        ("keep_levels", ctypes.c_int32),
        ("coarse_fp64_dofs", ctypes.c_int32),
        ("pivoting", ctypes.c_int32),
    ]


class hs_info(ctypes.Structure):
    _fields_ = [
        ("nlevels", ctypes.c_int32),
        ("ncolors_total", ctypes.c_int32),
        ("n", ctypes.c_int64),
        ("coarse_dofs", ctypes.c_int64 * 64),
        ("level_clusters", ctypes.c_int32 * 64),
        ("level_colors", ctypes.c_int32 * 64),
        ("max_cluster", ctypes.c_int32),
        ("breakdown_level", ctypes.c_int32),
        ("breakdown_cluster", ctypes.c_int32),
        ("factor_flops", ctypes.c_double),
        ("apply_flops_per_rhs", ctypes.c_double),
        ("factor_bytes", ctypes.c_double),
        ("symbolic_seconds", ctypes.c_double),
        ("numeric_seconds", ctypes.c_double),
        ("device_bytes", ctypes.c_double),
        ("peak_device_bytes", ctypes.c_double),
    ]


_lib = None

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_D = ctypes.c_double
_PI32 = ctypes.POINTER(ctypes.c_int32)
_PD = ctypes.POINTER(ctypes.c_double)

class hs_server_opts(ctypes.Structure):
    _fields_ = [
        ("hbm_cap_bytes", ctypes.c_double),
        ("workers", ctypes.c_int32),
        ("max_batch", ctypes.c_int32),
        ("max_new_ops", ctypes.c_int32),
    ]


class hs_result(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("iterations", ctypes.c_int32),
        ("relres", ctypes.c_double),
        ("latency_s", ctypes.c_double),
        ("queue_s", ctypes.c_double),
        ("reused", ctypes.c_int32),
        ("batch_size", ctypes.c_int32),
    ]


class hs_server_stats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "completed", "failed", "batches", "reused", "factored_ops", "evictions")] + [
        (k, ctypes.c_double) for k in ("p50_latency_s", "p99_latency_s", "mean_queue_s", "unknowns_per_s", "requests_per_s", "held_bytes", "peak_held_bytes")
    ]


_SIGS = {
    "hs_factor": (ctypes.c_int, [ctypes.POINTER(hs_csr), ctypes.POINTER(hs_geometry), ctypes.POINTER(hs_opts), _P, ctypes.POINTER(_P)]),
    "hs_factor_batch": (ctypes.c_int, [_I32, ctypes.POINTER(hs_csr), ctypes.POINTER(hs_geometry), ctypes.POINTER(hs_opts), _P, ctypes.POINTER(_P)]),
    "hs_factor_systems": (ctypes.c_int, [_P, _PI32, ctypes.POINTER(_I64)]),
    "hs_solve": (ctypes.c_int, [_P, _I64, _P, _I64, _P, _I64, _P]),
    "hs_solve_noalloc": (ctypes.c_int, [_P, _I64, _P, _I64, _P, _I64, _P]),
    "hs_pcg": (ctypes.c_int, [_P, _I64, _P, _I64, _P, _I64, _D, _I32, _PI32, _PD, _P]),
    "hs_gmres": (ctypes.c_int, [_P, _I64, _P, _I64, _P, _I64, _D, _I32, _I32, _PI32, _PD, _P]),
    "hs_factor_info": (ctypes.c_int, [_P, ctypes.POINTER(hs_info)]),
    "hs_factor_ranks": (ctypes.c_int, [_P, _I32, _PI32]),
    "hs_factor_sizes": (ctypes.c_int, [_P, _I32, _PI32]),
    "hs_factor_level_matrix": (ctypes.c_int, [_P, _I32, _PD, _I64]),
    "hs_factor_record": (ctypes.c_int, [_P, _I32, _I32, _I32, _PD, _I64, ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    "hs_free": (None, [_P]),
    "hs_factor_trim": (ctypes.c_int, [_P, _P]),
    "hs_server_create": (ctypes.c_int, [ctypes.POINTER(hs_server_opts), ctypes.POINTER(_P)]),
    "hs_submit": (ctypes.c_int, [_P, _I64, ctypes.POINTER(hs_csr), ctypes.POINTER(hs_geometry), ctypes.POINTER(hs_opts), _I32, _P, _P, _D, _I32, ctypes.POINTER(_I64)]),
    "hs_poll": (ctypes.c_int, [_P, _I64, _PI32]),
    "hs_wait": (ctypes.c_int, [_P, _I64, ctypes.POINTER(hs_result)]),
    "hs_server_stats_get": (ctypes.c_int, [_P, ctypes.POINTER(hs_server_stats)]),
    "hs_server_destroy": (None, [_P]),
    "hs_symbolic_create": (ctypes.c_int, [ctypes.POINTER(hs_csr), ctypes.POINTER(hs_geometry), _I32, ctypes.POINTER(_P)]),
    "hs_symbolic_levels": (ctypes.c_int, [_P, _PI32]),
    "hs_symbolic_level": (ctypes.c_int, [_P, _I32, _PI32, _PI32, ctypes.POINTER(_I64), ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    "hs_symbolic_leaves": (ctypes.c_int, [_P, _PI32, _PI32]),
    "hs_symbolic_arrays": (ctypes.c_int, [_P, _I32, _PI32, _PI32, _PI32, _PI32, _PI32, _PI32, _PI32, _PI32]),
    "hs_symbolic_free": (None, [_P]),
    "hs_set_allocator": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, _P]),
    "hs_profile_enable": (ctypes.c_int, [_I32]),
    "hs_profile_reset": (ctypes.c_int, []),
    "hs_profile_select": (ctypes.c_int, [ctypes.c_char_p]),
    "hs_profile_read": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(_I64), _PD, _PD, _PD]),
    "hs_last_error": (ctypes.c_char_p, []),
    "hs_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "hs_version": (ctypes.c_char_p, []),
    "hs_config_set": (ctypes.c_int, [ctypes.c_char_p, _D]),
    "hs_config_get": (ctypes.c_int, [ctypes.c_char_p, _PD]),
    "hs_config_reset": (ctypes.c_int, []),
}


def header_functions() -> list:
    """Names of the functions declared in include/hs.h."""
    with open(HEADER) as f:
        txt = f.read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hs_[a-z_0-9]+)\s*\(", txt)))


def lib() -> ctypes.CDLL:
    """Load libhs.so (built by paper_1712_07297_amd.build); raises if absent.
    With a GPU visible, the library's device memory then comes from PyTorch's
    caching allocator (use_torch_allocator) unless HS_ALLOCATOR=hip."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1712_07297_amd.build`")
        want_torch = os.environ.get("HS_ALLOCATOR", "torch") == "torch" and _torch_gpu()
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
        if want_torch:
            use_torch_allocator(True)
    return _lib


def _torch_gpu() -> bool:
    try:
        import torch
    except ImportError:
        return False
    return torch.cuda.is_available()


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)
_torch_callbacks = None  # (alloc, free) kept alive while installed


def _torch_alloc(nbytes, stream, ctx):
    import torch

    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(), int(stream or 0))
    except Exception:  # out of memory: the library reports HS_ERR_NOMEM
        return None


def _torch_free(ptr, stream, ctx):
    try:
        import torch

        torch.cuda.caching_allocator_delete(int(ptr))
    except Exception:  # interpreter shutdown: the process's memory goes with it
        pass


def use_torch_allocator(on: bool = True) -> None:
    """Give the library's device memory (level stores, records, workspaces,
    solve vectors) from PyTorch's caching allocator, on the stream each call
    runs on (hs_set_allocator), so that the library and torch share one cache
    and repeated factorizations reuse blocks instead of mapping memory; off:
    HIP's stream-ordered pool.  No factorization may exist (HsError)."""
    global _torch_callbacks
    L = lib()
    if on:
        cbs = (_ALLOC_FN(_torch_alloc), _FREE_FN(_torch_free))
        _check(L.hs_set_allocator(ctypes.cast(cbs[0], ctypes.c_void_p), ctypes.cast(cbs[1], ctypes.c_void_p), None),
               "hs_set_allocator")
        _torch_callbacks = cbs
    else:
        _check(L.hs_set_allocator(None, None, None), "hs_set_allocator")
        _torch_callbacks = None


def torch_allocator_installed() -> bool:
    return _torch_callbacks is not None


def _check(code: int, what: str) -> int:
    if code < 0:
        msg = lib().hs_last_error().decode()
        raise HsError(code, f"{what}: {lib().hs_strerror(code).decode()}: {msg}")
    return code


def _ptr(x) -> int:
    if x is None:
        return 0
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    return x.data_ptr()  # torch tensor


def _csr_struct(row_ptr, col_idx, val, keep: list) -> hs_csr:
    """Host numpy arrays or torch CUDA tensors."""
    on_dev = not isinstance(row_ptr, np.ndarray)
    if not on_dev:
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
    else:
        import torch

        assert row_ptr.dtype == torch.int64 and col_idx.dtype == torch.int32 and val.dtype == torch.float64
        row_ptr, col_idx, val = row_ptr.contiguous(), col_idx.contiguous(), val.contiguous()
    keep += [row_ptr, col_idx, val]
    n = int(row_ptr.shape[0]) - 1
    nnz = int(col_idx.shape[0])
    return hs_csr(n, nnz, _ptr(row_ptr), _ptr(col_idx), _ptr(val), 1 if on_dev else 0)


def _stream(stream) -> int:
    if stream is not None:
        return int(stream)
    import torch

    return int(torch.cuda.current_stream().cuda_stream)


def _geom(dims: Optional[Sequence[int]]) -> hs_geometry:
    """Grid of the unknowns; None: no grid (the graph of A is partitioned)."""
    if dims is None:
        return hs_geometry(0, 0, 0, 0)
    nx, ny, nz = (list(dims) + [1, 1])[:3]
    dim = 3 if nz > 1 else (2 if ny > 1 else 1)
    return hs_geometry(dim, int(nx), int(ny), int(nz))


def _rhs(B):
    """(nrhs, n) or (n,) CUDA float64 tensor -> (tensor (nrhs, n), nrhs, ld, squeeze)."""
    import torch

    if not isinstance(B, torch.Tensor) or not B.is_cuda or B.dtype != torch.float64:
        raise TypeError("right-hand sides must be CUDA float64 torch tensors")
    sq = B.dim() == 1
    B2 = B.reshape(1, -1) if sq else B
    if B2.stride(1) != 1:
        B2 = B2.contiguous()
    return B2, B2.shape[0], B2.stride(0), sq


class Factor:
    """A device-resident factorization (hs_factor, or hs_factor_batch through
    Factor.batch).  Right-hand sides are (nrhs, n) CUDA float64 tensors, rows
    of a batch stacked in the order of its systems."""

    def __init__(self, row_ptr, col_idx, val, dims, eps: float, leaf: int = 64, symmetric: int = -1,
                 precision: int = HS_FP64, fixed_rank: int = 0, keep_levels: bool = False, stream=None,
                 coarse_fp64_dofs: int = 0, _systems=None, pivoting: int = 0):
        keep: list = []
        opts = hs_opts(float(eps), int(fixed_rank), int(leaf), int(precision), int(symmetric), 1 if keep_levels else 0,
                       int(coarse_fp64_dofs), int(pivoting))
        h = _P()
        if _systems is None:
            A = _csr_struct(row_ptr, col_idx, val, keep)
            geom = _geom(dims)
            _check(lib().hs_factor(ctypes.byref(A), ctypes.byref(geom), ctypes.byref(opts), _stream(stream), ctypes.byref(h)), "hs_factor")
        else:
            ns = len(_systems)
            As = (hs_csr * ns)(*[_csr_struct(r, c, v, keep) for (r, c, v, _) in _systems])
            Gs = (hs_geometry * ns)(*[_geom(d) for (_, _, _, d) in _systems])
            _check(lib().hs_factor_batch(ns, As, Gs, ctypes.byref(opts), _stream(stream), ctypes.byref(h)), "hs_factor_batch")
        self._h = h
        ns = _I32(0)
        _check(lib().hs_factor_systems(h, ctypes.byref(ns), None), "hs_factor_systems")
        self.nsys = int(ns.value)
        off = (_I64 * (self.nsys + 1))()
        _check(lib().hs_factor_systems(h, ctypes.byref(ns), off), "hs_factor_systems")
        self.row_off = np.array(off[:], dtype=np.int64)
        self.n = int(self.row_off[-1])

    @classmethod
    def batch(cls, systems, eps: float, leaf: int = 64, symmetric: int = -1, precision: int = HS_FP64,
              fixed_rank: int = 0, stream=None, coarse_fp64_dofs: int = 0, pivoting: int = 0) -> "Factor":
        """hs_factor_batch over systems = [(row_ptr, col_idx, val, dims), ...]."""
        return cls(None, None, None, None, eps, leaf, symmetric, precision, fixed_rank, False, stream,
                   coarse_fp64_dofs, _systems=list(systems), pivoting=pivoting)

    def _lanes(self, rel, nrhs):
        a = np.array(rel[:])
        return a if self.nsys == 1 else a.reshape(nrhs, self.nsys)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.hs_free(h)
            self._h = None

    def free(self):
        self.__del__()

    def solve(self, B, X=None, stream=None):
        import torch

        B2, nrhs, ldb, sq = _rhs(B)
        if X is None:
            X = torch.empty_like(B2)
        _check(lib().hs_solve(self._h, nrhs, _ptr(B2), ldb, _ptr(X), X.stride(0), _stream(stream)), "hs_solve")
        return X.reshape(-1) if sq else X

    def solve_noalloc(self, B, X, stream=None):
        """hs_solve_noalloc: X = A_fac^{-1} B with no device allocation by the
        library (X is the caller's output tensor, shaped like B)."""
        B2, nrhs, ldb, sq = _rhs(B)
        X2 = X.reshape(B2.shape) if sq else X
        if X2.shape != B2.shape or X2.dtype != B2.dtype or not X2.is_cuda or X2.stride(1) != 1:
            raise TypeError("X must be a CUDA float64 tensor shaped like B with unit column stride")
        _check(lib().hs_solve_noalloc(self._h, nrhs, _ptr(B2), ldb, _ptr(X2), X2.stride(0), _stream(stream)),
               "hs_solve_noalloc")
        return X

    def pcg(self, B, tol: float = 1e-10, maxit: int = 500, X=None, stream=None):
        import torch

        B2, nrhs, ldb, sq = _rhs(B)
        if X is None:
            X = torch.empty_like(B2)
        it = _I32(0)
        rel = (ctypes.c_double * (nrhs * self.nsys))()
        rc = _check(lib().hs_pcg(self._h, nrhs, _ptr(B2), ldb, _ptr(X), X.stride(0), float(tol), int(maxit), ctypes.byref(it), rel, _stream(stream)), "hs_pcg")
        return (X.reshape(-1) if sq else X), int(it.value), self._lanes(rel, nrhs), rc == HS_OK

    def gmres(self, B, tol: float = 1e-10, maxit: int = 500, restart: int = 30, X=None, stream=None):
        import torch

        B2, nrhs, ldb, sq = _rhs(B)
        if X is None:
            X = torch.empty_like(B2)
        it = _I32(0)
        rel = (ctypes.c_double * (nrhs * self.nsys))()
        rc = _check(lib().hs_gmres(self._h, nrhs, _ptr(B2), ldb, _ptr(X), X.stride(0), float(tol), int(maxit), int(restart), ctypes.byref(it), rel, _stream(stream)), "hs_gmres")
        return (X.reshape(-1) if sq else X), int(it.value), self._lanes(rel, nrhs), rc == HS_OK

    def trim(self, stream=None):
        """Release the solve / Krylov work vectors (hs_factor_trim)."""
        _check(lib().hs_factor_trim(self._h, _stream(stream)), "hs_factor_trim")

    def info(self) -> hs_info:
        out = hs_info()
        _check(lib().hs_factor_info(self._h, ctypes.byref(out)), "hs_factor_info")
        return out

    def ranks(self, level: int) -> np.ndarray:
        nc = self.info().level_clusters[level]
        out = np.zeros(nc, dtype=np.int32)
        _check(lib().hs_factor_ranks(self._h, level, out.ctypes.data_as(_PI32)), "hs_factor_ranks")
        return out

    def sizes(self, level: int) -> np.ndarray:
        nc = self.info().level_clusters[level]
        out = np.zeros(nc, dtype=np.int32)
        _check(lib().hs_factor_sizes(self._h, level, out.ctypes.data_as(_PI32)), "hs_factor_sizes")
        return out

    def record(self, level: int, cluster: int, which: str) -> np.ndarray:
        """Stored operator of a cluster: 'TL', 'TR', 'ER' or 'EL'."""
        w = {"TL": 0, "TR": 1, "ER": 2, "EL": 3}[which]
        r, c = _I64(0), _I64(0)
        _check(lib().hs_factor_record(self._h, level, cluster, w, None, 0, ctypes.byref(r), ctypes.byref(c)), "hs_factor_record")
        out = np.zeros((r.value, c.value), order="F")
        if out.size:
            _check(lib().hs_factor_record(self._h, level, cluster, w, out.ctypes.data_as(_PD), out.size, ctypes.byref(r), ctypes.byref(c)), "hs_factor_record")
        return out

    def level_matrix(self, level: int) -> np.ndarray:
        dim = int(self.sizes(level).sum())
        out = np.zeros((dim, dim), order="F")
        _check(lib().hs_factor_level_matrix(self._h, level, out.ctypes.data_as(_PD), dim), "hs_factor_level_matrix")
        return out


class Server:
    """The serving request loop (hs_server_*).  submit() queues one solve and
    returns a ticket; wait() blocks until its X is written.  The tensors of a
    request are kept alive here until it completes."""

    def __init__(self, hbm_cap_gb: float, workers: int = 2, max_batch: int = 32, max_new_ops: int = 8):
        o = hs_server_opts(float(hbm_cap_gb) * 1e9, int(workers), int(max_batch), int(max_new_ops))
        h = _P()
        _check(lib().hs_server_create(ctypes.byref(o), ctypes.byref(h)), "hs_server_create")
        self._h = h
        self._keep = {}

    def submit(self, op_key: int, row_ptr, col_idx, val, dims, B, eps: float, leaf: int = 64, symmetric: int = 1,
               precision: int = HS_FP64, tol: float = 1e-10, maxit: int = 300, X=None, coarse_fp64_dofs: int = 0) -> int:
        import torch

        keep: list = []
        A = _csr_struct(row_ptr, col_idx, val, keep)
        B2, nrhs, ldb, sq = _rhs(B)
        if ldb != A.n:
            B2 = B2.contiguous()
        if X is None:
            X = torch.empty_like(B2)
        opts = hs_opts(float(eps), 0, int(leaf), int(precision), int(symmetric), 0, int(coarse_fp64_dofs), 0)
        geom = _geom(dims)
        t = _I64(0)
        _check(lib().hs_submit(self._h, int(op_key), ctypes.byref(A), ctypes.byref(geom), ctypes.byref(opts), nrhs,
                               _ptr(B2), _ptr(X), float(tol), int(maxit), ctypes.byref(t)), "hs_submit")
        self._keep[int(t.value)] = (keep, B2, X, sq)
        return int(t.value)

    def poll(self, ticket: int) -> bool:
        d = _I32(0)
        _check(lib().hs_poll(self._h, int(ticket), ctypes.byref(d)), "hs_poll")
        return bool(d.value)

    def wait(self, ticket: int):
        """(X, result dict) of a request."""
        r = hs_result()
        rc = lib().hs_wait(self._h, int(ticket), ctypes.byref(r))
        keep, B2, X, sq = self._keep.pop(int(ticket))
        res = {k: getattr(r, k) for k, _ in hs_result._fields_}
        if rc < 0 and r.status == 0:
            _check(rc, "hs_wait")
        return (X.reshape(-1) if sq else X), res

    def stats(self) -> dict:
        s = hs_server_stats()
        _check(lib().hs_server_stats_get(self._h, ctypes.byref(s)), "hs_server_stats_get")
        return {k: getattr(s, k) for k, _ in hs_server_stats._fields_}

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.hs_server_destroy(h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        self.close()


class Symbolic:
    """The integer part of the method (host only)."""

    def __init__(self, row_ptr, col_idx, dims, leaf: int):
        keep: list = []
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
        A = _csr_struct(row_ptr, col_idx, np.zeros(col_idx.size), keep)
        geom = _geom(dims)
        h = _P()
        _check(lib().hs_symbolic_create(ctypes.byref(A), ctypes.byref(geom), int(leaf), ctypes.byref(h)), "hs_symbolic_create")
        self._h = h
        self.n = A.n
        nl = _I32(0)
        _check(lib().hs_symbolic_levels(h, ctypes.byref(nl)), "hs_symbolic_levels")
        self.nlevels = int(nl.value)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.hs_symbolic_free(h)
            self._h = None

    def leaves(self) -> Tuple[np.ndarray, np.ndarray]:
        a = np.zeros(self.n, dtype=np.int32)
        b = np.zeros(self.n, dtype=np.int32)
        _check(lib().hs_symbolic_leaves(self._h, a.ctypes.data_as(_PI32), b.ctypes.data_as(_PI32)), "hs_symbolic_leaves")
        return a, b

    def level(self, level: int) -> dict:
        ncl, nco = _I32(0), _I32(0)
        nadj, nfill, npat = _I64(0), _I64(0), _I64(0)
        _check(lib().hs_symbolic_level(self._h, level, ctypes.byref(ncl), ctypes.byref(nco), ctypes.byref(nadj), ctypes.byref(nfill), ctypes.byref(npat)), "hs_symbolic_level")
        c = int(ncl.value)
        arr = {k: np.zeros(sz, dtype=np.int32) for k, sz in [("colors", c), ("order", c), ("adj_ptr", c + 1), ("adj", nadj.value), ("fill_ptr", c + 1), ("fill", nfill.value), ("pat_ptr", c + 1), ("pat", npat.value)]}
        _check(lib().hs_symbolic_arrays(self._h, level, *[arr[k].ctypes.data_as(_PI32) for k in ["colors", "order", "adj_ptr", "adj", "fill_ptr", "fill", "pat_ptr", "pat"]]), "hs_symbolic_arrays")
        arr["ncolors"] = int(nco.value)
        arr["nclusters"] = c
        return arr


def profile_enable(on: bool = True) -> None:
    _check(lib().hs_profile_enable(1 if on else 0), "hs_profile_enable")


def profile_select(families: str = "") -> None:
    """Time only these families (comma-separated; "" = all)."""
    _check(lib().hs_profile_select(families.encode()), "hs_profile_select")


def profile_reset() -> None:
    _check(lib().hs_profile_reset(), "hs_profile_reset")


def profile_read(family: str) -> dict:
    n = _I64(0)
    sec, by, fl = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0)
    _check(lib().hs_profile_read(family.encode(), ctypes.byref(n), ctypes.byref(sec), ctypes.byref(by), ctypes.byref(fl)), "hs_profile_read")
    return {"launches": int(n.value), "seconds": sec.value, "bytes": by.value, "flops": fl.value}


def strerror(code: int) -> str:
    return lib().hs_strerror(code).decode()


def version() -> str:
    return lib().hs_version().decode()


def config_set(name: str, value: float) -> None:
    """hs_config_set: lower a kernel-variant threshold (process-wide)."""
    _check(lib().hs_config_set(name.encode(), float(value)), f"hs_config_set({name})")


def config_get(name: str) -> float:
    v = ctypes.c_double()
    _check(lib().hs_config_get(name.encode(), ctypes.byref(v)), f"hs_config_get({name})")
    return v.value


def config_reset() -> None:
    _check(lib().hs_config_reset(), "hs_config_reset")
