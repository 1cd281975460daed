"""MI355X-native randomized Kaczmarz with averaging (RKA) and its block
variant (RKAB) -- arXiv 2401.17474 -- Python binding over ``librka.so``.

This module only marshals torch tensors into the C ABI declared in
``include/rka.h``; every step of the solve runs in the HIP kernels of the
library.  PyTorch supplies device memory and the current stream.  There is no
CPU fallback: if the library is not built, or a tensor is not on the GPU, the
call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librka.so")

OK, NOT_CONVERGED, EINVAL, EZERONORM, EDIVERGED, ENOMEM, EDEVICE = 0, 1, -1, -2, -3, -4, -5

_lib = None


class RKAError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{status_string(status)}: {msg}")
        self.status = status


class _Info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("projections", ctypes.c_int64),
                ("rel_err", ctypes.c_double), ("status", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class _Opts(ctypes.Structure):
    _fields_ = [("check_every", ctypes.c_int64), ("grid", ctypes.c_int32),
                ("collect_timing", ctypes.c_int32), ("allreduce", ctypes.c_int32),
                ("accumulate", ctypes.c_int32), ("stream_id", ctypes.c_int32),
                ("sampling", ctypes.c_int32), ("worker_alpha", ctypes.c_void_p),
                ("row_weight", ctypes.c_void_p), ("steps_per_exchange", ctypes.c_int32),
                ("rkab_split", ctypes.c_int32), ("rka_block", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("norms_ms", ctypes.c_double), ("prefix_ms", ctypes.c_double),
                ("sample_ms", ctypes.c_double), ("iterate_ms", ctypes.c_double),
                ("measure_ms", ctypes.c_double), ("iterate_launches", ctypes.c_int64),
                ("kernel", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("threads", ctypes.c_int32), ("bucket", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("accumulate", ctypes.c_int32),
                ("coef_ms", ctypes.c_double)]


class _RefineOpts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("q", ctypes.c_int32),
                ("block_size", ctypes.c_int32), ("accumulate", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("inner_iters", ctypes.c_int64),
                ("range_iters", ctypes.c_int64), ("range_q", ctypes.c_int32),
                ("max_sweeps", ctypes.c_int32), ("range_alpha", ctypes.c_double),
                ("tol", ctypes.c_double)]


class _BatchSystem(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("lda", ctypes.c_int64), ("b", ctypes.c_void_p), ("ldb", ctypes.c_int64),
                ("x", ctypes.c_void_p), ("ldx", ctypes.c_int64), ("x_ref", ctypes.c_void_p),
                ("ldxr", ctypes.c_int64), ("nrhs", ctypes.c_int32), ("q", ctypes.c_int32),
                ("block_size", ctypes.c_int32), ("tpr", ctypes.c_int32),
                ("rhs_per_task", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("max_iter", ctypes.c_int64)]


class _BatchResult(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("rel", ctypes.c_double),
                ("alpha", ctypes.c_double),
                ("status", ctypes.c_int32), ("q", ctypes.c_int32), ("block_size", ctypes.c_int32),
                ("tpr", ctypes.c_int32), ("rhs_per_task", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class _BatchStats(ctypes.Structure):
    _fields_ = [("tasks", ctypes.c_int32), ("chunks", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("setup_ms", ctypes.c_double), ("iterate_ms", ctypes.c_double)]


class _RefineInfo(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int32), ("status", ctypes.c_int32),
                ("rel", ctypes.c_double), ("projections", ctypes.c_int64)]


@dataclass
class Info:
    iterations: int
    projections: int
    rel_err: float
    status: int


def lib():
    """Load librka.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        P, I64, I32, D, U64 = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                               ctypes.c_double, ctypes.c_uint64)
        L.rka_solve.argtypes = [P, ctypes.c_int, I64, I64, I64, P, P, P, I32, D, I64, D, U64, P,
                                I64, I64, P, ctypes.POINTER(_Info)]
        L.rkab_solve.argtypes = [P, ctypes.c_int, I64, I64, I64, P, P, P, I32, I32, D, I64, D,
                                 U64, P, I64, I64, P, ctypes.POINTER(_Info)]
        L.rka_solve_ex.argtypes = [P, ctypes.c_int, I64, I64, I64, P, P, P, I32, I32, I32, D,
                                   I64, D, U64, P, I64, ctypes.POINTER(_Opts), P,
                                   ctypes.POINTER(_Info), ctypes.POINTER(_Stats)]
        L.rka_solve_ex_noalloc.argtypes = L.rka_solve_ex.argtypes
        L.rka_row_norms.argtypes = [P, ctypes.c_int, I64, I64, I64, P, P]
        L.rka_prefix.argtypes = [P, I64, P, P, P]
        L.rka_sample_indices.argtypes = [P, P, I64, U64, I64, I64, I32, I32, I32, P, P]
        L.rka_gemv.argtypes = [P, ctypes.c_int, I64, I64, I64, P, P, D, P, P]
        L.rka_transpose.argtypes = [P, ctypes.c_int, I64, I64, I64, P, I64, P]
        L.rka_lsq_grad_A.argtypes = [I64, I64, P, P, P, P, P, ctypes.c_int, I64, P]
        L.rka_refine_solve.argtypes = [P, P, ctypes.c_int, I64, I64, I64, I64, P, P, P,
                                       ctypes.POINTER(_RefineOpts), U64, P, P, P,
                                       ctypes.POINTER(_RefineInfo)]
        L.rka_batch_solve.argtypes = [ctypes.POINTER(_BatchSystem), I32, ctypes.c_int, U64, D,
                                      I64, I64, I32, P, ctypes.POINTER(_BatchResult),
                                      ctypes.POINTER(_BatchStats)]
        L.rka_batch_refine_solve.argtypes = [ctypes.POINTER(_BatchSystem), I32, ctypes.c_int,
                                             U64, D, I64, I32, I32, P,
                                             ctypes.POINTER(_BatchResult),
                                             ctypes.POINTER(_BatchStats)]
        L.rka_batch_sample_indices.argtypes = [ctypes.POINTER(_BatchSystem), I32, ctypes.c_int,
                                               U64, I64, P, P]
        L.rka_batch_tune.argtypes = [ctypes.POINTER(_BatchSystem), I32, ctypes.c_int, U64, P,
                                     ctypes.POINTER(I32)]
        L.rka_gemv_t.argtypes = [P, ctypes.c_int, I64, I64, I64, P, P, D, P, P]
        L.rka_spectral_bounds.argtypes = [P, ctypes.c_int, I64, I64, I64, I32, U64, P,
                                          ctypes.POINTER(D), ctypes.POINTER(D),
                                          ctypes.POINTER(D)]
        L.rka_partial_alpha.argtypes = [P, ctypes.c_int, I64, I64, I64, I32, I32, U64, P, P]
        L.rka_sample_blocks.argtypes = [P, I64, U64, I64, I64, I32, I32, I32, P, P]
        PP = ctypes.POINTER(ctypes.c_void_p)
        L.rka_plan_create.argtypes = [P, ctypes.c_int, I64, I64, I64, P, PP]
        L.rka_plan_destroy.argtypes = [P]
        L.rka_plan_query.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I64),
                                     ctypes.POINTER(D), ctypes.POINTER(I64)]
        L.rka_plan_row_norms.argtypes = [P, P, P]
        L.rka_plan_sample_indices.argtypes = [P, U64, I64, I64, I32, I32, I32, P, P]
        L.rka_plan_solve.argtypes = [P, P, P, P, I32, I32, I32, D, I64, D, U64, P, I64,
                                     ctypes.POINTER(_Opts), P, ctypes.POINTER(_Info),
                                     ctypes.POINTER(_Stats)]
        L.rka_plan_refine_solve.argtypes = [P, P, P, P, P, ctypes.POINTER(_RefineOpts), U64, P,
                                            P, P, ctypes.POINTER(_RefineInfo)]
        L.rka_alpha_star.argtypes = [D, D, I32, ctypes.POINTER(D)]
        L.rka_status_string.argtypes = [ctypes.c_int]
        L.rka_status_string.restype = ctypes.c_char_p
        L.rka_last_error.argtypes = []
        L.rka_last_error.restype = ctypes.c_char_p
        L.rka_version.restype = ctypes.c_int
        for f in ("rka_solve", "rkab_solve", "rka_solve_ex", "rka_row_norms", "rka_prefix",
                  "rka_sample_indices", "rka_gemv", "rka_transpose", "rka_lsq_grad_A",
                  "rka_refine_solve", "rka_batch_solve", "rka_batch_tune",
                  "rka_batch_refine_solve", "rka_gemv_t", "rka_spectral_bounds",
                  "rka_partial_alpha", "rka_sample_blocks", "rka_plan_create",
                  "rka_plan_destroy", "rka_plan_query", "rka_plan_row_norms",
                  "rka_plan_sample_indices", "rka_plan_solve", "rka_plan_refine_solve",
                  "rka_alpha_star", "rka_solve_ex_noalloc", "rka_batch_sample_indices"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(status: int) -> str:
    names = {OK: "RKA_OK", NOT_CONVERGED: "RKA_NOT_CONVERGED", EINVAL: "RKA_EINVAL",
             EZERONORM: "RKA_EZERONORM", EDIVERGED: "RKA_EDIVERGED", ENOMEM: "RKA_ENOMEM",
             EDEVICE: "RKA_EDEVICE"}
    return names.get(status, f"status {status}")


def _raise_if(status):
    if status < 0:
        raise RKAError(status, lib().rka_last_error().decode())


# -- tensor marshalling --------------------------------------------------------

def _torch():
    import torch
    return torch


def _dtype_code(t):
    torch = _torch()
    codes = {torch.float64: 0, torch.float32: 1, torch.bfloat16: 2}
    if t.dtype not in codes:
        raise TypeError(f"A must be float64, float32 or bfloat16, got {t.dtype}")
    return codes[t.dtype]


def _matrix(A):
    if A.dim() != 2:
        raise ValueError("A must be a 2-D tensor")
    if not A.is_cuda:
        raise ValueError("A must be a GPU tensor")
    if A.stride(1) != 1 or (A.shape[0] > 1 and A.stride(0) < A.shape[1]):
        raise ValueError("A must be row-major with unit column stride")
    lda = A.stride(0) if A.shape[0] > 1 else A.shape[1]
    return _dtype_code(A), A.shape[0], A.shape[1], lda


def _vec(v, n, name, allow_none=True):
    torch = _torch()
    if v is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    if not v.is_cuda or v.dtype != torch.float64 or v.dim() != 1 or v.shape[0] != n \
            or not v.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 GPU vector of length {n}")
    return v


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# -- solvers -------------------------------------------------------------------

def rka_solve(A, b, *, q, alpha=1.0, max_iter=1000, tol=0.0, seed=1, x0=None, x_ref=None,
              iter_offset=0, check_every=1, out=None, stream=None, raise_on_error=True):
    """RKA with uniform weight alpha (Eq. (7), Sec. 3.3.1).  Returns (x, Info)."""
    torch = _torch()
    code, m, n, lda = _matrix(A)
    b = _vec(b, m, "b", False)
    x = out if out is not None else torch.empty(n, dtype=torch.float64, device=A.device)
    _vec(x, n, "out", False)
    info = _Info()
    st = lib().rka_solve(_ptr(A), code, m, n, lda, _ptr(b), _ptr(_vec(x0, n, "x0")), _ptr(x), q,
                         alpha, max_iter, tol, seed, _ptr(_vec(x_ref, n, "x_ref")), iter_offset,
                         check_every, _stream(stream), ctypes.byref(info))
    if raise_on_error:
        _raise_if(st)
    return x, Info(info.iterations, info.projections, info.rel_err, st)


def rkab_solve(A, b, *, q, block_size, alpha=1.0, max_iter=1000, tol=0.0, seed=1, x0=None,
               x_ref=None, iter_offset=0, check_every=1, out=None, stream=None,
               raise_on_error=True):
    """RKAB (Sec. 3.4.1, Algorithm 3).  Returns (x, Info)."""
    torch = _torch()
    code, m, n, lda = _matrix(A)
    b = _vec(b, m, "b", False)
    x = out if out is not None else torch.empty(n, dtype=torch.float64, device=A.device)
    _vec(x, n, "out", False)
    info = _Info()
    st = lib().rkab_solve(_ptr(A), code, m, n, lda, _ptr(b), _ptr(_vec(x0, n, "x0")), _ptr(x),
                          q, block_size, alpha, max_iter, tol, seed,
                          _ptr(_vec(x_ref, n, "x_ref")), iter_offset, check_every,
                          _stream(stream), ctypes.byref(info))
    if raise_on_error:
        _raise_if(st)
    return x, Info(info.iterations, info.projections, info.rel_err, st)


def solve_ex(A, b, *, method, q, block_size=1, alpha=1.0, max_iter=1000, tol=0.0, seed=1,
             x0=None, x_ref=None, iter_offset=0, check_every=1, grid=0, allreduce=0,
             timing=False, accumulate=0, stream_id=0, sampling=0, worker_alpha=None,
             row_weight=None, steps_per_exchange=0, rkab_split=0, rka_block=0, out=None,
             stream=None, raise_on_error=True, no_alloc=False):
    """rka_solve_ex: method 0 = RKA, 1 = RKAB.  Returns (x, Info, stats dict);
    with ``timing`` the stats hold per-phase HIP-event times (ms) measured on
    the stream the kernels run on.  ``accumulate=1`` computes in FP32 (narrow
    storage only); ``stream_id`` is the row stream's counter domain;
    ``sampling=1`` is the Distributed Approach (worker w samples its own row
    block), ``sampling=2`` the cyclic row order (Cyclic Kaczmarz at q=1);
    ``worker_alpha`` is a float64 GPU vector of per-worker weights and
    ``row_weight`` one of per-row weights w_i (Eq. (7)); ``steps_per_exchange``
    (RKA) runs blocks of up to that many iterations per exchange between
    workgroups (0: the library's choice, 1: one); ``rkab_split`` (RKAB) picks
    the worker-split (1) or column-split (2) kernel (0: the library's choice).
    ``no_alloc`` calls rka_solve_ex_noalloc (scratch from the library's fixed
    device array instead of stream-ordered allocations)."""
    code, m, n, lda = _matrix(A)
    fn = lib().rka_solve_ex_noalloc if no_alloc else lib().rka_solve_ex
    return _solve_ex_call(lambda b_, x0_, x_, opts, info, stats: fn(
        _ptr(A), code, m, n, lda, b_, x0_, x_, method, q, block_size, alpha, max_iter, tol, seed,
        _ptr(_vec(x_ref, n, "x_ref")), iter_offset, ctypes.byref(opts), _stream(stream),
        ctypes.byref(info), ctypes.byref(stats)), A.device, m, n, b, x0, out, q, check_every,
        grid, timing, allreduce, accumulate, stream_id, sampling, worker_alpha, row_weight,
        steps_per_exchange, rkab_split, rka_block, raise_on_error)


def _solve_ex_call(call, device, m, n, b, x0, out, q, check_every, grid, timing, allreduce,
                   accumulate, stream_id, sampling, worker_alpha, row_weight,
                   steps_per_exchange, rkab_split, rka_block, raise_on_error):
    torch = _torch()
    b = _vec(b, m, "b", False)
    x = out if out is not None else torch.empty(n, dtype=torch.float64, device=device)
    _vec(x, n, "out", False)
    info, stats = _Info(), _Stats()
    if worker_alpha is not None:
        _vec(worker_alpha, q, "worker_alpha", False)
    if row_weight is not None:
        _vec(row_weight, m, "row_weight", False)
    opts = _Opts(check_every, grid, 1 if timing else 0, allreduce, accumulate, stream_id,
                 sampling, None if worker_alpha is None else worker_alpha.data_ptr(),
                 None if row_weight is None else row_weight.data_ptr(), steps_per_exchange,
                 rkab_split, rka_block)
    st = call(_ptr(b), _ptr(_vec(x0, n, "x0")), _ptr(x), opts, info, stats)
    if raise_on_error:
        _raise_if(st)
    sd = {f: getattr(stats, f) for f, _ in _Stats._fields_}
    return x, Info(info.iterations, info.projections, info.rel_err, st), sd


class Plan:
    """rka_plan_create: the squared row norms, running sum, ||A||_F^2 and last
    positive row of A (Eq. (4)), computed once on the device and reused by
    every solve, refinement and row stream over A.  Keeps a reference to A
    (the plan points into its storage).  Freed by close() or when collected."""

    def __init__(self, A, stream=None):
        code, m, n, lda = _matrix(A)
        h = ctypes.c_void_p()
        _raise_if(lib().rka_plan_create(_ptr(A), code, m, n, lda, _stream(stream),
                                        ctypes.byref(h)))
        self._h, self.A, self.m, self.n = h, A, m, n
        f = ctypes.c_double()
        _raise_if(lib().rka_plan_query(h, None, None, ctypes.byref(f), None))
        self.fro2 = f.value

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _raise_if(lib().rka_plan_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        if self._h is None or not self._h.value:
            raise ValueError("the plan has been closed")
        return self._h

    def last_pos(self):
        v = ctypes.c_int64()
        _raise_if(lib().rka_plan_query(self.handle, None, None, None, ctypes.byref(v)))
        return v.value

    def row_norms(self, stream=None):
        """The plan's squared row norms as a float64 GPU tensor (a copy)."""
        torch = _torch()
        w = torch.empty(self.m, dtype=torch.float64, device=self.A.device)
        _raise_if(lib().rka_plan_row_norms(self.handle, _ptr(w), _stream(stream)))
        return w

    def sample_indices(self, *, seed, iter_offset=0, K, q, bs=1, dom=0, stream=None):
        """The row stream from the plan's running sum (rka_plan_sample_indices)."""
        torch = _torch()
        idx = torch.empty(K * q * bs, dtype=torch.int32, device=self.A.device)
        _raise_if(lib().rka_plan_sample_indices(self.handle, seed, iter_offset, K, q, bs, dom,
                                                _ptr(idx), _stream(stream)))
        return idx

    def solve(self, b, *, method, q, block_size=1, alpha=1.0, max_iter=1000, tol=0.0, seed=1,
              x0=None, x_ref=None, iter_offset=0, check_every=1, grid=0, allreduce=0,
              timing=False, accumulate=0, stream_id=0, sampling=0, worker_alpha=None,
              row_weight=None, steps_per_exchange=0, rkab_split=0, rka_block=0, out=None,
              stream=None, raise_on_error=True):
        """rka_plan_solve: solve_ex on the plan's matrix without the per-call set-up."""
        h = self.handle
        return _solve_ex_call(lambda b_, x0_, x_, opts, info, stats: lib().rka_plan_solve(
            h, b_, x0_, x_, method, q, block_size, alpha, max_iter, tol, seed,
            _ptr(_vec(x_ref, self.n, "x_ref")), iter_offset, ctypes.byref(opts), _stream(stream),
            ctypes.byref(info), ctypes.byref(stats)), self.A.device, self.m, self.n, b, x0, out,
            q, check_every, grid, timing, allreduce, accumulate, stream_id, sampling,
            worker_alpha, row_weight, steps_per_exchange, rkab_split, rka_block, raise_on_error)


def row_norms(A, stream=None):
    """Squared row norms (Eq. (4) numerators) as a float64 GPU tensor."""
    torch = _torch()
    code, m, n, lda = _matrix(A)
    w = torch.empty(m, dtype=torch.float64, device=A.device)
    _raise_if(lib().rka_row_norms(_ptr(A), code, m, n, lda, _ptr(w), _stream(stream)))
    return w


def prefix(w, stream=None):
    """Running sum of the weights and the last row with positive weight."""
    torch = _torch()
    m = w.shape[0]
    _vec(w, m, "w", False)
    c = torch.empty_like(w)
    last = torch.empty(1, dtype=torch.int64, device=w.device)
    _raise_if(lib().rka_prefix(_ptr(w), m, _ptr(c), _ptr(last), _stream(stream)))
    return c, last


def sample_indices(w, c, *, seed, iter_offset=0, K, q, bs=1, dom=0, stream=None):
    """The row stream: int32 tensor of K*q*bs indices, layout (k, worker, j)."""
    torch = _torch()
    m = w.shape[0]
    _vec(w, m, "w", False)
    _vec(c, m, "c", False)
    idx = torch.empty(K * q * bs, dtype=torch.int32, device=w.device)
    _raise_if(lib().rka_sample_indices(_ptr(w), _ptr(c), m, seed, iter_offset, K, q, bs, dom,
                                       _ptr(idx), _stream(stream)))
    return idx


# -- dense steps and refinement --------------------------------------------------

def gemv(M, v, *, c=None, gamma=1.0, out=None, stream=None):
    """out = (c or 0) + gamma * M v in FP64 (rka_gemv)."""
    torch = _torch()
    code, rows, cols, ld = _matrix(M)
    _vec(v, cols, "v", False)
    _vec(c, rows, "c")
    y = out if out is not None else torch.empty(rows, dtype=torch.float64, device=M.device)
    _vec(y, rows, "out", False)
    _raise_if(lib().rka_gemv(_ptr(M), code, rows, cols, ld, _ptr(v), _ptr(c), gamma, _ptr(y),
                             _stream(stream)))
    return y


def gemv_t(M, t, *, c=None, gamma=1.0, out=None, stream=None):
    """out = (c or 0) + gamma * M^T t in FP64 (rka_gemv_t), without a transposed copy."""
    torch = _torch()
    code, rows, cols, ld = _matrix(M)
    _vec(t, rows, "t", False)
    _vec(c, cols, "c")
    y = out if out is not None else torch.empty(cols, dtype=torch.float64, device=M.device)
    _vec(y, cols, "out", False)
    _raise_if(lib().rka_gemv_t(_ptr(M), code, rows, cols, ld, _ptr(t), _ptr(c), gamma, _ptr(y),
                               _stream(stream)))
    return y


def spectral_bounds(A, *, steps=120, seed=1, stream=None):
    """(lam_min, lam_max, ||A||_F^2): extreme Ritz values of A^T A by Lanczos on
    the device (rka_spectral_bounds); s = lam / ||A||_F^2 feeds alpha_star."""
    code, m, n, lda = _matrix(A)
    lo, hi, f = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _raise_if(lib().rka_spectral_bounds(_ptr(A), code, m, n, lda, steps, seed, _stream(stream),
                                        ctypes.byref(lo), ctypes.byref(hi), ctypes.byref(f)))
    return lo.value, hi.value, f.value


def partial_alpha(A, q, *, steps=120, seed=1, stream=None):
    """Per-worker weights of the partial-matrix variant (rka_partial_alpha):
    a float64 GPU vector of q entries, for solve_ex(worker_alpha=...)."""
    torch = _torch()
    code, m, n, lda = _matrix(A)
    out = (ctypes.c_double * q)()
    _raise_if(lib().rka_partial_alpha(_ptr(A), code, m, n, lda, q, steps, seed, _stream(stream),
                                      out))
    return torch.tensor(list(out), dtype=torch.float64, device=A.device)


def sample_blocks(w, *, seed, iter_offset=0, K, q, bs=1, dom=0, stream=None):
    """The Distributed Approach row stream (rka_sample_blocks): int32 tensor of
    K*q*bs indices, worker w drawing from its own row block."""
    torch = _torch()
    m = w.shape[0]
    _vec(w, m, "w", False)
    idx = torch.empty(K * q * bs, dtype=torch.int32, device=w.device)
    _raise_if(lib().rka_sample_blocks(_ptr(w), m, seed, iter_offset, K, q, bs, dom, _ptr(idx),
                                      _stream(stream)))
    return idx


def transpose(A, stream=None):
    """A contiguous transposed copy of A made by the library's kernel."""
    torch = _torch()
    code, m, n, lda = _matrix(A)
    At = torch.empty((n, m), dtype=A.dtype, device=A.device)
    _raise_if(lib().rka_transpose(_ptr(A), code, m, n, lda, _ptr(At), m, _stream(stream)))
    return At


def lsq_grad_A(r, lam, z, x, *, dtype=None, stream=None):
    """dA = r lam^T - z x^T (rka_lsq_grad_A), float64 or float32."""
    torch = _torch()
    m, n = r.shape[0], x.shape[0]
    for v, k, nm in ((r, m, "r"), (z, m, "z"), (lam, n, "lam"), (x, n, "x")):
        _vec(v, k, nm, False)
    dt = dtype or torch.float64
    if dt not in (torch.float64, torch.float32):
        raise TypeError("dtype must be float64 or float32")
    dA = torch.empty((m, n), dtype=dt, device=r.device)
    _raise_if(lib().rka_lsq_grad_A(m, n, _ptr(r), _ptr(lam), _ptr(z), _ptr(x), _ptr(dA),
                                   0 if dt == torch.float64 else 1, n, _stream(stream)))
    return dA


@dataclass
class RefineInfo:
    sweeps: int
    status: int
    rel: float
    projections: int
    measures: list


def refine_solve(A, b, *, At=None, method=0, q, block_size=1, accumulate=1, alpha=1.0,
                 inner_iters, range_iters=0, range_q=1, range_alpha=1.0, max_sweeps=4,
                 tol=0.0, seed=1, x0=None, x_ref=None, out=None, stream=None,
                 raise_on_error=True, plan=None, plan_t=None):
    """rka_refine_solve: FP64 refinement sweeps around inner RKA/RKAB solves
    (optionally FP32), with the residual projected onto range(A) by a column
    solve on ``At`` when ``range_iters`` > 0.  With ``plan`` (a Plan of A) and
    ``plan_t`` (a Plan of At) the norms and running sums come from the plans
    (rka_plan_refine_solve).  Returns (x, RefineInfo)."""
    torch = _torch()
    if plan is not None:
        A = plan.A
        if range_iters > 0 and plan_t is None:
            raise ValueError("with plan and range_iters > 0, give plan_t (a Plan of At)")
        if plan_t is not None:
            At = plan_t.A
    code, m, n, lda = _matrix(A)
    ldat = 0
    if At is not None:
        ct, nt, mt, ldat = _matrix(At)
        if ct != code or nt != n or mt != m:
            raise ValueError("At must be the n x m transpose of A, same dtype")
    b = _vec(b, m, "b", False)
    x = out if out is not None else torch.empty(n, dtype=torch.float64, device=A.device)
    _vec(x, n, "out", False)
    o = _RefineOpts(method, q, block_size, accumulate, alpha, inner_iters, range_iters, range_q,
                    max_sweeps, range_alpha, tol)
    meas = (ctypes.c_double * max_sweeps)()
    info = _RefineInfo()
    if plan is not None:
        st = lib().rka_plan_refine_solve(plan.handle, None if plan_t is None else plan_t.handle,
                                         _ptr(b), _ptr(_vec(x0, n, "x0")), _ptr(x),
                                         ctypes.byref(o), seed, _ptr(_vec(x_ref, n, "x_ref")),
                                         meas, _stream(stream), ctypes.byref(info))
    else:
        st = lib().rka_refine_solve(_ptr(A), _ptr(At), code, m, n, lda, ldat, _ptr(b),
                                    _ptr(_vec(x0, n, "x0")), _ptr(x), ctypes.byref(o), seed,
                                    _ptr(_vec(x_ref, n, "x_ref")), meas, _stream(stream),
                                    ctypes.byref(info))
    if raise_on_error:
        _raise_if(st)
    return x, RefineInfo(info.sweeps, st, info.rel, info.projections,
                         [meas[i] for i in range(info.sweeps)])


# -- batching ------------------------------------------------------------------

@dataclass
class BatchSystem:
    """One system of a batch: A (m x n, float32 or bfloat16, GPU), B (m) or
    (nrhs x m) float64, X (n) or (nrhs x n) float64 -- start values in,
    results out.  q, block_size, tpr, alpha = 0 let the library (its tuner)
    choose."""
    A: object
    B: object
    X: object
    X_ref: object = None
    q: int = 0
    block_size: int = 0
    tpr: int = 0
    rhs_per_task: int = 0
    alpha: float = 1.0
    max_iter: int = 1000


def _rows(t, length, name):
    torch = _torch()
    if t.dim() == 1:
        t = t.unsqueeze(0)
    if not t.is_cuda or t.dtype != torch.float64 or t.dim() != 2 or t.shape[1] != length \
            or t.stride(1) != 1:
        raise ValueError(f"{name} must be float64 GPU rows of length {length}")
    return t, (t.stride(0) if t.shape[0] > 1 else length)


def _batch_array(systems):
    n_sys = len(systems)
    arr = (_BatchSystem * n_sys)()
    dtypes = set()
    for i, S in enumerate(systems):
        code, m, n, lda = _matrix(S.A)
        dtypes.add(code)
        B, ldb = _rows(S.B, m, "B")
        X, ldx = _rows(S.X, n, "X")
        if B.shape[0] != X.shape[0]:
            raise ValueError("B and X must hold the same number of right-hand sides")
        XR, ldxr = (None, 0) if S.X_ref is None else _rows(S.X_ref, n, "X_ref")
        arr[i] = _BatchSystem(S.A.data_ptr(), m, n, lda, B.data_ptr(), ldb, X.data_ptr(), ldx,
                              None if XR is None else XR.data_ptr(), ldxr, B.shape[0], S.q,
                              S.block_size, S.tpr, S.rhs_per_task, 0, S.alpha, S.max_iter)
    if len(dtypes) != 1:
        raise ValueError("every system of a batch must have the same storage type")
    return arr, dtypes.pop()


def batch_tune(systems, *, seed=1, stream=None):
    """rka_batch_tune: fill q, block_size and tpr (where 0) of every
    BatchSystem from timed candidates; returns the number of candidates."""
    arr, code = _batch_array(systems)
    trials = ctypes.c_int32(0)
    _raise_if(lib().rka_batch_tune(arr, len(systems), code, seed, _stream(stream),
                                   ctypes.byref(trials)))
    for S, a in zip(systems, arr):
        S.q, S.block_size, S.tpr, S.alpha = a.q, a.block_size, a.tpr, a.alpha
    return trials.value


def batch_sample_indices(systems, *, seed=1, chunk_iters=0, stream=None):
    """rka_batch_sample_indices: the row streams a batch solve would draw
    (every system must give q and block_size), as one int32 GPU tensor per
    system of max_iter * q * block_size indices."""
    torch = _torch()
    arr, code = _batch_array(systems)
    sizes = [S.max_iter * S.q * S.block_size for S in systems]
    idx = torch.empty(max(1, sum(sizes)), dtype=torch.int32, device=systems[0].A.device)
    _raise_if(lib().rka_batch_sample_indices(arr, len(systems), code, seed, chunk_iters,
                                             _ptr(idx), _stream(stream)))
    out, off = [], 0
    for z in sizes:
        out.append(idx[off:off + z])
        off += z
    return out


def batch_solve(systems, *, seed=1, tol=0.0, check_every=1, chunk_iters=0, graph=True,
                refine_sweeps=0, stream=None, raise_on_error=True):
    """rka_batch_solve (or, with refine_sweeps > 0, rka_batch_refine_solve)
    over a list of BatchSystem.  Returns (results, stats):
    per-system dicts (iterations, rel, status, q, block_size, tpr,
    rhs_per_task) and launch facts.  With ``graph`` the launches run as one
    captured HIP graph on a side stream ordered after the current one."""
    torch = _torch()
    n_sys = len(systems)
    arr, code = _batch_array(systems)
    res = (_BatchResult * n_sys)()
    st = _BatchStats()
    cur = torch.cuda.current_stream()
    side = torch.cuda.Stream() if graph else None
    if side is not None:
        side.wait_stream(cur)
    run_on = side if side is not None else (stream or cur)
    if refine_sweeps > 0:
        status = lib().rka_batch_refine_solve(arr, n_sys, code, seed, tol, check_every,
                                              refine_sweeps, 1 if graph else 0,
                                              ctypes.c_void_p(run_on.cuda_stream), res,
                                              ctypes.byref(st))
    else:
        status = lib().rka_batch_solve(arr, n_sys, code, seed, tol, check_every, chunk_iters,
                                       1 if graph else 0, ctypes.c_void_p(run_on.cuda_stream),
                                       res, ctypes.byref(st))
    if side is not None:
        cur.wait_stream(side)
    if raise_on_error:
        _raise_if(status)
    out = [{f: getattr(r, f) for f, _ in _BatchResult._fields_ if f != "reserved"} for r in res]
    return out, {f: getattr(st, f) for f, _ in _BatchStats._fields_}


# -- host helpers --------------------------------------------------------------

def alpha_star(s_min: float, s_max: float, q: int) -> float:
    """Optimal uniform weight for consistent systems, Eq. (6) (Sec. 2.3.1),
    from s = sigma^2(A) / ||A||_F^2 at the extreme singular values
    (rka_alpha_star)."""
    a = ctypes.c_double()
    _raise_if(lib().rka_alpha_star(float(s_min), float(s_max), int(q), ctypes.byref(a)))
    return a.value
