"""Plain CPU FP64 oracle for RKA / RKAB -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package.  The solver library never does, and
this package never imports the solver: the two share no code.

The arithmetic lives in ``rka_oracle.c`` (the paper's iterations) and
``forms_oracle.c`` (FP32 iterations, refinement, dense steps) -- plain C,
single thread, compiled with ``-O2 -ffp-contract=off`` -- and in
``lsq_grad.py`` (least-squares solution and gradient by FP64 QR); this module only marshals numpy arrays into
it through ctypes.  Each C function cites the passage of arXiv 2401.17474 it
follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "rka_oracle.c"), os.path.join(_HERE, "forms_oracle.c")]
LIB_PATH = os.path.join(_HERE, "liboracle.so")

OK, NOT_CONVERGED, EINVAL, EZERONORM, EDIVERGED = 0, 1, -1, -2, -3

_lib = None


def build() -> str:
    """Compile the oracle into ``oracle/liboracle.so`` (always recompiles)."""
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-Wall", "-Wextra", "-o", LIB_PATH + ".tmp", *_SRCS, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class _Info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("projections", ctypes.c_int64),
                ("rel_err", ctypes.c_double), ("status", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P, I64, I32, D, U64 = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                               ctypes.c_double, ctypes.c_uint64)
        L.oracle_philox4x32_10.argtypes = [P, P, P]
        L.oracle_philox4x32_10.restype = None
        L.oracle_uniform.argtypes = [U64, U64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]
        L.oracle_uniform.restype = D
        L.oracle_row_norms.argtypes = [P, ctypes.c_int, I64, I64, I64, P]
        L.oracle_prefix.argtypes = [P, I64, P]
        L.oracle_pick_row.argtypes = [P, P, I64, D]
        L.oracle_pick_row.restype = I64
        L.oracle_indices.argtypes = [P, I64, U64, I64, I64, I32, I32, I32, P]
        L.oracle_rka.argtypes = [P, ctypes.c_int, I64, I64, I64, P, P, P, I32, D, I64, D, U64,
                                 P, I64, I64, ctypes.POINTER(_Info)]
        L.oracle_rkab.argtypes = [P, ctypes.c_int, I64, I64, I64, P, P, P, I32, I32, D, I64, D,
                                  U64, P, I64, I64, ctypes.POINTER(_Info)]
        L.oracle_rka_given.argtypes = [P, ctypes.c_int, I64, I64, I64, P, P, I32, D, I64, P]
        L.oracle_rkab_given.argtypes = [P, ctypes.c_int, I64, I64, I64, P, P, I32, I32, D, I64,
                                        P]
        L.oracle_rka_f32_given.argtypes = [P, ctypes.c_int, I64, I64, I64, P, P, I32, D, I64, P]
        L.oracle_rkab_f32_given.argtypes = [P, ctypes.c_int, I64, I64, I64, P, P, I32, I32, D,
                                            I64, P]
        L.oracle_transpose.argtypes = [P, ctypes.c_int, I64, I64, I64, P]
        L.oracle_gemv.argtypes = [P, ctypes.c_int, I64, I64, I64, P, P, D, P]
        L.oracle_refine.argtypes = [P, ctypes.c_int, I64, I64, I64, P, P, P, I32, I32, I32, I32,
                                    D, I64, I64, I32, D, I32, U64, P, P]
        L.oracle_indices_blocks.argtypes = [P, I64, U64, I64, I64, I32, I32, I32, P]
        L.oracle_rka_walpha_given.argtypes = [P, ctypes.c_int, I64, I64, I64, P, P, I32, P, I64,
                                              P]
        L.oracle_rkab_walpha_given.argtypes = [P, ctypes.c_int, I64, I64, I64, P, P, I32, I32,
                                               P, I64, P]
        L.oracle_rka_wrow_given.argtypes = [P, ctypes.c_int, I64, I64, I64, P, P, I32, P, I64, P]
        L.oracle_rkab_wrow_given.argtypes = [P, ctypes.c_int, I64, I64, I64, P, P, I32, I32, P,
                                             I64, P]
        L.oracle_indices_cyclic.argtypes = [I64, I64, I64, I32, I32, P]
        L.oracle_ck.argtypes = [P, ctypes.c_int, I64, I64, I64, P, P, P, I64]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _matrix(A, dtype=None):
    """Return (array, dtype code, lda).  bfloat16 is passed as uint16 bits
    with ``dtype='bf16'``."""
    A = np.asarray(A)
    if A.ndim != 2 or A.strides[1] != A.itemsize or A.strides[0] % A.itemsize:
        A = np.ascontiguousarray(A)
    if dtype == "bf16" or A.dtype == np.uint16:
        if A.dtype != np.uint16:
            raise TypeError("bf16 matrices are passed as uint16 bit patterns")
        code = 2
    elif A.dtype == np.float64:
        code = 0
    elif A.dtype == np.float32:
        code = 1
    else:
        raise TypeError(f"unsupported matrix dtype {A.dtype}")
    lda = A.strides[0] // A.itemsize if A.shape[0] > 1 else A.shape[1]
    return A, code, lda


def _vec(v, n):
    if v is None:
        return None
    v = np.ascontiguousarray(v, dtype=np.float64)
    if v.shape != (n,):
        raise ValueError(f"expected a vector of length {n}, got {v.shape}")
    return v


def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return [int(v) for v in out]


def uniform(seed, k, w, j, dom=0):
    return lib().oracle_uniform(seed, k, w, j, dom)


def row_norms(A, dtype=None):
    A, code, lda = _matrix(A, dtype)
    m, n = A.shape
    w = np.zeros(m, dtype=np.float64)
    st = lib().oracle_row_norms(_ptr(A), code, m, n, lda, _ptr(w))
    if st != OK:
        raise ValueError(f"oracle_row_norms status {st}")
    return w


def prefix(w):
    w = np.ascontiguousarray(w, dtype=np.float64)
    c = np.zeros_like(w)
    st = lib().oracle_prefix(_ptr(w), w.shape[0], _ptr(c))
    return c, st


def pick_row(c, w, u):
    c = np.ascontiguousarray(c, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    return int(lib().oracle_pick_row(_ptr(c), _ptr(w), c.shape[0], float(u)))


def indices(w, seed, iter_offset, K, q, bs=1, dom=0):
    w = np.ascontiguousarray(w, dtype=np.float64)
    idx = np.zeros(K * q * bs, dtype=np.int32)
    st = lib().oracle_indices(_ptr(w), w.shape[0], seed, iter_offset, K, q, bs, dom, _ptr(idx))
    if st != OK:
        raise ValueError(f"oracle_indices status {st}")
    return idx


def _info(i):
    return {"iterations": i.iterations, "projections": i.projections, "rel_err": i.rel_err,
            "status": i.status}


def rka(A, b, *, q, alpha=1.0, max_iter=1000, tol=0.0, seed=1, x0=None, x_ref=None,
        iter_offset=0, check_every=1, dtype=None):
    A, code, lda = _matrix(A, dtype)
    m, n = A.shape
    b = _vec(b, m)
    x = np.zeros(n, dtype=np.float64)
    info = _Info()
    lib().oracle_rka(_ptr(A), code, m, n, lda, _ptr(b), _ptr(_vec(x0, n)), _ptr(x), q, alpha,
                     max_iter, tol, seed, _ptr(_vec(x_ref, n)), iter_offset, check_every,
                     ctypes.byref(info))
    return x, _info(info)


def rkab(A, b, *, q, block_size, alpha=1.0, max_iter=1000, tol=0.0, seed=1, x0=None,
         x_ref=None, iter_offset=0, check_every=1, dtype=None):
    A, code, lda = _matrix(A, dtype)
    m, n = A.shape
    b = _vec(b, m)
    x = np.zeros(n, dtype=np.float64)
    info = _Info()
    lib().oracle_rkab(_ptr(A), code, m, n, lda, _ptr(b), _ptr(_vec(x0, n)), _ptr(x), q,
                      block_size, alpha, max_iter, tol, seed, _ptr(_vec(x_ref, n)), iter_offset,
                      check_every, ctypes.byref(info))
    return x, _info(info)


def rka_given(A, b, x, idx, *, q, alpha=1.0, dtype=None):
    A, code, lda = _matrix(A, dtype)
    m, n = A.shape
    x = np.array(x, dtype=np.float64, copy=True)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    K = idx.size // q
    st = lib().oracle_rka_given(_ptr(A), code, m, n, lda, _ptr(_vec(b, m)), _ptr(x), q, alpha,
                                K, _ptr(idx))
    if st != OK:
        raise ValueError(f"oracle_rka_given status {st}")
    return x


def rkab_given(A, b, x, idx, *, q, block_size, alpha=1.0, dtype=None):
    A, code, lda = _matrix(A, dtype)
    m, n = A.shape
    x = np.array(x, dtype=np.float64, copy=True)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    K = idx.size // (q * block_size)
    st = lib().oracle_rkab_given(_ptr(A), code, m, n, lda, _ptr(_vec(b, m)), _ptr(x), q,
                                 block_size, alpha, K, _ptr(idx))
    if st != OK:
        raise ValueError(f"oracle_rkab_given status {st}")
    return x


# -- forms built on the iterations (forms_oracle.c) ----------------------------

def rka_f32_given(A, b, x, idx, *, q, alpha=1.0, dtype=None):
    """RKA with every iteration quantity in binary32 (A float32 or bf16 bits)."""
    A, code, lda = _matrix(A, dtype)
    m, n = A.shape
    x = np.array(x, dtype=np.float64, copy=True)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    K = idx.size // q
    st = lib().oracle_rka_f32_given(_ptr(A), code, m, n, lda, _ptr(_vec(b, m)), _ptr(x), q,
                                    alpha, K, _ptr(idx))
    if st != OK:
        raise ValueError(f"oracle_rka_f32_given status {st}")
    return x


def rkab_f32_given(A, b, x, idx, *, q, block_size, alpha=1.0, dtype=None):
    """RKAB with every iteration quantity in binary32."""
    A, code, lda = _matrix(A, dtype)
    m, n = A.shape
    x = np.array(x, dtype=np.float64, copy=True)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    K = idx.size // (q * block_size)
    st = lib().oracle_rkab_f32_given(_ptr(A), code, m, n, lda, _ptr(_vec(b, m)), _ptr(x), q,
                                     block_size, alpha, K, _ptr(idx))
    if st != OK:
        raise ValueError(f"oracle_rkab_f32_given status {st}")
    return x


def transpose(A, dtype=None):
    A, code, lda = _matrix(A, dtype)
    m, n = A.shape
    At = np.empty((n, m), dtype=A.dtype)
    if lib().oracle_transpose(_ptr(A), code, m, n, lda, _ptr(At)) != OK:
        raise ValueError("oracle_transpose failed")
    return At


def gemv(M, v, *, c=None, gamma=1.0, dtype=None):
    M, code, ld = _matrix(M, dtype)
    rows, cols = M.shape
    out = np.empty(rows, dtype=np.float64)
    if lib().oracle_gemv(_ptr(M), code, rows, cols, ld, _ptr(_vec(v, cols)),
                         _ptr(_vec(c, rows)), gamma, _ptr(out)) != OK:
        raise ValueError("oracle_gemv failed")
    return out


def refine(A, b, *, method=0, q, block_size=1, acc32=1, alpha=1.0, inner_iters,
           range_iters=0, range_q=1, range_alpha=1.0, sweeps, seed=1, x0=None, x_ref=None,
           dtype=None):
    """Refinement sweeps; returns (x, per-sweep measures)."""
    A, code, lda = _matrix(A, dtype)
    m, n = A.shape
    x = np.zeros(n, dtype=np.float64)
    meas = np.zeros(sweeps, dtype=np.float64)
    st = lib().oracle_refine(_ptr(A), code, m, n, lda, _ptr(_vec(b, m)), _ptr(_vec(x0, n)),
                             _ptr(x), method, q, block_size, acc32, alpha, inner_iters,
                             range_iters, range_q, range_alpha, sweeps, seed,
                             _ptr(_vec(x_ref, n)), _ptr(meas))
    if st != OK:
        raise ValueError(f"oracle_refine status {st}")
    return x, meas


# -- the Distributed Approach and per-worker weights (Sec. 3.3.2) ---------------

def indices_blocks(w, seed, iter_offset, K, q, bs=1, dom=0):
    """Row stream with worker w restricted to its own row block."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    idx = np.empty(K * q * bs, dtype=np.int32)
    st = lib().oracle_indices_blocks(_ptr(w), w.size, seed, iter_offset, K, q, bs, dom, _ptr(idx))
    if st != OK:
        raise ValueError(f"oracle_indices_blocks status {st}")
    return idx


def rka_walpha_given(A, b, x, idx, walpha, *, q, dtype=None):
    A, code, lda = _matrix(A, dtype)
    m, n = A.shape
    x = np.array(x, dtype=np.float64, copy=True)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    wa = np.ascontiguousarray(walpha, dtype=np.float64)
    st = lib().oracle_rka_walpha_given(_ptr(A), code, m, n, lda, _ptr(_vec(b, m)), _ptr(x), q,
                                       _ptr(wa), idx.size // q, _ptr(idx))
    if st != OK:
        raise ValueError(f"oracle_rka_walpha_given status {st}")
    return x


def rkab_walpha_given(A, b, x, idx, walpha, *, q, block_size, dtype=None):
    A, code, lda = _matrix(A, dtype)
    m, n = A.shape
    x = np.array(x, dtype=np.float64, copy=True)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    wa = np.ascontiguousarray(walpha, dtype=np.float64)
    st = lib().oracle_rkab_walpha_given(_ptr(A), code, m, n, lda, _ptr(_vec(b, m)), _ptr(x), q,
                                        block_size, _ptr(wa), idx.size // (q * block_size),
                                        _ptr(idx))
    if st != OK:
        raise ValueError(f"oracle_rkab_walpha_given status {st}")
    return x


# -- row weights of Eq. (7) and the cyclic order of Sec. 2.1 ---------------------

def rka_wrow_given(A, b, x, idx, wrow, *, q, dtype=None):
    """RKA on a given stream with per-row weights w_i (Eq. (7))."""
    A, code, lda = _matrix(A, dtype)
    m, n = A.shape
    x = np.array(x, dtype=np.float64, copy=True)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    wr = _vec(wrow, m)
    st = lib().oracle_rka_wrow_given(_ptr(A), code, m, n, lda, _ptr(_vec(b, m)), _ptr(x), q,
                                     _ptr(wr), idx.size // q, _ptr(idx))
    if st != OK:
        raise ValueError(f"oracle_rka_wrow_given status {st}")
    return x


def rkab_wrow_given(A, b, x, idx, wrow, *, q, block_size, dtype=None):
    """RKAB on a given stream with per-row weights w_i."""
    A, code, lda = _matrix(A, dtype)
    m, n = A.shape
    x = np.array(x, dtype=np.float64, copy=True)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    wr = _vec(wrow, m)
    st = lib().oracle_rkab_wrow_given(_ptr(A), code, m, n, lda, _ptr(_vec(b, m)), _ptr(x), q,
                                      block_size, _ptr(wr), idx.size // (q * block_size),
                                      _ptr(idx))
    if st != OK:
        raise ValueError(f"oracle_rkab_wrow_given status {st}")
    return x


def indices_cyclic(m, iter_offset, K, q, bs=1):
    """The cyclic row order: draw (k, w, j) takes row ((k+off)q+w)bs+j mod m."""
    idx = np.empty(K * q * bs, dtype=np.int32)
    st = lib().oracle_indices_cyclic(m, iter_offset, K, q, bs, _ptr(idx))
    if st != OK:
        raise ValueError(f"oracle_indices_cyclic status {st}")
    return idx


def ck(A, b, *, iters, relax=None, x0=None, dtype=None):
    """Cyclic Kaczmarz (Sec. 2.1): iters projections onto rows 0, 1, ... in
    turn, row i relaxed by relax[i] (default 1), from x0 (default zero)."""
    A, code, lda = _matrix(A, dtype)
    m, n = A.shape
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    rl = None if relax is None else _vec(relax, m)
    st = lib().oracle_ck(_ptr(A), code, m, n, lda, _ptr(_vec(b, m)), _ptr(x),
                         None if rl is None else _ptr(rl), iters)
    if st != OK:
        raise ValueError(f"oracle_ck status {st}")
    return x
