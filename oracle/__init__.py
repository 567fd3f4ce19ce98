"""CPU oracle for the signature kernel (arXiv 2502.20392, Sec. 2).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU
library never imports it and it never imports the GPU library; the two share
no code.

Functions (all FP64 in/out, numpy arrays, row-major ``[length, d]`` paths):

* ``pair(x, y)``            k(x, y) by the raster sweep of the tile-centred
                             series (Prop. 2.8), per-cell truncation to 2^-64.
* ``pair_ld(x, y)``         the same computed in long double (80-bit), used to
                             bound the double version's rounding.
* ``pair_diag(x, y)``       k plus diagnostics (corner mismatch, orders used).
* ``gram(X, Y, sym)``       Gram matrix over a thread pool (one pair per task).
* ``ragged(pool, offsets, pairs)``  kernel values for a list of path pairs.
* ``grad(x, y)``            continuous adjoint: (k, dk/dx, dk/dy).
* ``pair_fixed(x, y, N)``   the fixed-order approximant k^[N] (tiles keep their
                             (N+1) x (N+1) coefficient matrix).
* ``cell(a, b, c, N)``      one cell's coefficient matrix and edge series.
"""
import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle_sigk.so")
_lib = None
_lock = threading.Lock()

_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)
_I32 = ctypes.POINTER(ctypes.c_int32)
_LD = ctypes.POINTER(ctypes.c_longdouble)


class OracleError(RuntimeError):
    pass


_ERRS = {-1: "invalid argument", -2: "out of memory",
         -5: "more than 160 series coefficients needed in a cell"}


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(_LIB_PATH)
        for sfx, kt in (("_f64", _D), ("_ld", _LD)):
            f = getattr(lib, "sigk_oracle_pair" + sfx)
            f.argtypes = [_D, ctypes.c_int64, _D, ctypes.c_int64, ctypes.c_int64, _D, kt, _D]
            f.restype = ctypes.c_int
            f = getattr(lib, "sigk_oracle_ragged" + sfx)
            f.argtypes = [_D, _I64, ctypes.c_int64, ctypes.c_int64, _I32, ctypes.c_int64, _D,
                          ctypes.c_int]
            f.restype = ctypes.c_int
            f = getattr(lib, "sigk_oracle_grad" + sfx)
            f.argtypes = [_D, ctypes.c_int64, _D, ctypes.c_int64, ctypes.c_int64, _D, _D, _D]
            f.restype = ctypes.c_int
            f = getattr(lib, "sigk_oracle_pair_fixed" + sfx)
            f.argtypes = [_D, ctypes.c_int64, _D, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                          _D]
            f.restype = ctypes.c_int
            f = getattr(lib, "sigk_oracle_cell" + sfx)
            f.argtypes = [_D, ctypes.c_int, _D, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                          _D, _D, _D]
            f.restype = ctypes.c_int
        _lib = lib
        return lib


def _path(z):
    z = np.ascontiguousarray(z, dtype=np.float64)
    if z.ndim != 2:
        raise ValueError("path must be 2-D [length, d]")
    return z


def _ptr(a, typ=_D):
    return a.ctypes.data_as(typ)


def _check(rc):
    if rc != 0:
        raise OracleError(_ERRS.get(rc, f"oracle error {rc}"))


def pair(x, y):
    """k(x, y) in double."""
    x, y = _path(x), _path(y)
    if x.shape[1] != y.shape[1]:
        raise ValueError("dimension mismatch")
    out = ctypes.c_double()
    _check(_load().sigk_oracle_pair_f64(_ptr(x), x.shape[0], _ptr(y), y.shape[0], x.shape[1],
                                        ctypes.byref(out), None, None))
    return out.value


def pair_diag(x, y):
    """(k, diag) with diag = [corner mismatch, max N, top/right mismatch, max edge length]."""
    x, y = _path(x), _path(y)
    out = ctypes.c_double()
    diag = np.zeros(4)
    _check(_load().sigk_oracle_pair_f64(_ptr(x), x.shape[0], _ptr(y), y.shape[0], x.shape[1],
                                        ctypes.byref(out), None, _ptr(diag)))
    return out.value, diag


def pair_ld(x, y):
    """k(x, y) computed in long double; returned as a numpy longdouble."""
    x, y = _path(x), _path(y)
    out = ctypes.c_double()
    ext = ctypes.c_longdouble()
    _check(_load().sigk_oracle_pair_ld(_ptr(x), x.shape[0], _ptr(y), y.shape[0], x.shape[1],
                                       ctypes.byref(out), ctypes.byref(ext), None))
    return np.longdouble(ext.value)


def ragged(pool, offsets, pairs, nthreads=0):
    """Kernel values for path pairs of a concatenated pool ``[sum len, d]``."""
    pool = _path(pool)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    out = np.zeros(pairs.shape[0])
    _check(_load().sigk_oracle_ragged_f64(_ptr(pool), _ptr(offsets, _I64), offsets.shape[0] - 1,
                                          pool.shape[1], _ptr(pairs, _I32), pairs.shape[0],
                                          _ptr(out), int(nthreads)))
    return out


def gram(X, Y=None, symmetric=None, nthreads=0):
    """Gram matrix G[i, j] = k(X[i], Y[j]) for equal-length batches ``[n, len, d]``."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    if Y is None:
        Y = X
        if symmetric is None:
            symmetric = True
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    nx, lx, d = X.shape
    ny, ly, _ = Y.shape
    pool = np.concatenate([X.reshape(-1, d), Y.reshape(-1, d)], axis=0)
    offsets = np.concatenate([np.arange(nx + 1) * lx, nx * lx + np.arange(1, ny + 1) * ly])
    if symmetric:
        idx = [(i, j) for i in range(nx) for j in range(i, ny)]
    else:
        idx = [(i, j) for i in range(nx) for j in range(ny)]
    pairs = np.array([(i, nx + j) for i, j in idx], dtype=np.int32)
    vals = ragged(pool, offsets, pairs, nthreads)
    G = np.zeros((nx, ny))
    for (i, j), v in zip(idx, vals):
        G[i, j] = v
        if symmetric:
            G[j, i] = v
    return G


def grad(x, y, extended=False):
    """(k, dk/dx, dk/dy) by the continuous adjoint (Riemann function) formula."""
    x, y = _path(x), _path(y)
    out = ctypes.c_double()
    gx = np.zeros_like(x)
    gy = np.zeros_like(y)
    fn = _load().sigk_oracle_grad_ld if extended else _load().sigk_oracle_grad_f64
    _check(fn(_ptr(x), x.shape[0], _ptr(y), y.shape[0], x.shape[1], ctypes.byref(out),
              _ptr(gx), _ptr(gy)))
    return out.value, gx, gy


def pair_fixed(x, y, N):
    """k^[N](x, y): every tile keeps its (N+1) x (N+1) coefficient matrix (the
    fixed-order approximant of the paper's error analysis)."""
    x, y = _path(x), _path(y)
    if x.shape[1] != y.shape[1]:
        raise ValueError("dimension mismatch")
    out = ctypes.c_double()
    _check(_load().sigk_oracle_pair_fixed_f64(_ptr(x), x.shape[0], _ptr(y), y.shape[0],
                                              x.shape[1], int(N), ctypes.byref(out)))
    return out.value


def cell(a, b, c, N):
    """One cell: returns (C [N, N], top [N], right [N]) for monomial edge series a, b."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    C = np.zeros((N, N))
    top = np.zeros(N)
    right = np.zeros(N)
    _check(_load().sigk_oracle_cell_f64(_ptr(a), a.shape[0], _ptr(b), b.shape[0], float(c),
                                        int(N), _ptr(C), _ptr(top), _ptr(right)))
    return C, top, right
