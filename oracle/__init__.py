"""ORACLE -- test infrastructure only.

Python access to the plain CPU reference solver in ``oracle.c`` (double-double
Sturm bisection + inverse iteration for the symmetric tridiagonal eigenproblem
of the paper's introduction).  Only the tests, ``__graft_entry__.smoke`` and
the benchmark's CPU-baseline leg may import this package; the product path
never does, and this package never imports the product package.

Functions
---------
eigvals(d, e, il, iu)        -> (w_hi, w_lo) double-double eigenvalues il..iu
eigvecs(d, e, w_hi, w_lo)    -> Z (n x m, FP64, column-major as numpy F-order)
solve(d, e, il, iu)          -> (w, Z) convenience wrapper
count(d, e, sigma)           -> number of eigenvalues strictly below sigma
dd_op(op, a, b)              -> double-double primitive, for pinning
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _stale(lib: str, src: str) -> bool:
    return not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src)


def build(force: bool = False, out: str | None = None, mutant: int = 0) -> str:
    """Compile the oracle with gcc (-O2 -fopenmp).  ``mutant`` > 0 builds a
    deliberately wrong variant into ``out`` (used only by the pin tests)."""
    path = out or _LIB_PATH
    if force or mutant or _stale(path, os.path.join(_HERE, "oracle.c")):
        tmp = path + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp,
                               f"-DORACLE_MUTANT={int(mutant)}",
                               os.path.join(_HERE, "oracle.c"), "-lm"])
        os.replace(tmp, path)
    return path


def use_library(path: str | None) -> None:
    """Point this module at another build of oracle.c (None = the real one)."""
    global _lib
    _lib = None
    _load(path)


def _load(path: str | None = None):
    global _lib
    if _lib is None:
        path = path or _LIB_PATH
        if path == _LIB_PATH and not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        i = ctypes.c_int
        lib.oracle_eigvals.argtypes = [i, dp, dp, i, i, dp, dp, i]
        lib.oracle_eigvals.restype = i
        lib.oracle_count.argtypes = [i, dp, dp, ctypes.c_double, ctypes.c_double]
        lib.oracle_count.restype = i
        lib.oracle_eigvecs.argtypes = [i, dp, dp, i, dp, dp, dp, ctypes.c_ulonglong,
                                       ctypes.c_double, i]
        lib.oracle_eigvecs.restype = i
        lib.oracle_tnorm.argtypes = [i, dp, dp]
        lib.oracle_tnorm.restype = ctypes.c_double
        lib.oracle_dd_op.argtypes = [i, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, dp, dp]
        lib.oracle_dd_op.restype = None
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _prep(d, e):
    d = np.ascontiguousarray(np.asarray(d, dtype=np.float64))
    n = d.size
    e = np.ascontiguousarray(np.asarray(e, dtype=np.float64).reshape(-1)[: max(n - 1, 0)])
    if e.size == 0:
        e = np.zeros(1)
    return n, d, e


def eigvals(d, e, il: int = 1, iu: int | None = None, threads: int = 0):
    n, d, e = _prep(d, e)
    if iu is None:
        iu = n
    m = max(iu - il + 1, 0)
    w_hi = np.zeros(max(m, 1))
    w_lo = np.zeros(max(m, 1))
    rc = _load().oracle_eigvals(n, _p(d), _p(e), il, iu, _p(w_hi), _p(w_lo), threads)
    if rc != 0:
        raise ValueError(f"oracle_eigvals: bad arguments (rc={rc})")
    return w_hi[:m], w_lo[:m]


def eigvecs(d, e, w_hi, w_lo, seed: int = 12345, group_tol: float = 0.0, threads: int = 0):
    n, d, e = _prep(d, e)
    w_hi = np.ascontiguousarray(w_hi, dtype=np.float64)
    w_lo = np.ascontiguousarray(w_lo, dtype=np.float64)
    m = w_hi.size
    z = np.zeros((max(m, 1), max(n, 1)))  # row k = eigenvector k (column-major n x m)
    rc = _load().oracle_eigvecs(n, _p(d), _p(e), m, _p(w_hi), _p(w_lo), _p(z), seed,
                                group_tol, threads)
    if rc != 0:
        raise ValueError(f"oracle_eigvecs: bad arguments (rc={rc})")
    return z[:m, :n].T.copy()


def solve(d, e, il: int = 1, iu: int | None = None, seed: int = 12345, threads: int = 0):
    w_hi, w_lo = eigvals(d, e, il, iu, threads)
    Z = eigvecs(d, e, w_hi, w_lo, seed=seed, threads=threads)
    return w_hi + w_lo, Z


def count(d, e, sigma_hi: float, sigma_lo: float = 0.0) -> int:
    n, d, e = _prep(d, e)
    return int(_load().oracle_count(n, _p(d), _p(e), float(sigma_hi), float(sigma_lo)))


def tnorm(d, e) -> float:
    n, d, e = _prep(d, e)
    return float(_load().oracle_tnorm(n, _p(d), _p(e)))


_OPS = {"add": 0, "sub": 1, "mul": 2, "div": 3, "sqrt": 4}


def dd_op(op: str, a, b=(0.0, 0.0)):
    rh = ctypes.c_double()
    rl = ctypes.c_double()
    lib = _load()
    lib.oracle_dd_op(_OPS[op], float(a[0]), float(a[1]), float(b[0]), float(b[1]),
                     ctypes.byref(rh), ctypes.byref(rl))
    return rh.value, rl.value
