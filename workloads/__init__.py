"""Seeded synthetic inputs for the symmetric tridiagonal eigenproblem T z = lambda z.

This module only *generates* matrices (diagonal ``d`` of length n and
off-diagonal ``e`` of length n-1); it contains no eigensolver arithmetic.  It is
the one piece shared by the CPU oracle, the HIP path, the tests and the
benchmark.  Every generator is deterministic in its ``seed`` (numpy PCG64
``default_rng``); FP32 inputs are drawn in FP64 and rounded to nearest.

Matrix families (stand-ins for the test types named in the paper's experiments
section: 1-2-1, Clement, Wilkinson, uniform/geometric eigenvalue distributions):

* ``uniform``            d, e ~ U(-1, 1)
* ``normal``             d, e ~ N(0, 1)
* ``toeplitz_121``       d = 2, e = 1, eigenvalues 2 + 2 cos(k pi / (n+1))
* ``clement``            d = 0, e_i = sqrt(i (n-i)), eigenvalues -(n-1), -(n-3), ..., n-1
* ``glued_wilkinson``    W21+ blocks (d_i = |10 - (i mod 21)|, e = 1) glued by 1e-10,
                         truncated at n
* ``prescribed_spectrum`` T with a prescribed spectrum (geometric magnitudes from
                         1 down to 1e-8, random signs) built from a Gaussian
                         start vector; see ``rkpw.c``
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "librkpw.so")
_lib = None


def _stale(lib: str, src: str) -> bool:
    return not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src)


def build_native(force: bool = False) -> str:
    """Compile the O(n^2) spectrum reconstruction helper with gcc."""
    if force or _stale(_LIB_PATH, os.path.join(_HERE, "rkpw.c")):
        src = os.path.join(_HERE, "rkpw.c")
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_native()
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.wl_rkpw.argtypes = [ctypes.c_int, dp, dp, dp, dp]
        lib.wl_rkpw.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _cast(d: np.ndarray, e: np.ndarray, dtype):
    return (np.ascontiguousarray(d, dtype=np.float64).astype(dtype),
            np.ascontiguousarray(e, dtype=np.float64).astype(dtype))


def uniform(n: int, seed: int = 0, dtype=np.float32):
    rng = np.random.default_rng(seed)
    d = rng.uniform(-1.0, 1.0, n)
    e = rng.uniform(-1.0, 1.0, max(n - 1, 0))
    return _cast(d, e, dtype)


def normal(n: int, seed: int = 0, dtype=np.float32):
    rng = np.random.default_rng(seed)
    d = rng.standard_normal(n)
    e = rng.standard_normal(max(n - 1, 0))
    return _cast(d, e, dtype)


def toeplitz_121(n: int, dtype=np.float32):
    return _cast(np.full(n, 2.0), np.full(max(n - 1, 0), 1.0), dtype)


def toeplitz_121_noisy(n: int, seed: int = 0, sigma: float = 1e-6, dtype=np.float32):
    """1-2-1 plus N(0, sigma^2) noise on d and e (sigma is a standard deviation)."""
    rng = np.random.default_rng(seed)
    d = 2.0 + sigma * rng.standard_normal(n)
    e = 1.0 + sigma * rng.standard_normal(max(n - 1, 0))
    return _cast(d, e, dtype)


def toeplitz_121_eigs(n: int) -> np.ndarray:
    """Closed-form eigenvalues of the 1-2-1 matrix in ascending order."""
    k = np.arange(n, 0, -1, dtype=np.float64)
    return 2.0 + 2.0 * np.cos(k * np.pi / (n + 1))


def clement(n: int, dtype=np.float32):
    i = np.arange(1, n, dtype=np.float64)
    return _cast(np.zeros(n), np.sqrt(i * (n - i)), dtype)


def glued_wilkinson(n: int, dtype=np.float64, block: int = 21, glue: float = 1e-10):
    half = block // 2
    i = np.arange(n)
    d = np.abs(half - (i % block)).astype(np.float64)
    e = np.ones(max(n - 1, 0))
    j = np.arange(max(n - 1, 0))
    e[(j + 1) % block == 0] = glue
    return _cast(d, e, dtype)


def prescribed_eigenvalues(n: int, seed: int = 0, smallest: float = 1e-8) -> np.ndarray:
    """Geometric magnitudes from 1 down to ``smallest`` with seeded random signs."""
    rng = np.random.default_rng(seed)
    mags = np.geomspace(1.0, smallest, n) if n > 1 else np.ones(n)
    signs = rng.choice(np.array([-1.0, 1.0]), size=n)
    return mags * signs


def prescribed_spectrum(n: int, seed: int = 0, smallest: float = 1e-8, dtype=np.float64):
    """Tridiagonal with the spectrum of ``prescribed_eigenvalues`` whose Lanczos
    start vector (first row of the eigenvector matrix) is a seeded N(0,1) draw.

    Returns ``(d, e, lam)`` where ``lam`` is the prescribed spectrum (unsorted).
    """
    lam = prescribed_eigenvalues(n, seed, smallest)
    rng = np.random.default_rng(seed + 7919)
    v = rng.standard_normal(n)
    w = v / np.linalg.norm(v) if n > 0 else v
    d = np.zeros(n)
    e = np.zeros(max(n - 1, 0))
    if n > 0:
        lib = _load()
        lam_c = np.ascontiguousarray(lam)
        w_c = np.ascontiguousarray(w)
        rc = lib.wl_rkpw(n, _ptr(lam_c), _ptr(w_c), _ptr(d), _ptr(e if n > 1 else np.zeros(1)))
        if rc != 0:
            raise RuntimeError("wl_rkpw failed")
    d, e = _cast(d, e, dtype)
    return d, e, lam


def lanczos_full_reorth(lam: np.ndarray, w: np.ndarray):
    """Plain n-step Lanczos on diag(lam) with full reorthogonalisation (twice).

    O(n^3); only for cross-checking ``prescribed_spectrum`` at small n.
    """
    n = lam.size
    Q = np.zeros((n, n))
    alpha = np.zeros(n)
    beta = np.zeros(max(n - 1, 0))
    q = w / np.linalg.norm(w)
    for k in range(n):
        Q[:, k] = q
        r = lam * q
        alpha[k] = q @ r
        for _ in range(2):
            r -= Q[:, :k + 1] @ (Q[:, :k + 1].T @ r)
        if k + 1 < n:
            beta[k] = np.linalg.norm(r)
            q = r / beta[k]
    return alpha, beta


def log_uniform_sizes(count: int, lo: int, hi: int, seed: int = 0) -> np.ndarray:
    """Sizes n = round(exp(U(ln lo, ln hi)))."""
    rng = np.random.default_rng(seed)
    return np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), count))).astype(np.int64)


def batch_normal(count: int = 4096, lo: int = 32, hi: int = 1024, seed: int = 0, dtype=np.float32):
    """Batched workload: ``count`` independent tridiagonals, n log-uniform in
    [lo, hi], d, e ~ N(0, 1).  Returns a list of (d, e)."""
    sizes = log_uniform_sizes(count, lo, hi, seed)
    return [normal(int(n), seed * 1_000_003 + 17 * i + 1, dtype) for i, n in enumerate(sizes)]


def served_requests(count: int, seed: int = 0, lo: int = 64, hi: int = 8192):
    """Request mix for the served stream: n log-uniform in [lo, hi], half FP32
    and half FP64 I/O, 30% asking for an index range covering 10% of the
    spectrum at a uniform random start, half U(-1,1) and half 1-2-1 plus
    N(0, 1e-6^2) noise.  Returns a list of dicts (arrival times are drawn by
    the caller from the chosen rate)."""
    rng = np.random.default_rng(seed)
    sizes = log_uniform_sizes(count, lo, hi, seed + 1)
    out = []
    for i, n in enumerate(sizes):
        n = int(n)
        dtype = np.float32 if rng.uniform() < 0.5 else np.float64
        if rng.uniform() < 0.5:
            d, e = uniform(n, seed * 7_000_003 + i, dtype)
            kind = "uniform"
        else:
            d, e = toeplitz_121_noisy(n, seed * 7_000_003 + i, 1e-6, dtype)
            kind = "121noisy"
        if rng.uniform() < 0.3:
            m = max(1, int(np.ceil(0.1 * n)))
            il = int(rng.integers(1, n - m + 2))
            rng_ = ("index", il, il + m - 1)
        else:
            rng_ = ("all", 1, n)
        out.append({"n": n, "dtype": dtype, "d": d, "e": e, "kind": kind, "range": rng_})
    return out


def random_unitary(n: int, seed: int = 0, complex_: bool = False) -> np.ndarray:
    """Seeded random orthogonal (or unitary) matrix: the Q factor of a
    Gaussian matrix with the signs (phases) of R's diagonal moved into Q, so
    that it is Haar distributed."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n))
    if complex_:
        G = G + 1j * rng.standard_normal((n, n))
    Q, R = np.linalg.qr(G)
    dg = np.diagonal(R).copy()
    dg[dg == 0] = 1.0
    return Q * (dg / np.abs(dg))


def dense_from_tridiagonal(d: np.ndarray, e: np.ndarray, seed: int = 0, complex_: bool = False,
                           dtype=None) -> np.ndarray:
    """The dense inputs of the paper's dense experiments: A = Q T Q^H for the
    tridiagonal T = (d, e) and a seeded random orthogonal (unitary) Q, formed
    in binary64 (complex128) and rounded to ``dtype`` (default: float64, or
    complex128 for the unitary case); exactly Hermitian."""
    n = d.size
    T = np.diag(d.astype(np.float64))
    if n > 1:
        T += np.diag(e.astype(np.float64), 1) + np.diag(e.astype(np.float64), -1)
    Q = random_unitary(n, seed, complex_)
    A = Q @ T @ Q.conj().T
    A = 0.5 * (A + A.conj().T)
    return A.astype(dtype or (np.complex128 if complex_ else np.float64))


def dense_normal(n: int, seed: int = 0, complex_: bool = False, dtype=None) -> np.ndarray:
    """Seeded random symmetric (Hermitian) matrix with N(0, 1) entries
    (default dtype float64, or complex128)."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, n))
    if complex_:
        G = G + 1j * rng.standard_normal((n, n))
    return (0.5 * (G + G.conj().T)).astype(dtype or (np.complex128 if complex_ else np.float64))
