"""ORACLE -- test infrastructure only.

The dense symmetric / Hermitian eigenproblem of the paper's dense experiments
(Sec. 4.2, Fig. 3): A is brought to a real symmetric tridiagonal T by the
textbook Householder reduction (for k = 0 .. n-3 one reflector
H_k = I - tau v v^H annihilates A[k+2:, k] and is applied from both sides),
a diagonal unitary scaling then makes the off-diagonal real and non-negative
(the Hermitian case), and T's eigenvalues come from the tridiagonal oracle
(double-double bisection).  numpy, binary64 / complex128, O(n^3) rank-one
updates: for n up to a few thousand.

Same import rules as the rest of the oracle: only the tests, the smoke check
and the benchmark's CPU-baseline leg use it; it imports nothing of the
product.

reflector(x)          -> (v, tau, alpha) with (I - tau v v^H) x = alpha e_1
tridiagonalize(A)     -> (d, e, Q): Q unitary, Q^H A Q = tridiag(e, d, e), e >= 0
eigvals(A, il, iu)    -> (w_hi, w_lo) double-double eigenvalues il..iu of T
"""
from __future__ import annotations

import numpy as np


def reflector(x: np.ndarray):
    """Householder vector for x: v = x - alpha e_1 with alpha = -phase(x_0)
    ||x||, tau = 2 / (v^H v), so that (I - tau v v^H) x = alpha e_1 and the
    subtraction in v_0 adds magnitudes (no cancellation)."""
    nx = float(np.linalg.norm(x))
    if nx == 0.0:
        return np.zeros_like(x), 0.0, 0.0 * x[0]
    x0 = x[0]
    phase = x0 / abs(x0) if x0 != 0 else 1.0
    alpha = -phase * nx
    v = x.copy()
    v[0] = x0 - alpha
    tau = 2.0 / float(np.real(np.vdot(v, v)))
    return v, tau, alpha


def _apply_left(M: np.ndarray, v: np.ndarray, tau: float) -> None:
    """M := (I - tau v v^H) M, as a rank-one update."""
    M -= tau * np.outer(v, v.conj() @ M)


def _apply_right(M: np.ndarray, v: np.ndarray, tau: float) -> None:
    """M := M (I - tau v v^H), as a rank-one update."""
    M -= tau * np.outer(M @ v, v.conj())


def tridiagonalize(A: np.ndarray):
    n = A.shape[0]
    cplx = np.iscomplexobj(A)
    T = np.array(A, dtype=np.complex128 if cplx else np.float64)
    Q = np.eye(n, dtype=T.dtype)
    for k in range(n - 2):
        v, tau, _ = reflector(T[k + 1:, k].copy())
        if tau == 0.0:
            continue
        _apply_left(T[k + 1:, :], v, tau)
        _apply_right(T[:, k + 1:], v, tau)
        _apply_right(Q[:, k + 1:], v, tau)
    d = np.real(np.diagonal(T)).copy()
    off = np.array([T[k + 1, k] for k in range(n - 1)])
    # D^H T D with D = diag(s), s_0 = 1, s_{k+1} = s_k * phase(off_k): the
    # off-diagonal becomes |off_k|; Q D carries the scaling
    s = np.ones(n, dtype=T.dtype)
    for k in range(n - 1):
        a = abs(off[k])
        s[k + 1] = s[k] * (off[k] / a if a != 0 else 1.0)
    e = np.abs(off).astype(np.float64)
    return d, e, Q * s[None, :]


def eigvals(A: np.ndarray, il: int = 1, iu: int | None = None):
    """Double-double eigenvalues il..iu (1-based) of A through T."""
    from . import eigvals as tri_eigvals

    d, e, _ = tridiagonalize(A)
    return tri_eigvals(d, e if e.size else np.zeros(0), il, iu)
