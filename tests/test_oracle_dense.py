"""Pins of the dense oracle (the reduction A = Q T Q^H of the dense
experiments, Sec. 4.2) against what the mathematics fixes: Q is unitary and
reproduces A, a tridiagonal input comes back with its own diagonal and
off-diagonal magnitudes, the eigenvalues agree with LAPACK's dense solver
(numpy.linalg.eigvalsh) and with a spectrum planted by a unitary similarity,
and plausible slips in the reduction (a lost conjugate, a wrong reflector
sign) fail these pins."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import dense as D

EPS = 2.0 ** -53


def _norm1(A):
    return float(np.abs(A).sum(axis=0).max())


def _pins(A, tol=1.0):
    """Largest pin ratios (<= tol passes) of the reduction of A."""
    n = A.shape[0]
    d, e, Q = D.tridiagonalize(A)
    T = np.diag(d) + (np.diag(e, 1) + np.diag(e, -1) if n > 1 else 0)
    unit = np.abs(Q.conj().T @ Q - np.eye(n)).max() / (10 * n * EPS)
    rec = np.abs(Q @ T @ Q.conj().T - A).max() / (10 * n * EPS * _norm1(A))
    hi, lo = oracle.eigvals(d, e if n > 1 else np.zeros(0))
    lap = np.abs(hi + lo - np.linalg.eigvalsh(A)).max() / (10 * n * EPS * _norm1(A))
    return max(unit, rec, lap), (d, e, Q)


@pytest.mark.parametrize("complex_", [False, True])
@pytest.mark.parametrize("n", [1, 2, 3, 17, 120])
def test_reduction_unitary_reconstructs_and_matches_lapack(n, complex_):
    A = W.dense_normal(n, 3 + n, complex_)
    worst, (d, e, Q) = _pins(A)
    assert worst <= 1.0, worst
    assert np.all(e >= 0)


def test_tridiagonal_input_comes_back():
    d, e = W.uniform(60, 4, np.float64)
    A = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    d2, e2, _ = D.tridiagonalize(A)
    assert np.abs(d2 - d).max() <= 10 * EPS * _norm1(A)
    assert np.abs(e2 - np.abs(e)).max() <= 10 * EPS * _norm1(A)


@pytest.mark.parametrize("complex_", [False, True])
def test_planted_spectrum(complex_):
    n = 90
    lam = np.sort(W.prescribed_eigenvalues(n, 5, 1e-6))
    U = W.random_unitary(n, 6, complex_)
    A = (U * lam[None, :]) @ U.conj().T
    A = 0.5 * (A + A.conj().T)
    hi, lo = D.eigvals(A)
    assert np.abs(hi + lo - lam).max() <= 10 * n * EPS * _norm1(A)


def test_dense_from_tridiagonal_keeps_the_spectrum():
    d, e, _ = W.prescribed_spectrum(80, 2)
    for cp in (False, True):
        A = W.dense_from_tridiagonal(d, e, 9, cp)
        assert np.allclose(A, A.conj().T, atol=0, rtol=0)
        hi, lo = D.eigvals(A)
        ref_hi, ref_lo = oracle.eigvals(d, e)
        assert np.abs((hi + lo) - (ref_hi + ref_lo)).max() <= 10 * 80 * EPS * _norm1(A)


def test_mutants_fail_the_pins(monkeypatch):
    """Each planted slip makes some pin fail."""
    A = W.dense_normal(40, 8, True)
    real = D.reflector
    mutants = {
        # a lost conjugate in the right-hand update
        "_apply_right": lambda M, v, tau: M.__isub__(tau * np.outer(M @ v, v)),
        # a lost conjugate in the left-hand update
        "_apply_left": lambda M, v, tau: M.__isub__(tau * np.outer(v, v @ M)),
        # a wrong reflector scale
        "reflector": lambda x: (lambda r: (r[0], 0.5 * r[1], r[2]))(real(x)),
    }
    for name, fn in mutants.items():
        monkeypatch.setattr(D, name, fn)
        assert _pins(A)[0] > 1.0, name
        monkeypatch.undo()
    assert _pins(A)[0] <= 1.0
