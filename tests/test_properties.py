"""Property-based checks of the oracle (hypothesis, CPU only): on small
tridiagonals drawn with zeros, repeats, graded and mixed-scale entries, the
Sturm count equals the inertia of T - sigma I computed exactly in rationals,
the eigenvalues are sorted, lie in the Gerschgorin interval, sum to the trace
and their squares to the Frobenius norm, and the eigenvectors are orthonormal
with residuals at the gate.  Draws are derandomized, so a run is
reproducible."""
from fractions import Fraction

import numpy as np
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from tests import metrics as M

EPS = 2.0 ** -53

# Nonzero magnitudes stay above 2^-400: the squares of all entries, after the
# oracle's scaling to ||T||_1 in [1/2, 1), must be representable in binary64
# for a Sturm count to match the exact inertia (an eigenvalue of size
# e^2 ~ 2^-900 at a shift of exactly 0 is beyond any binary64 computation).
entry = st.one_of(
    st.floats(-1.0, 1.0, allow_nan=False, allow_infinity=False).filter(
        lambda x: x == 0.0 or abs(x) >= 2.0 ** -400),
    st.sampled_from([0.0, 1.0, -1.0, 0.5, 2.0 ** -30]),
    st.integers(-40, 40).map(lambda k: float(2.0 ** k)),
)


@st.composite
def tridiagonal(draw, nmax=10):
    n = draw(st.integers(1, nmax))
    d = np.array(draw(st.lists(entry, min_size=n, max_size=n)), dtype=np.float64)
    e = np.array(draw(st.lists(entry, min_size=max(n - 1, 0), max_size=max(n - 1, 0))),
                 dtype=np.float64)
    return d, e


def _exact_negcount(d, e, sigma):
    q, neg = None, 0
    for j in range(len(d)):
        t = Fraction(d[j]) - sigma
        if j > 0:
            if q == 0:
                return None
            t -= Fraction(e[j - 1]) ** 2 / q
        if t == 0:
            return None
        neg += t < 0
        q = t
    return neg


SETTINGS = settings(max_examples=150, deadline=None, derandomize=True, database=None,
                    suppress_health_check=[HealthCheck.too_slow])


@SETTINGS
@given(tridiagonal(), st.floats(-4.0, 4.0, allow_nan=False))
def test_count_is_exact_inertia(T, sigma):
    d, e = T
    ex = _exact_negcount(d, e, Fraction(sigma))
    if ex is not None:
        assert oracle.count(d, e if d.size > 1 else np.zeros(0), sigma) == ex


@SETTINGS
@given(tridiagonal())
def test_eigenvalue_invariants(T):
    d, e = T
    n = d.size
    ee = e if n > 1 else np.zeros(0)
    hi, lo = oracle.eigvals(d, ee)
    w = hi + lo
    tn = M.tnorm(d, ee)
    assert np.all(np.diff(w) >= 0)
    assert np.all(w >= -tn * (1 + 1e-15)) and np.all(w <= tn * (1 + 1e-15))
    # trace and Frobenius norm (exact up to the dd rounding of each eigenvalue)
    assert abs(float(np.sum(hi) + np.sum(lo)) - float(np.sum(d))) <= 8 * n * EPS * max(tn, 1e-300)
    fro = float(np.sum(d * d) + 2 * np.sum(ee * ee))
    assert abs(float(np.sum(w * w)) - fro) <= 16 * n * EPS * max(tn, 1e-300) ** 2


@SETTINGS
@given(tridiagonal(nmax=8))
def test_eigenvectors_at_the_gates(T):
    d, e = T
    n = d.size
    ee = e if n > 1 else np.zeros(0)
    hi, lo = oracle.eigvals(d, ee)
    Z = oracle.eigvecs(d, ee, hi, lo)
    assert M.orthogonality(Z) <= 10 * n * EPS
    assert M.residual(d, ee, hi + lo, Z) <= 10 * n * EPS


@settings(max_examples=60, deadline=None, derandomize=True, database=None,
          suppress_health_check=[HealthCheck.too_slow])
@given(tridiagonal(nmax=8), st.integers(-900, 900))
def test_power_of_two_scaling_is_exact(T, k):
    """T 2^k has eigenvalues lambda 2^k and the same eigenvectors, bit for
    bit, across the whole exponent range (the oracle scales its input to
    ||T||_1 in [1/2, 1) first, so its squares stay in range)."""
    d, e = T
    n = d.size
    ee = e if n > 1 else np.zeros(0)
    ds, es = np.ldexp(d, k), np.ldexp(ee, k)
    # skip draws whose scaled entries leave the normal range (inexact scaling)
    nz = np.concatenate([d[d != 0], ee[ee != 0]])
    if nz.size and (np.abs(np.ldexp(nz, k)).min() < 2.0 ** -1021 or np.abs(np.ldexp(nz, k)).max() > 2.0 ** 1000):
        return
    hi, lo = oracle.eigvals(d, ee)
    hs, ls = oracle.eigvals(ds, es)
    assert np.array_equal(hs, np.ldexp(hi, k)) and np.array_equal(ls, np.ldexp(lo, k))
    Z = oracle.eigvecs(d, ee, hi, lo)
    Zs = oracle.eigvecs(ds, es, hs, ls)
    assert np.array_equal(Z, Zs)
    assert np.all(np.isfinite(Zs))
