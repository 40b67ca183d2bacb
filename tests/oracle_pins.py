"""Pins for the CPU oracle: checks against facts that do not come from the oracle
itself -- exact rational arithmetic, closed forms, brute-force Jacobi in
multiprecision, trace invariants, Weyl-bound multiplicity counts and a
prescribed spectrum.  Each ``pin_*`` returns (ok, detail) so that the mutant
test can run them against deliberately broken builds of the oracle.
"""
from __future__ import annotations

from fractions import Fraction

import mpmath
import numpy as np

import oracle
import workloads as W

U = 2.0 ** -53


def _frac_dd(hi, lo):
    return Fraction(hi) + Fraction(lo)


def _sin_angle(u, v):
    """sin of the angle between two vectors, accurate for tiny angles."""
    u = u / np.linalg.norm(u)
    v = v / np.linalg.norm(v)
    if u @ v < 0:
        v = -v
    return float(np.linalg.norm(u - (u @ v) * v))


# --------------------------------------------------------------------------
# double-double primitives vs exact rationals
# --------------------------------------------------------------------------
def pin_dd_ops(seed=0, trials=300):
    rng = np.random.default_rng(seed)
    worst = 0.0
    for t in range(trials):
        ah = rng.uniform(-1, 1) * 2.0 ** rng.integers(-20, 20)
        al = ah * rng.uniform(-1, 1) * U
        bh = rng.uniform(-1, 1) * 2.0 ** rng.integers(-20, 20)
        if t % 5 == 0:  # near-cancellation for add/sub
            bh = -ah * (1 + rng.uniform(-1, 1) * 1e-12)
        bl = bh * rng.uniform(-1, 1) * U
        A, B = _frac_dd(ah, al), _frac_dd(bh, bl)
        for op, exact in (("add", A + B), ("sub", A - B), ("mul", A * B), ("div", A / B)):
            r = _frac_dd(*oracle.dd_op(op, (ah, al), (bh, bl)))
            if exact == 0:
                err = abs(float(r))
            else:
                err = abs(float((r - exact) / exact))
            worst = max(worst, err)
        if ah > 0:
            r = oracle.dd_op("sqrt", (ah, al))
            exact2 = A
            r2 = _frac_dd(*r) ** 2
            worst = max(worst, abs(float((r2 - exact2) / exact2)) / 2)
    # published double-double bounds are small multiples of u^2 = 2^-106
    return worst <= 2.0 ** -100, f"worst relative error {worst:.3e}"


# --------------------------------------------------------------------------
# Sturm count == inertia (exact rational LDL^T) on tiny matrices
# --------------------------------------------------------------------------
def _exact_negcount(d, e, sigma):
    q = None
    neg = 0
    for j in range(len(d)):
        t = Fraction(d[j]) - sigma
        if j > 0:
            t -= Fraction(e[j - 1]) ** 2 / q
        if t == 0:
            return None  # sigma hits a leading-submatrix eigenvalue; skip
        if t < 0:
            neg += 1
        q = t
    return neg


def pin_sturm_inertia(seed=1, trials=60):
    rng = np.random.default_rng(seed)
    bad = 0
    for _ in range(trials):
        n = int(rng.integers(1, 9))
        d = rng.uniform(-1, 1, n)
        e = rng.uniform(-1, 1, max(n - 1, 0))
        s = float(rng.uniform(-3, 3))
        ex = _exact_negcount(d, e, Fraction(s))
        if ex is None:
            continue
        if oracle.count(d, e, s) != ex:
            bad += 1
    return bad == 0, f"{bad} mismatches"


# --------------------------------------------------------------------------
# eigenvalues: closed forms and brute force
# --------------------------------------------------------------------------
def _oracle_vals_mp(d, e, il=1, iu=None):
    hi, lo = oracle.eigvals(d, e, il, iu)
    return [mpmath.mpf(h) + mpmath.mpf(l) for h, l in zip(hi, lo)]


def pin_121_eigenvalues(n=97):
    mpmath.mp.dps = 40
    d, e = W.toeplitz_121(n, np.float64)
    got = _oracle_vals_mp(d, e)
    exact = sorted(2 + 2 * mpmath.cos(k * mpmath.pi / (n + 1)) for k in range(1, n + 1))
    err = max(abs(g - x) for g, x in zip(got, exact))
    return err <= mpmath.mpf(4) * 2 ** -96 * 4, f"max error {mpmath.nstr(err, 5)}"


def pin_clement_eigenvalues(n=50):
    d, e = W.clement(n, np.float64)
    hi, lo = oracle.eigvals(d, e)
    exact = np.arange(-(n - 1), n, 2, dtype=np.float64)
    # inputs sqrt(i(n-i)) are rounded to FP64: Weyl bounds the shift by
    # max |rounding of e| * 2 <= 2 * U * n / 2
    err = np.max(np.abs(hi + lo - exact))
    return err <= 2 * U * n, f"max error {err:.3e}"


def _jacobi_mp(d, e, dps=50):
    """Cyclic Jacobi on the dense matrix in multiprecision (brute force)."""
    mpmath.mp.dps = dps
    n = len(d)
    A = mpmath.matrix(n, n)
    for i in range(n):
        A[i, i] = mpmath.mpf(float(d[i]))
        if i + 1 < n:
            A[i, i + 1] = A[i + 1, i] = mpmath.mpf(float(e[i]))
    V = mpmath.eye(n)
    for _sweep in range(30):
        off = mpmath.fsum(A[i, j] ** 2 for i in range(n) for j in range(n) if i != j)
        if off < mpmath.mpf(10) ** (-2 * dps + 10):
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                if A[p, q] == 0:
                    continue
                theta = (A[q, q] - A[p, p]) / (2 * A[p, q])
                t = mpmath.sign(theta) / (abs(theta) + mpmath.sqrt(theta ** 2 + 1)) if theta != 0 else mpmath.mpf(1)
                c = 1 / mpmath.sqrt(t ** 2 + 1)
                s = t * c
                for k in range(n):
                    akp, akq = A[k, p], A[k, q]
                    A[k, p] = c * akp - s * akq
                    A[k, q] = s * akp + c * akq
                for k in range(n):
                    apk, aqk = A[p, k], A[q, k]
                    A[p, k] = c * apk - s * aqk
                    A[q, k] = s * apk + c * aqk
                for k in range(n):
                    vkp, vkq = V[k, p], V[k, q]
                    V[k, p] = c * vkp - s * vkq
                    V[k, q] = s * vkp + c * vkq
    vals = [A[i, i] for i in range(n)]
    order = sorted(range(n), key=lambda i: vals[i])
    return [vals[i] for i in order], [[V[k, i] for k in range(n)] for i in order]


def pin_jacobi_bruteforce(seed=2, sizes=(2, 3, 5, 8, 11)):
    rng = np.random.default_rng(seed)
    worst_val = mpmath.mpf(0)
    worst_sin = 0.0
    for n in sizes:
        d = rng.uniform(-1, 1, n)
        e = rng.uniform(-1, 1, n - 1)
        vals, vecs = _jacobi_mp(d, e)
        got = _oracle_vals_mp(d, e)
        worst_val = max(worst_val, max(abs(g - v) for g, v in zip(got, vals)))
        hi, lo = oracle.eigvals(d, e)
        Z = oracle.eigvecs(d, e, hi, lo)
        for i in range(n):
            v = np.array([float(x) for x in vecs[i]])
            worst_sin = max(worst_sin, _sin_angle(v, Z[:, i]))
    ok = worst_val <= mpmath.mpf(2) ** -90 and worst_sin <= 1e-14
    return ok, f"eig {mpmath.nstr(worst_val, 4)} sin {worst_sin:.2e}"


def pin_trace_invariants(seed=3, n=64):
    rng = np.random.default_rng(seed)
    d = rng.uniform(-1, 1, n)
    e = rng.uniform(-1, 1, n - 1)
    hi, lo = oracle.eigvals(d, e)
    lam = [Fraction(h) + Fraction(l) for h, l in zip(hi, lo)]
    s1 = sum(lam) - sum(Fraction(x) for x in d)
    s2 = sum(x * x for x in lam) - (sum(Fraction(x) ** 2 for x in d) + 2 * sum(Fraction(x) ** 2 for x in e))
    tn = oracle.tnorm(d, e)
    ok = abs(float(s1)) <= n * 2.0 ** -94 * tn and abs(float(s2)) <= n * 2.0 ** -92 * tn * tn
    return ok, f"trace {float(s1):.2e} frob {float(s2):.2e}"


def pin_glued_wilkinson_multiplicity(n=336):
    """Each eigenvalue of W21+ appears once per block: with 16 blocks glued by
    1e-10, Weyl puts every eigenvalue within 2e-10 of an eigenvalue of the
    unglued block-diagonal matrix.  Count the eigenvalues near each W21+
    eigenvalue and compare with the block count (merged close pairs count
    together)."""
    d, e = W.glued_wilkinson(n)
    hi, lo = oracle.eigvals(d, e)
    lam = hi + lo
    db, eb = W.glued_wilkinson(21)
    wb = np.linalg.eigvalsh(np.diag(db) + np.diag(eb, 1) + np.diag(eb, -1))
    blocks = n // 21
    ok = True
    worst = ""
    used = np.zeros(lam.size, dtype=bool)
    for v in np.unique(np.round(wb, 9)):
        mult = int(np.sum(np.abs(wb - v) < 1e-9))
        near = np.abs(lam - v) < 3e-10 + 1e-9
        cnt = int(near.sum())
        used |= near
        if cnt != mult * blocks:
            ok = False
            worst = f"value {v}: {cnt} vs {mult * blocks}"
    ok = ok and bool(used.all())
    return ok, worst or "all multiplicities match"


def pin_prescribed_spectrum(n=400, seed=5):
    d, e, lam = W.prescribed_spectrum(n, seed)
    hi, lo = oracle.eigvals(d, e)
    err = np.max(np.abs(hi + lo - np.sort(lam)))
    # construction error of the stable reconstruction is a few units of
    # sqrt(n) * eps * ||T||
    return err <= 20 * np.sqrt(n) * U, f"max error {err:.3e}"


# --------------------------------------------------------------------------
# eigenvectors
# --------------------------------------------------------------------------
def pin_121_eigenvectors(n=64):
    d, e = W.toeplitz_121(n, np.float64)
    hi, lo = oracle.eigvals(d, e)
    Z = oracle.eigvecs(d, e, hi, lo)
    j = np.arange(1, n + 1)
    worst = 0.0
    for i in range(n):
        k = n - i  # ascending index i <-> k = n - i (0-based i)
        v = np.sqrt(2.0 / (n + 1)) * np.sin(j * k * np.pi / (n + 1))
        worst = max(worst, _sin_angle(v, Z[:, i]))
    return worst <= 1e-13, f"max sin angle {worst:.2e}"


def pin_residual_exact(seed=6, n=40):
    """Residual of the returned (FP64-rounded) pairs, evaluated exactly."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(-1, 1, n)
    e = rng.uniform(-1, 1, n - 1)
    hi, lo = oracle.eigvals(d, e)
    Z = oracle.eigvecs(d, e, hi, lo)
    worst = 0.0
    for i in range(n):
        z = [Fraction(x) for x in Z[:, i]]
        lam = Fraction(hi[i]) + Fraction(lo[i])
        r = 0
        for j in range(n):
            t = Fraction(d[j]) * z[j] - lam * z[j]
            if j > 0:
                t += Fraction(e[j - 1]) * z[j - 1]
            if j + 1 < n:
                t += Fraction(e[j]) * z[j + 1]
            r += abs(t)
        worst = max(worst, float(r))
    tn = oracle.tnorm(d, e)
    # z is rounded to FP64: residual is a few eps per component
    return worst / tn <= 4 * n * U, f"R = {worst / tn:.2e}"


def pin_repeated_eigenvalues():
    """Two identical decoupled blocks: exact double eigenvalues; the oracle must
    return an orthonormal basis of each 2-dimensional eigenspace."""
    rng = np.random.default_rng(7)
    m = 9
    db = rng.uniform(-1, 1, m)
    eb = rng.uniform(0.1, 1, m - 1)
    d = np.concatenate([db, db])
    e = np.concatenate([eb, [0.0], eb])
    hi, lo = oracle.eigvals(d, e)
    Z = oracle.eigvecs(d, e, hi, lo)
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    O = np.max(np.abs(Z.T @ Z - np.eye(2 * m)))
    R = np.max(np.abs(T @ Z - Z * (hi + lo)))
    pairs = np.max(np.abs(hi[0::2] - hi[1::2]))
    ok = O <= 1e-14 and R <= 1e-14 and pairs == 0.0
    return ok, f"O {O:.2e} R {R:.2e} pair split {pairs:.1e}"


def pin_value_range_counts(seed=8, n=120):
    rng = np.random.default_rng(seed)
    d = rng.uniform(-1, 1, n)
    e = rng.uniform(-1, 1, n - 1)
    hi, lo = oracle.eigvals(d, e)
    lam = np.sort(np.linalg.eigvalsh(np.diag(d) + np.diag(e, 1) + np.diag(e, -1)))
    gaps = np.diff(lam)
    bad = 0
    for i in range(1, n):
        mid = 0.5 * (lam[i - 1] + lam[i])
        if gaps[i - 1] > 1e-10 and oracle.count(d, e, mid) != i:
            bad += 1
    return bad == 0, f"{bad} count mismatches"


# --------------------------------------------------------------------------
# zero-pivot guards and the norm
# --------------------------------------------------------------------------
def _strict_count_exact(d, e, sigma):
    """#{lambda < sigma} in exact rationals: the inertia at sigma - delta for a
    delta far below every gap of these small integer-valued cases (Sylvester:
    the count only changes where sigma crosses an eigenvalue)."""
    for k in (300, 301, 302, 303):
        c = _exact_negcount(d, e, Fraction(sigma) - Fraction(1, 2 ** k))
        if c is not None:
            return c
    raise AssertionError("no regular point below sigma")


def pin_count_zero_pivot():
    """The Sturm count where a pivot of T - sigma I is exactly zero.  Every
    pivot decreases as sigma grows, so the count of eigenvalues strictly
    below sigma is the inertia just below sigma: an eigenvalue equal to sigma
    (a zero last pivot) is not counted, and a zero pivot before the last row
    does not change the count.  Cases with exact rational eigenvalues (n = 1;
    [[2,1],[1,2]] with eigenvalues 1 and 3; 1-2-1 of order 3 at 2; [[0,1],[1,0]]
    at 0) and random integer matrices at sigma = d_1 (first pivot zero) and at
    their integer eigenvalues found by exact count."""
    cases = [
        ([0.5], [], 0.5, 0),
        ([2.0, 2.0], [1.0], 1.0, 0),
        ([2.0, 2.0], [1.0], 3.0, 1),
        ([2.0, 2.0, 2.0], [1.0, 1.0], 2.0, 1),
        ([0.0, 0.0], [1.0], 0.0, 1),
    ]
    rng = np.random.default_rng(31)
    for _ in range(40):
        n = int(rng.integers(2, 7))
        d = [float(x) for x in rng.integers(-3, 4, n)]
        e = [float(x) for x in rng.integers(1, 3, n - 1)]
        cases.append((d, e, d[0], _strict_count_exact(d, e, d[0])))
        # integer sigmas that are eigenvalues: count jumps across sigma
        for s in range(-6, 7):
            lo = _strict_count_exact(d, e, s)
            hi = _exact_negcount(d, e, Fraction(s) + Fraction(1, 2 ** 300))
            if hi is not None and hi > lo:
                cases.append((d, e, float(s), lo))
    bad = [(d, e, s, want, oracle.count(np.array(d), np.array(e or [0.0]), s))
           for d, e, s, want in cases
           if oracle.count(np.array(d), np.array(e or [0.0]), s) != want]
    return not bad, f"{len(bad)} of {len(cases)} wrong" + (f", first {bad[0]}" if bad else "")


def pin_inverse_iteration_zero_pivot():
    """Inverse iteration at an eigenvalue that is exact, so that elimination
    of T - lambda I meets an exactly zero pivot: the guarded pivot must still
    give the exact eigenvector (finite, to FP64 accuracy)."""
    cases = [
        ([2.0, 2.0], [1.0], [1.0, 3.0], [[1, -1], [1, 1]]),
        ([2.0, 2.0, 2.0], [1.0, 1.0], [2.0], [[1, 0, -1]]),
        ([0.0, 0.0], [1.0], [-1.0, 1.0], [[1, -1], [1, 1]]),
        ([1.0, 1.0, 1.0], [0.0, 0.0], [1.0, 1.0, 1.0], None),
    ]
    worst = 0.0
    for d, e, lam, vecs in cases:
        d, e, lam = np.array(d), np.array(e), np.array(lam)
        Z = oracle.eigvecs(d, e, lam, np.zeros_like(lam))
        if not np.all(np.isfinite(Z)):
            return False, f"non-finite vector for d={d.tolist()} lambda={lam.tolist()}"
        if vecs is None:  # identity: any orthonormal basis of the whole space
            worst = max(worst, float(np.max(np.abs(Z.T @ Z - np.eye(d.size)))))
            continue
        for k, v in enumerate(vecs):
            worst = max(worst, _sin_angle(np.array(v, dtype=np.float64), Z[:, k]))
    return worst <= 1e-15, f"worst {worst:.2e}"


def pin_tnorm(seed=32):
    """||T||_1 = max_i (|e_{i-1}| + |d_i| + |e_i|), the norm of the gates,
    against the exact rational row sums (the oracle adds in FP64: two
    roundings)."""
    rng = np.random.default_rng(seed)
    worst = 0.0
    for n in (1, 2, 3, 7, 100):
        for _ in range(5):
            d = rng.uniform(-1, 1, n) * 2.0 ** rng.integers(-3, 4, n)
            e = rng.uniform(-1, 1, max(n - 1, 0)) * 2.0 ** rng.integers(-3, 4, max(n - 1, 0))
            rows = []
            for i in range(n):
                r = abs(Fraction(d[i]))
                if i > 0:
                    r += abs(Fraction(e[i - 1]))
                if i + 1 < n:
                    r += abs(Fraction(e[i]))
                rows.append(r)
            exact = max(rows)
            got = oracle.tnorm(d, e if n > 1 else np.zeros(1))
            worst = max(worst, abs(float((Fraction(got) - exact) / exact)))
    return worst <= 2 * U, f"worst relative error {worst:.2e}"


ALL_PINS = [
    pin_dd_ops,
    pin_sturm_inertia,
    pin_121_eigenvalues,
    pin_clement_eigenvalues,
    pin_jacobi_bruteforce,
    pin_trace_invariants,
    pin_glued_wilkinson_multiplicity,
    pin_prescribed_spectrum,
    pin_121_eigenvectors,
    pin_residual_exact,
    pin_repeated_eigenvalues,
    pin_value_range_counts,
    pin_count_zero_pivot,
    pin_inverse_iteration_zero_pivot,
    pin_tnorm,
]
