"""Accuracy measures and gates shared by the GPU tests.

Gates (spec numbers; eps = unit roundoff of the I/O format, 2^-24 or
2^-53; norms are 1-norms as in the paper's eq. (1)):
    |lambda - lambda_oracle|          <= 4 n eps ||T||_1
    ||T z - lambda z||_1 / ||T||_1    <= 10 n eps
    max |Z^T Z - I|                   <= 10 n eps
Eigenvectors are compared with the oracle through subspace angles per group of
close eigenvalues (Davis-Kahan / the Gap Theorem of the paper's Sec. 2), never
bitwise.
"""
from __future__ import annotations

import numpy as np

EPS = {np.dtype(np.float32): 2.0 ** -24, np.dtype(np.float64): 2.0 ** -53}


def eps_of(dtype) -> float:
    return EPS[np.dtype(dtype)]


def tnorm(d, e) -> float:
    d = np.asarray(d, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)
    n = d.size
    if n == 0:
        return 0.0
    row = np.abs(d).copy()
    if n > 1:
        row[:-1] += np.abs(e[: n - 1])
        row[1:] += np.abs(e[: n - 1])
    return float(row.max())


def residual(d, e, W, Z) -> float:
    """max_i ||T z_i - w_i z_i||_1 / ||T||_1 in FP64."""
    d = np.asarray(d, dtype=np.float64)
    e = np.asarray(e, dtype=np.float64)[: max(d.size - 1, 0)]
    W = np.asarray(W, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    if W.size == 0:
        return 0.0
    TZ = d[:, None] * Z - W[None, :] * Z
    if d.size > 1:
        TZ[:-1] += e[:, None] * Z[1:]
        TZ[1:] += e[:, None] * Z[:-1]
    tn = tnorm(d, e)
    return float(np.abs(TZ).sum(0).max() / (tn if tn > 0 else 1.0))


def orthogonality(Z) -> float:
    Z = np.asarray(Z, dtype=np.float64)
    if Z.shape[1] == 0:
        return 0.0
    G = Z.T @ Z
    return float(np.abs(G - np.eye(G.shape[0])).max())


def groups_by_gap(w, tol):
    """Maximal runs of consecutive eigenvalues closer than tol."""
    w = np.asarray(w)
    if w.size == 0:
        return []
    cuts = np.nonzero(np.diff(w) > tol)[0] + 1
    bounds = np.concatenate([[0], cuts, [w.size]])
    return [(int(bounds[i]), int(bounds[i + 1])) for i in range(len(bounds) - 1)]


def subspace_sines(w_ref, Z_ref, Z, R, tn, group_tol, O=None):
    """For each group G of reference eigenvalues, sin of the largest principal
    angle between span(Z_ref[:, G]) and span(Z[:, G]), with the bound
    sqrt(|G|) * R * ||T||_1 / delta_G + orth of the theory (delta_G = gap of
    the group to the rest of the reference spectrum).  O = max|Z^T Z - I| if
    already known (it is computed otherwise).  Returns (worst ratio
    sin / bound, worst sin)."""
    w_ref = np.asarray(w_ref, dtype=np.float64)
    worst_ratio, worst = 0.0, 0.0
    if O is None:
        O = orthogonality(Z)
    for a, b in groups_by_gap(w_ref, group_tol):
        left = w_ref[a] - w_ref[a - 1] if a > 0 else np.inf
        right = w_ref[b] - w_ref[b - 1] if b < w_ref.size else np.inf
        delta = min(left, right)
        Qr, _ = np.linalg.qr(Z_ref[:, a:b])
        Qg, _ = np.linalg.qr(Z[:, a:b])
        M = Qg - Qr @ (Qr.T @ Qg)
        s = float(np.linalg.norm(M, 2)) if M.size else 0.0
        bound = np.sqrt(b - a) * R * tn / delta + 4 * O + 1e-300 if np.isfinite(delta) else np.inf
        worst = max(worst, s)
        if np.isfinite(bound):
            worst_ratio = max(worst_ratio, s / bound)
    return worst_ratio, worst


def residual_ld(d, e, w, z):
    """||T z - w z||_1 of one vector evaluated in x87 extended precision
    (64-bit significand): products of binary64 numbers carry a relative error
    of 2^-64 instead of 2^-53, so the evaluation error (bounded by the second
    return value) stays far below binary64 residuals."""
    ld = np.longdouble
    d = np.asarray(d, dtype=ld)
    e = np.asarray(e, dtype=ld)[: max(d.size - 1, 0)]
    z = np.asarray(z, dtype=ld)
    r = (d - ld(w)) * z
    if d.size > 1:
        r[:-1] += e * z[1:]
        r[1:] += e * z[:-1]
    u = float(np.finfo(ld).eps) / 2
    tn = tnorm(d.astype(np.float64), e.astype(np.float64))
    bound = 6 * u * (tn + abs(float(w))) * float(np.abs(z).sum())
    return float(np.abs(r).sum()), bound


def gap_theorem_sine(d, e, w, z, z_ref, lam_others):
    """Angle between a computed eigenvector z (eigenvalue approximation w) and
    the reference vector z_ref, with the bound of the Gap Theorem (the
    paper's Sec. 2): sin angle <= ||T zn - w zn||_2 / min_j |lambda_j - w| for
    the unit vector zn = z / ||z|| and the other eigenvalues lambda_j (only
    the nearest ones matter).  The residual is evaluated in extended
    precision and its evaluation error added; ||.||_2 <= ||.||_1.  Returns
    (sin, bound)."""
    z = np.asarray(z, dtype=np.float64)
    zr = np.asarray(z_ref, dtype=np.float64)
    zr = zr / np.linalg.norm(zr)
    nz = float(np.linalg.norm(z))
    zn = z / nz
    c = float(zr @ zn)
    s = float(np.linalg.norm(zn - c * zr))
    r, rb = residual_ld(d, e, w, zn)
    gap = min(abs(float(l) - float(w)) for l in lam_others)
    return s, (r + rb) / gap


def alone_vs_mix(w_a, Z_a, w_m, Z_m, R, O, tn, eps):
    """Compare the results of one problem solved alone (w_a, Z_a) and inside a
    batch or a served mix (w_m, Z_m): eigenvalues within 4 n eps ||T||_1;
    eigenvectors by |z_a^T z_m| >= 1 - 10 n eps for every eigenvalue whose
    gap delta to its neighbours pins its vector that tightly (both vectors
    lie within R ||T||_1 / delta of the true one by the Gap Theorem, and
    (2 R ||T||_1 / delta)^2 <= 5 n eps), and by the largest principal angle
    within 2 sqrt(|G|) R ||T||_1 / delta_G + 4 O (Davis-Kahan) for the groups
    of closer eigenvalues.  R and O are the larger residual and orthogonality
    of the two results.  Returns (worst 1 - |cos| of the singletons, worst
    sin / bound of the groups, number of groups)."""
    w_a = np.asarray(w_a, dtype=np.float64)
    w_m = np.asarray(w_m, dtype=np.float64)
    n = Z_a.shape[0]
    assert w_a.shape == w_m.shape
    if w_a.size == 0:
        return 0.0, 0.0, 0
    assert np.max(np.abs(w_a - w_m)) <= 4 * n * eps * tn
    Z_a = np.asarray(Z_a, dtype=np.float64)
    Z_m = np.asarray(Z_m, dtype=np.float64)
    tol = 2.0 * R * tn / np.sqrt(5.0 * n * eps)
    worst_c, worst_ratio, ngroups = 0.0, 0.0, 0
    for a, b in groups_by_gap(w_a, tol):
        if b - a == 1:
            c = abs(float(Z_a[:, a] @ Z_m[:, a]))
            worst_c = max(worst_c, 1.0 - c)
            assert 1.0 - c <= 10 * n * eps, (a, c)
            continue
        ngroups += 1
        left = w_a[a] - w_a[a - 1] if a > 0 else np.inf
        right = w_a[b] - w_a[b - 1] if b < w_a.size else np.inf
        delta = min(left, right)
        Qa, _ = np.linalg.qr(Z_a[:, a:b])
        Qm, _ = np.linalg.qr(Z_m[:, a:b])
        s = float(np.linalg.norm(Qm - Qa @ (Qa.T @ Qm), 2))
        if np.isfinite(delta):
            bound = 2.0 * np.sqrt(b - a) * R * tn / delta + 4 * O
            worst_ratio = max(worst_ratio, s / bound)
            assert s <= bound, (a, b, s, bound)
    return worst_c, worst_ratio, ngroups
