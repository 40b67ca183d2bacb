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


def subspace_sines(w_ref, Z_ref, Z, R, tn, group_tol):
    """For each group G of reference eigenvalues, sin of the largest principal
    angle between span(Z_ref[:, G]) and span(Z[:, G]), with the bound
    sqrt(|G|) * R * ||T||_1 / delta_G + orth of the theory (delta_G = gap of
    the group to the rest of the reference spectrum).  Returns (worst ratio
    sin / bound, worst sin)."""
    w_ref = np.asarray(w_ref, dtype=np.float64)
    worst_ratio, worst = 0.0, 0.0
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
