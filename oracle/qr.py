"""Householder-QR oracle: the comparator of Sec. III.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. III solves the same least-squares problem without normal equations:
with the Vandermonde matrix V (V_ik = x_i^k), V p = Y in the least-squares
sense; factor V = QR by Householder reflections and solve R p = Q^T Y.
Reading: the printed algebra ("Holder Reflections", Q Q^T = I, p = (Q^T Y)\\R)
is taken as the standard thin QR: Q^T Q = I and p = R^-1 (Q^T Y).

For large n the tall-skinny tree form is used: factor row blocks of the
augmented matrix [V | Y] separately, stack their R factors and factor again.
The stacked factorisation spans the same column space, so the final R (and
its last column, Q^T Y) equals that of one factorisation of all rows up to
the signs of the rows, which cancel in R p = Q^T Y.
"""
from __future__ import annotations

import numpy as np


def householder_r(M: np.ndarray) -> np.ndarray:
    """Upper-triangular R of M = QR (k = ncols rows) by Householder reflections."""
    M = np.array(M, dtype=np.float64, copy=True)
    n, p = M.shape
    for k in range(min(n, p)):
        col = M[k:, k]
        norm = np.sqrt(np.dot(col, col))
        if norm == 0.0:
            continue
        alpha = -norm if col[0] >= 0.0 else norm
        v = col.copy()
        v[0] -= alpha
        vv = np.dot(v, v)
        if vv == 0.0:
            continue
        # H = I - 2 v v^T / (v^T v) applied to the trailing columns
        M[k:, k:] -= np.outer(v, (2.0 / vv) * (v @ M[k:, k:]))
        M[k + 1:, k] = 0.0
    return np.triu(M[:p, :]) if n >= p else np.triu(M)


def householder_qr(V: np.ndarray):
    """Explicit thin Q and R (for tests of the factorisation itself)."""
    V = np.asarray(V, dtype=np.float64)
    n, p = V.shape
    aug = np.hstack([V, np.eye(n)])
    R_full = householder_r(aug)          # rows: [R | Q^T]
    R = R_full[:p, :p]
    Qt = R_full[:p, p:]
    return Qt.T, R


def vandermonde(x, m: int, center: float = 0.0, scale: float = 1.0) -> np.ndarray:
    t = (np.asarray(x, dtype=np.float64) - center) / scale
    V = np.empty((t.shape[0], m + 1))
    V[:, 0] = 1.0
    for k in range(1, m + 1):
        V[:, k] = V[:, k - 1] * t
    return V


def back_substitute(R: np.ndarray, z: np.ndarray) -> np.ndarray:
    p = R.shape[0]
    out = np.zeros(p)
    for i in range(p - 1, -1, -1):
        out[i] = (z[i] - np.dot(R[i, i + 1:], out[i + 1:])) / R[i, i]
    return out


def tsqr_r(x, y, m: int, center: float = 0.0, scale: float = 1.0, block: int = 1 << 20) -> np.ndarray:
    """R factor of [V | y] (m+2 columns) by a one-level tall-skinny tree."""
    n = len(x)
    rs = []
    for s in range(0, n, block):
        e = min(n, s + block)
        V = vandermonde(x[s:e], m, center, scale)
        aug = np.hstack([V, np.asarray(y[s:e], dtype=np.float64)[:, None]])
        rs.append(householder_r(aug))
    stacked = np.vstack(rs)
    return householder_r(stacked) if len(rs) > 1 else rs[0]


def lstsq_qr(x, y, m: int, center: float = 0.0, scale: float = 1.0, block: int = 1 << 20):
    """t-basis coefficients b of the least-squares fit by Householder QR."""
    Raug = tsqr_r(x, y, m, center, scale, block)
    R = Raug[: m + 1, : m + 1]
    z = Raug[: m + 1, m + 1]
    return back_substitute(R, z)
