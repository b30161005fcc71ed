"""Float64 oracle: the paper's normal-equation route written out plainly.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Steps, in the paper's order (Sec. II):

1. optional change of variable t_i = (x_i - c)/s.  The least-squares fit is
   invariant under an affine map of x (polynomials of degree <= m map onto
   themselves), so only rounding changes; ``unscale`` maps back.
2. power sums S_p = sum_i t_i^p (p = 0..2m) and T_j = sum_i t_i^j y_i
   (j = 0..m) -- the sums that appear in the expanded normal equations
   (Sec. II).  Each sum is correctly rounded (``math.fsum``); the terms t^p are
   formed by repeated multiplication in float64.
3. the matrix A_jk = S_(j+k) and vector B_j = T_j of the system AX = B.
   Reading: the printed A has A_00 = 1 and a last row of S_m, S_(m+2), ...;
   the expanded equations fix A_00 = S_0 = n and row m = S_m..S_2m.
4. Gaussian elimination (end of Sec. II).  Reading: with partial pivoting,
   the first row of largest magnitude is the pivot; the system is declared
   singular when a pivot's magnitude is at most 2^-40 times the largest
   entry of A (the paper says nothing about singular systems).
5. back to the x-basis: a_k = sum_{j>=k} b_j C(j,k) (-c)^(j-k) s^(-j).
"""
from __future__ import annotations

import math

import numpy as np

OK, SINGULAR, NONFINITE = "ok", "singular", "nonfinite"
SINGULAR_REL = 2.0 ** -40


def change_of_variable(x, center: float = 0.0, scale: float = 1.0) -> np.ndarray:
    """t = (x - c)/s in float64."""
    x = np.asarray(x, dtype=np.float64)
    return (x - center) / scale


def power_sums(x, y, m: int, center: float = 0.0, scale: float = 1.0):
    """S_0..S_2m and T_0..T_m of t = (x - c)/s, each sum correctly rounded."""
    t = change_of_variable(x, center, scale)
    y = np.asarray(y, dtype=np.float64)
    S = [float(t.shape[0])]
    T = [math.fsum(y.tolist())]
    p = np.ones_like(t)
    for k in range(1, 2 * m + 1):
        p = p * t
        S.append(math.fsum(p.tolist()))
        if k <= m:
            T.append(math.fsum((p * y).tolist()))
    return S, T


def assemble(S, T, m: int):
    """Hankel A_jk = S_(j+k) and B_j = T_j of the normal equations."""
    A = [[S[j + k] for k in range(m + 1)] for j in range(m + 1)]
    B = [T[j] for j in range(m + 1)]
    return A, B


def gepp(A, B, singular_rel: float = SINGULAR_REL):
    """Solve A X = B by Gaussian elimination with partial pivoting.

    Returns (X, status).  Pivot: the first row of largest |entry| in the
    current column.  Singular when |pivot| <= singular_rel * max|A|.
    """
    n = len(A)
    if not all(math.isfinite(v) for row in A for v in row) or not all(math.isfinite(v) for v in B):
        return [math.nan] * n, NONFINITE
    M = [list(map(float, A[i])) + [float(B[i])] for i in range(n)]
    amax = max(abs(v) for row in A for v in row)
    for k in range(n):
        p = max(range(k, n), key=lambda r: abs(M[r][k]))   # max() keeps the first maximum
        if not abs(M[p][k]) > singular_rel * amax:
            return [math.nan] * n, SINGULAR
        if p != k:
            M[k], M[p] = M[p], M[k]
        for r in range(k + 1, n):
            l = M[r][k] / M[k][k]
            for c in range(k, n + 1):
                M[r][c] -= l * M[k][c]
    X = [0.0] * n
    for i in range(n - 1, -1, -1):
        acc = M[i][n]
        for c in range(i + 1, n):
            acc -= M[i][c] * X[c]
        X[i] = acc / M[i][i]
    if not all(math.isfinite(v) for v in X):
        return [math.nan] * n, NONFINITE
    return X, OK


def gepp_many(A, B, singular_rel: float = SINGULAR_REL):
    """``gepp`` applied to K independent systems at once (A: K x n x n, B: K x n).

    Each system goes through the same steps as ``gepp`` -- first row of
    largest |entry| as pivot, elimination of the rows below, back
    substitution -- so every system gets the bits ``gepp`` gives it; only the
    loop over systems is vectorised.  Returns (X [K, n], ok [K]); rows of X
    for singular or non-finite systems are NaN.
    """
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    K, n = B.shape
    M = np.concatenate([A, B[:, :, None]], axis=2).copy()
    finite = np.isfinite(M).all(axis=(1, 2))
    amax = np.where(finite, np.abs(np.where(np.isfinite(A), A, 0.0)).max(axis=(1, 2)), 0.0)
    ok = finite.copy()
    rows = np.arange(K)
    for k in range(n):
        p = k + np.argmax(np.abs(M[:, k:, k]), axis=1)      # argmax keeps the first maximum
        ok &= np.abs(M[rows, p, k]) > singular_rel * amax
        pk = M[rows, p, :].copy()
        M[rows, p, :] = M[:, k, :]
        M[:, k, :] = pk
        with np.errstate(divide="ignore", invalid="ignore"):
            for r in range(k + 1, n):
                l = M[:, r, k] / M[:, k, k]
                for c in range(k, n + 1):
                    M[:, r, c] -= l * M[:, k, c]
    X = np.zeros((K, n))
    with np.errstate(divide="ignore", invalid="ignore"):
        for i in range(n - 1, -1, -1):
            acc = M[:, i, n].copy()
            for c in range(i + 1, n):
                acc -= M[:, i, c] * X[:, c]
            X[:, i] = acc / M[:, i, i]
    ok &= np.isfinite(X).all(axis=1)
    X[~ok] = np.nan
    return X, ok


def unscale(b, center: float = 0.0, scale: float = 1.0):
    """t-basis coefficients b (t = (x-c)/s) -> x-basis a, both ascending."""
    m = len(b) - 1
    a = [0.0] * (m + 1)
    for k in range(m + 1):
        terms = [b[j] * math.comb(j, k) * (-center) ** (j - k) * scale ** (-j) for j in range(k, m + 1)]
        a[k] = math.fsum(terms)
    return a


def fit(x, y, m: int, center: float = 0.0, scale: float = 1.0) -> dict:
    """The whole route: returns x-basis ``a``, t-basis ``b``, ``S``, ``T`` and ``status``."""
    S, T = power_sums(x, y, m, center, scale)
    A, B = assemble(S, T, m)
    b, status = gepp(A, B)
    a = unscale(b, center, scale) if status == OK else [math.nan] * (m + 1)
    return {"a": np.array(a), "b": np.array(b), "S": np.array(S), "T": np.array(T),
            "status": status, "center": center, "scale": scale}


def fit_batched(x, y, offsets, degrees, centers=None, scales=None) -> list:
    """Independent fits over CSR segments offsets[f]:offsets[f+1]."""
    out = []
    for f in range(len(degrees)):
        lo, hi = int(offsets[f]), int(offsets[f + 1])
        m = int(degrees[f])
        c = 0.0 if centers is None else float(centers[f])
        s = 1.0 if scales is None else float(scales[f])
        if hi - lo < m + 1:
            out.append({"a": np.full(m + 1, np.nan), "b": np.full(m + 1, np.nan), "status": SINGULAR})
            continue
        out.append(fit(x[lo:hi], y[lo:hi], m, c, s))
    return out


def polyval(a, x) -> np.ndarray:
    """f(x) = sum_k a_k x^k (ascending), float64, Horner."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    for c in list(a)[::-1]:
        out = out * x + c
    return out


def sse(x, y, a) -> float:
    """Pi = sum_i [y_i - f(x_i)]^2, the objective of Sec. II."""
    r = np.asarray(y, dtype=np.float64) - polyval(a, x)
    return math.fsum((r * r).tolist())
