"""Exact rational oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``fit_exact`` follows the route of Sec. II in ``fractions.Fraction``: exact
  power sums, the Hankel normal matrix A_jk = S_(j+k) (A_00 = S_0 = n) with
  right side B_j = T_j, Gaussian elimination with partial pivoting (in exact
  arithmetic any non-zero pivot gives the same answer; the largest-magnitude
  rule is kept for symmetry with the float routes), and the exact change back
  to the x-basis.  Singular means an exactly zero pivot.
* ``normal_residual`` returns V^T r exactly, which is zero at the minimiser
  (the first-order conditions of Sec. II: dPi/da_j = -2 sum_i x_i^j r_i).
* ``periodic_power_sums`` gives the exact power sums of points lo..hi-1 of
  the periodic pattern x_i = (2 (i mod 1024) - 1023)/1024,
  y_i = (i mod 1021)/1024 (the inputs of the 64-bit indexing checks) from
  their closed form: a sum over i collapses to counts of each residue, and
  the joint residues of (x, y) repeat every 1024 * 1021 points.
* ``grid_power_sums`` gives exact power sums for large float inputs whose
  shifted abscissae u_i = (x_i - c)/q are integers (a float32 x in
  [1000, 1001) lies on the 2^-14 grid): the sums over points collapse to sums
  over distinct u values, with the y values of each u summed exactly.
"""
from __future__ import annotations

from fractions import Fraction
from math import comb

import numpy as np


def frac(v) -> Fraction:
    """Exact value: decimal strings as written, floats as stored."""
    if isinstance(v, Fraction):
        return v
    if isinstance(v, str):
        return Fraction(v)
    return Fraction(float(v))


def power_sums_exact(xs, ys, m: int, center=0, scale=1):
    c, s = frac(center), frac(scale)
    ts = [(frac(x) - c) / s for x in xs]
    yv = [frac(y) for y in ys]
    S = [sum((t ** p for t in ts), Fraction(0)) for p in range(2 * m + 1)]
    T = [sum((t ** j * y for t, y in zip(ts, yv)), Fraction(0)) for j in range(m + 1)]
    return S, T


def gepp_exact(A, B):
    """Exact Gaussian elimination with partial pivoting; returns (X, singular?)."""
    n = len(A)
    M = [[Fraction(v) for v in A[i]] + [Fraction(B[i])] for i in range(n)]
    for k in range(n):
        p = max(range(k, n), key=lambda r: abs(M[r][k]))
        if M[p][k] == 0:
            return None, True
        M[k], M[p] = M[p], M[k]
        for r in range(k + 1, n):
            l = M[r][k] / M[k][k]
            for c in range(k, n + 1):
                M[r][c] -= l * M[k][c]
    X = [Fraction(0)] * n
    for i in range(n - 1, -1, -1):
        acc = M[i][n]
        for c in range(i + 1, n):
            acc -= M[i][c] * X[c]
        X[i] = acc / M[i][i]
    return X, False


def unscale_exact(b, center=0, scale=1):
    """a_k = sum_{j>=k} b_j C(j,k) (-c)^(j-k) s^(-j), exactly."""
    c, s = frac(center), frac(scale)
    m = len(b) - 1
    return [sum((b[j] * comb(j, k) * (-c) ** (j - k) / s ** j for j in range(k, m + 1)), Fraction(0))
            for k in range(m + 1)]


def solve_from_sums(S, T, m: int):
    A = [[S[j + k] for k in range(m + 1)] for j in range(m + 1)]
    return gepp_exact(A, T[: m + 1])


def fit_exact(xs, ys, m: int, center=0, scale=1):
    """Exact minimiser; returns (a, b) as Fractions, or (None, None) if singular."""
    S, T = power_sums_exact(xs, ys, m, center, scale)
    b, singular = solve_from_sums(S, T, m)
    if singular:
        return None, None
    return unscale_exact(b, center, scale), b


def polyval_exact(a, x):
    acc = Fraction(0)
    for c in reversed(a):
        acc = acc * frac(x) + c
    return acc


def normal_residual(xs, ys, a):
    """[sum_i x_i^k (y_i - f(x_i))]_k, exactly."""
    m = len(a) - 1
    r = [frac(y) - polyval_exact(a, x) for x, y in zip(xs, ys)]
    return [sum((frac(x) ** k * ri for x, ri in zip(xs, r)), Fraction(0)) for k in range(m + 1)]


def sse_exact(xs, ys, a) -> Fraction:
    return sum(((frac(y) - polyval_exact(a, x)) ** 2 for x, y in zip(xs, ys)), Fraction(0))


def _exact_bin_sums_f32(bin_index: np.ndarray, nbins: int, y32: np.ndarray):
    """Exact sum of float32 y over each bin, as Fractions.

    y = mant * 2^e with mant in [0.5, 1); mant * 2^24 is an integer of at most
    24 bits for any float32 (subnormals included).  Integers of that size sum
    exactly in float64 as long as the total stays below 2^53, which holds for
    fewer than 2^29 points, so a weighted bincount per (bin, exponent) is exact.
    """
    assert y32.dtype == np.float32
    assert y32.shape[0] < (1 << 29)
    mant, ex = np.frexp(y32.astype(np.float64))
    m24 = mant * float(1 << 24)
    emin, emax = int(ex.min()), int(ex.max())
    ne = emax - emin + 1
    key = bin_index.astype(np.int64) * ne + (ex - emin)
    sums = np.bincount(key, weights=m24, minlength=nbins * ne)
    out = [Fraction(0)] * nbins
    nz = np.nonzero(sums)[0]
    for k in nz.tolist():
        bi, ei = divmod(k, ne)
        iv = int(sums[k])
        assert float(iv) == sums[k]
        e = ei + emin - 24
        out[bi] += Fraction(iv) * (Fraction(2) ** e)
    return out


def grid_power_sums(x, y, m: int, center, scale, quantum):
    """Exact S_p, T_j of t = (x - c)/s for x on a grid: (x - c)/quantum integral.

    Checks exactness of the grid for every distinct x and returns Fractions.
    ``y`` must be float32 (its values are summed exactly per grid point).
    """
    c, s, q = frac(center), frac(scale), frac(quantum)
    xv = np.asarray(x)
    uniq, inv = np.unique(xv, return_inverse=True)
    us = []
    for xu in uniq.tolist():
        u = (frac(xu) - c) / q
        if u.denominator != 1:
            raise ValueError(f"x = {xu!r} is not on the grid c + k*q")
        us.append(int(u))
    counts = np.bincount(inv, minlength=len(uniq))
    ybin = _exact_bin_sums_f32(inv, len(uniq), np.asarray(y))
    ratio = q / s
    S, T = [], []
    for p in range(2 * m + 1):
        S.append(sum((int(cnt) * u ** p for cnt, u in zip(counts.tolist(), us)), 0) * ratio ** p)
    for j in range(m + 1):
        T.append(sum((Fraction(u) ** j * yb for u, yb in zip(us, ybin)), Fraction(0)) * ratio ** j)
    return [Fraction(v) for v in S], T


def fit_exact_grid(x, y, m: int, center, scale, quantum):
    """Exact minimiser for gridded large inputs: (a, b) as Fractions."""
    S, T = grid_power_sums(x, y, m, center, scale, quantum)
    b, singular = solve_from_sums(S, T, m)
    if singular:
        return None, None
    return unscale_exact(b, center, scale), b


# --- the periodic pattern --------------------------------------------------------
def _residue_counts(lo: int, hi: int, p: int) -> list:
    """How many i in [lo, hi) have i mod p == r, for r = 0..p-1."""
    def upto(n):   # counts over [0, n)
        q, r = divmod(n, p)
        return [q + (1 if k < r else 0) for k in range(p)]
    a, b = upto(hi), upto(lo)
    return [u - v for u, v in zip(a, b)]


def periodic_power_sums(lo: int, hi: int, m: int, px: int = 1024, py: int = 1021):
    """Exact S_0..S_2m and T_0..T_m (Sec. II sums, c = 0, s = 1) of points
    lo..hi-1 with x_i = (2 (i mod px) - (px - 1))/px and y_i = (i mod py)/1024."""
    if m > 3:
        raise ValueError("the period sums below stay within int64 up to m = 3")
    cx = _residue_counts(lo, hi, px)
    num = [2 * a - (px - 1) for a in range(px)]          # x = num / px
    S = [Fraction(sum(c * v ** k for c, v in zip(cx, num)), px ** k) for k in range(2 * m + 1)]
    # T_j = sum_i (i mod py) num(i mod px)^j / (1024 px^j): one joint period of
    # P = px py points, then the remainder, as exact integers
    P = px * py
    i = np.arange(P, dtype=np.int64)
    a = i % py
    b = 2 * (i % px) - (px - 1)
    T = []
    for j in range(m + 1):
        terms = a * b ** j                                 # |terms| <= 1020 * 1023^3 < 2^41
        pref = np.concatenate([[0], np.cumsum(terms)])     # |pref| < 2^41 * 2^20 = 2^61
        full = int(pref[-1])

        def upto(n):
            q, r = divmod(n, P)
            return q * full + int(pref[r])
        T.append(Fraction(upto(hi) - upto(lo), 1024 * px ** j))
    return S, T

