"""Chebyshev-basis oracle for higher-degree fits.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. V of the paper leaves higher-order polynomials as further work.  The
least-squares problem is the same (minimise sum_i [y_i - f(x_i)]^2 over
polynomials f of degree <= m, Sec. II); only the basis in which f is written
changes: f(x) = sum_j c_j T_j(t) with t = (x - c0)/s and the Chebyshev
polynomials T_0 = 1, T_1 = t, T_(k+1) = 2 t T_k - T_(k-1).  With
V_ij = T_j(t_i) the normal equations read G c = V^T y, G = V^T V.

* ``fit_cheb``: G and V^T y formed entry by entry as sums of products
  (correctly rounded with ``math.fsum``), then ``fp64.gepp``.  This is the
  plain definition written out, without the product identity the GPU path
  uses to need only 2m+1 sums.
* ``fit_cheb_exact``: the same in exact rational arithmetic.
* ``cheb_to_monomial``: c -> b with sum_j c_j T_j(t) = sum_k b_k t^k, from the
  recurrence applied to coefficient vectors.
* ``cheb_range``: the (c, s) that put the data's extent on [-1, 1].
* ``cheb_gradients``: dL/dx and dL/dy of a scalar loss L(c) of the Chebyshev
  coefficients, for a given (c, s).  With lambda = G^-1 dL/dc (G symmetric),
  dL/dD = lambda and dL/dG = -lambda c^T; since D_j = sum_i y_i T_j(t_i) and
  G_jk = sum_i T_j(t_i) T_k(t_i),
    dL/dy_i = q(t_i),  dL/dt_i = q'(t_i) (y_i - f(t_i)) - q(t_i) f'(t_i),
  with f = sum_j c_j T_j, q = sum_j lambda_j T_j, and dL/dx_i = dL/dt_i / s.
  T_j' = j U_(j-1) with the second-kind U_0 = 1, U_1 = 2t,
  U_(k+1) = 2t U_k - U_(k-1).
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from . import exact, fp64


def cheb_range(x) -> tuple[float, float]:
    """(c, s) that map the extent [lo, hi] of the finite x onto [-1, 1]:
    c = hi/2 + lo/2, s = hi/2 - lo/2 (s = 1 when the extent is a point, and
    (0, 1) when no x is finite).  The T_k are orthogonal on [-1, 1]; the
    Chebyshev route takes this range when none is given."""
    v = np.asarray(x, dtype=np.float64)
    v = v[np.isfinite(v)]
    if v.size == 0:
        return 0.0, 1.0
    lo, hi = float(v.min()), float(v.max())
    half = 0.5 * hi - 0.5 * lo
    return 0.5 * hi + 0.5 * lo, (half if half > 0.0 else 1.0)


def cheb_values(t, m: int) -> list:
    """[T_0(t), .., T_m(t)] for an array t (float64)."""
    t = np.asarray(t, dtype=np.float64)
    T = [np.ones_like(t)]
    if m >= 1:
        T.append(t.copy())
    for k in range(1, m):
        T.append(2.0 * t * T[k] - T[k - 1])
    return T


def fit_cheb(x, y, m: int, center: float = 0.0, scale: float = 1.0) -> dict:
    """Chebyshev coefficients c of the least-squares fit, and its monomial
    t-basis b and x-basis a (float64)."""
    t = fp64.change_of_variable(x, center, scale)
    yv = np.asarray(y, dtype=np.float64)
    T = cheb_values(t, m)
    G = [[math.fsum((T[j] * T[k]).tolist()) for k in range(m + 1)] for j in range(m + 1)]
    r = [math.fsum((T[j] * yv).tolist()) for j in range(m + 1)]
    c, status = fp64.gepp(G, r)
    if status != fp64.OK:
        return {"c": np.full(m + 1, np.nan), "status": status}
    b = cheb_to_monomial(c)
    a = fp64.unscale(b, center, scale)
    return {"c": np.array(c), "b": np.array(b), "a": np.array(a), "status": status}


def cheb_to_monomial(c):
    """Coefficients b_k of sum_j c_j T_j(t) in powers of t (works for floats or Fractions)."""
    m = len(c) - 1
    zero = c[0] * 0
    Tprev = [zero] * (m + 1)
    Tprev[0] = zero + 1          # T_0
    Tcur = [zero] * (m + 1)
    if m >= 1:
        Tcur[1] = zero + 1       # T_1
    b = [c[0] * Tprev[k] for k in range(m + 1)]
    if m >= 1:
        b = [b[k] + c[1] * Tcur[k] for k in range(m + 1)]
    for j in range(1, m):
        Tnext = [(2 * Tcur[k - 1] if k >= 1 else zero) - Tprev[k] for k in range(m + 1)]
        b = [b[k] + c[j + 1] * Tnext[k] for k in range(m + 1)]
        Tprev, Tcur = Tcur, Tnext
    return b


def fit_cheb_exact(xs, ys, m: int, center=0, scale=1):
    """Exact Chebyshev coefficients (Fractions) of the least-squares fit."""
    c0, s = exact.frac(center), exact.frac(scale)
    ts = [(exact.frac(x) - c0) / s for x in xs]
    yv = [exact.frac(y) for y in ys]
    cols = []
    for t in ts:
        row = [Fraction(1)]
        if m >= 1:
            row.append(t)
        for k in range(1, m):
            row.append(2 * t * row[k] - row[k - 1])
        cols.append(row)
    G = [[sum((row[j] * row[k] for row in cols), Fraction(0)) for k in range(m + 1)] for j in range(m + 1)]
    r = [sum((row[j] * yy for row, yy in zip(cols, yv)), Fraction(0)) for j in range(m + 1)]
    c, singular = exact.gepp_exact(G, r)
    return None if singular else c


def cheb_derivative_values(t, m: int) -> list:
    """[T_0'(t), .., T_m'(t)] for an array t (float64), T_j' = j U_(j-1)."""
    t = np.asarray(t, dtype=np.float64)
    U = [np.ones_like(t), 2.0 * t]
    for k in range(1, m):
        U.append(2.0 * t * U[k] - U[k - 1])
    return [np.zeros_like(t)] + [j * U[j - 1] for j in range(1, m + 1)]


def cheb_gradients(x, y, m: int, gbar, center: float = 0.0, scale: float = 1.0) -> dict:
    """Gradients of L with dL/dc = gbar through the Chebyshev-basis fit (float64)."""
    t = fp64.change_of_variable(x, center, scale)
    yv = np.asarray(y, dtype=np.float64)
    T = cheb_values(t, m)
    dT = cheb_derivative_values(t, m)
    G = [[math.fsum((T[j] * T[k]).tolist()) for k in range(m + 1)] for j in range(m + 1)]
    r = [math.fsum((T[j] * yv).tolist()) for j in range(m + 1)]
    c, st = fp64.gepp(G, r)
    lam, st2 = fp64.gepp(G, [float(g) for g in gbar])
    if st != fp64.OK or st2 != fp64.OK:
        return {"status": st if st != fp64.OK else st2}
    f = sum(cj * Tj for cj, Tj in zip(c, T))
    fp = sum(cj * dTj for cj, dTj in zip(c, dT))
    q = sum(lj * Tj for lj, Tj in zip(lam, T))
    qp = sum(lj * dTj for lj, dTj in zip(lam, dT))
    return {"gx": (qp * (yv - f) - q * fp) / scale, "gy": q, "lam": np.array(lam), "c": np.array(c),
            "status": fp64.OK}

