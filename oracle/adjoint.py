"""Adjoint (reverse-mode derivative) oracle of the least-squares fit.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The fit of Sec. II, in the variable t = (x - c)/s with v(t) = [1, t, .., t^m]:
A_t = sum_i v(t_i) v(t_i)^T, B_t = sum_i y_i v(t_i), A_t b = B_t, and the
x-basis coefficients a = M b with M_kj = C(j,k) (-c)^(j-k) s^(-j) (j >= k).
For a scalar loss L(a) with gbar = dL/da:

* dL/db = M^T gbar =: g_t, and with lambda = A_t^-1 g_t (A_t is symmetric),
  dL/dB_t = lambda and dL/dA_t = -lambda b^T;
* dL/dy_i = lambda . v(t_i) = q(t_i),   q(t) = sum_j lambda_j t^j;
* dL/dt_i = lambda . (y_i v'(t_i) - (v'(t_i) v(t_i)^T + v(t_i) v'(t_i)^T) b)
          = q'(t_i) r_i - q(t_i) f'(t_i),  r_i = y_i - f(t_i), f = sum_j b_j t^j;
* dL/dx_i = dL/dt_i / s.

The minimiser a does not depend on the choice of (c, s), so (c, s) are held
fixed.  ``fd_gradients`` differentiates the float64 fit numerically with
central differences, recomputing each perturbed fit from its power sums.
"""
from __future__ import annotations

import math

import numpy as np

from . import fp64


def basis_map(m: int, center: float, scale: float) -> np.ndarray:
    """M with a = M b (x-basis from t-basis)."""
    M = np.zeros((m + 1, m + 1))
    for j in range(m + 1):
        for k in range(j + 1):
            M[k, j] = math.comb(j, k) * (-center) ** (j - k) * scale ** (-j)
    return M


def _poly_and_derivative(coef, t):
    """p(t) and p'(t), coefficients ascending, float64."""
    p = np.zeros_like(t)
    dp = np.zeros_like(t)
    for c in list(coef)[::-1]:
        dp = dp * t + p
        p = p * t + c
    return p, dp


def gradients(x, y, m: int, gbar, center: float = 0.0, scale: float = 1.0) -> dict:
    """dL/dx, dL/dy (float64 arrays) for dL/da = gbar at the least-squares fit."""
    res = fp64.fit(x, y, m, center, scale)
    if res["status"] != fp64.OK:
        raise ValueError(f"fit is {res['status']}")
    b = res["b"]
    A, _ = fp64.assemble(res["S"], res["T"], m)
    g_t = basis_map(m, center, scale).T @ np.asarray(gbar, dtype=np.float64)
    lam, status = fp64.gepp(A, list(g_t))
    if status != fp64.OK:
        raise ValueError(f"adjoint system is {status}")
    t = fp64.change_of_variable(x, center, scale)
    yv = np.asarray(y, dtype=np.float64)
    f, df = _poly_and_derivative(b, t)
    q, dq = _poly_and_derivative(lam, t)
    r = yv - f
    return {"dx": (dq * r - q * df) / scale, "dy": q, "a": res["a"], "b": b, "lam": np.array(lam)}


def fd_gradients(x, y, m: int, loss_of_a, h: float = 1e-6, center: float = 0.0,
                 scale: float = 1.0, which: str = "both") -> dict:
    """Central differences of loss_of_a(fit(x, y)) w.r.t. every x_i and y_i.

    ``loss_of_a`` maps coefficient vectors to losses row-wise: an array of
    shape (K, m+1) of x-basis coefficients to K losses.  A perturbation of one
    point changes each power sum by one term, so each perturbed fit is solved
    from S +- (new term - old term), with the old and new terms taken from the
    point itself; the perturbed systems of all points are assembled as Hankel
    matrices, eliminated by ``fp64.gepp_many`` (the steps of ``fp64.gepp`` for
    each system) and mapped back to the x-basis with the sums of
    ``fp64.unscale``.
    """
    res = fp64.fit(x, y, m, center, scale)
    S0, T0 = np.array(res["S"]), np.array(res["T"])
    t = fp64.change_of_variable(x, center, scale)
    yv = np.asarray(y, dtype=np.float64)
    xv = np.asarray(x, dtype=np.float64)
    Mb = basis_map(m, center, scale)

    def terms(tv, yvv):
        """Per-point terms t^p (p = 0..2m) and t^j y (j = 0..m): arrays [n, .]."""
        S = np.stack([tv ** p for p in range(2 * m + 1)], axis=1)
        T = np.stack([tv ** j * yvv for j in range(m + 1)], axis=1)
        return S, T

    def losses(S, T):
        A = np.stack([np.stack([S[:, j + k] for k in range(m + 1)], axis=1) for j in range(m + 1)], axis=1)
        b, ok = fp64.gepp_many(A, T)
        if not ok.all():
            raise ValueError("a perturbed fit is singular")
        # a_k = sum_(j>=k) b_j M_kj, the terms of fp64.unscale in the same order
        a = np.zeros_like(b)
        for k in range(m + 1):
            for j in range(k, m + 1):
                a[:, k] += b[:, j] * Mb[k, j]
        return np.asarray(loss_of_a(a), dtype=np.float64)

    s_old, t_old = terms(t, yv)
    out = {}
    if which in ("both", "x"):
        vals = []
        for sgn in (1.0, -1.0):
            tp = (xv + sgn * h - center) / scale
            s_new, t_new = terms(tp, yv)
            vals.append(losses(S0 + (s_new - s_old), T0 + (t_new - t_old)))
        out["dx"] = (vals[0] - vals[1]) / (2.0 * h)
    if which in ("both", "y"):
        vals = []
        for sgn in (1.0, -1.0):
            _, t_new = terms(t, yv + sgn * h)
            vals.append(losses(np.broadcast_to(S0, s_old.shape), T0 + (t_new - t_old)))
        out["dy"] = (vals[0] - vals[1]) / (2.0 * h)
    return out
