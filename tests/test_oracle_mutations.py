"""Planted mistakes in the float64 oracle must break at least one pin.

Each case replaces one step of ``oracle.fp64`` (CPU only) with a plausible
wrong version -- a dropped term, a wrong sign or index, a transposed operand,
the printed A_00 = 1 -- and checks that the pin set rejects it.
"""
import math

import numpy as np
import pytest

from conftest import read_golden
from fractions import Fraction

from oracle import exact, fp64
from paper_1512_08017_amd import workloads as W


def _pins_hold() -> bool:
    rows, _ = read_golden("table_i.txt")
    x = np.array([float(r[0]) for r in rows])
    y = np.array([float(r[1]) for r in rows])
    coef_rows, _ = read_golden("polyfit_coefficients.txt")
    for m, k, v, d in coef_rows:
        a = fp64.fit(x, y, int(m))["a"]
        if not abs(a[int(k)] - float(v)) <= 0.5 * 10.0 ** -int(d) + 1e-12:
            return False
    # centred fit of shifted data must match the plain one (affine invariance)
    f = W.random_small(400, 3, seed=21, lo=-1.0, hi=2.0)
    a0 = fp64.fit(f.x, f.y, 3)["a"]
    a1 = fp64.fit(f.x, f.y, 3, center=0.5, scale=2.0)["a"]
    if not np.max(np.abs(a0 - a1)) < 1e-9 * np.max(np.abs(a0)):
        return False
    # least-squares optimality: V^T r = 0 to rounding
    r = f.y - fp64.polyval(a0, f.x)
    for k in range(4):
        t = f.x ** k * r
        if abs(math.fsum(t.tolist())) > 1e-10 * np.sum(np.abs(t)):
            return False
    return True


def test_unmodified_oracle_passes():
    assert _pins_hold()


def _a00_is_one(S, T, m):
    A = [[S[j + k] for k in range(m + 1)] for j in range(m + 1)]
    A[0][0] = 1.0
    return A, [T[j] for j in range(m + 1)]


def _printed_last_row(S, T, m):
    A = [[S[j + k] for k in range(m + 1)] for j in range(m + 1)]
    A[m] = [S[m]] + [S[m + k + 1] if m + k + 1 <= 2 * m else S[2 * m] for k in range(1, m + 1)]
    return A, [T[j] for j in range(m + 1)]


def _rhs_shifted(S, T, m):
    A = [[S[j + k] for k in range(m + 1)] for j in range(m + 1)]
    return A, [T[min(j + 1, m)] for j in range(m + 1)]


def _unscale_wrong_sign(b, center=0.0, scale=1.0):
    m = len(b) - 1
    return [math.fsum(b[j] * math.comb(j, k) * center ** (j - k) * scale ** (-j) for j in range(k, m + 1))
            for k in range(m + 1)]


def _unscale_dropped_scale(b, center=0.0, scale=1.0):
    m = len(b) - 1
    return [math.fsum(b[j] * math.comb(j, k) * (-center) ** (j - k) for j in range(k, m + 1))
            for k in range(m + 1)]


def _power_sums_dropped_y(x, y, m, center=0.0, scale=1.0):
    S, T = ORIG_POWER_SUMS(x, y, m, center, scale)
    T = [float(np.sum(fp64.change_of_variable(x, center, scale) ** j)) for j in range(m + 1)]
    return S, T


def _gepp_no_row_swap_update(A, B, singular_rel=fp64.SINGULAR_REL):
    n = len(A)
    M = [list(A[i]) + [B[i]] for i in range(n)]
    for k in range(n):
        for r in range(k + 1, n):
            l = M[r][k] / M[k][k]
            for c in range(k + 1, n + 1):     # forgets to eliminate into the pivot column's rhs
                M[r][c] -= l * M[k][c] if c < n else 0.0
    X = [0.0] * n
    for i in range(n - 1, -1, -1):
        X[i] = (M[i][n] - sum(M[i][c] * X[c] for c in range(i + 1, n))) / M[i][i]
    return X, fp64.OK


ORIG_POWER_SUMS = fp64.power_sums


@pytest.mark.parametrize("target,replacement", [
    ("assemble", _a00_is_one),
    ("assemble", _printed_last_row),
    ("assemble", _rhs_shifted),
    ("unscale", _unscale_wrong_sign),
    ("unscale", _unscale_dropped_scale),
    ("power_sums", _power_sums_dropped_y),
    ("gepp", _gepp_no_row_swap_update),
])
def test_planted_mistake_is_caught(monkeypatch, target, replacement):
    monkeypatch.setattr(fp64, target, replacement)
    assert not _pins_hold()


# --- V^T r (the first-order conditions of Sec. II) ---------------------------

def _normal_residual_pins_hold() -> bool:
    rows, _ = read_golden("table_i.txt")
    xs = [r[0] for r in rows]
    ys = [r[1] for r in rows]
    if exact.normal_residual([0, 1, 2], [1, 2, 2], [1, 1, 0]) != [-1, -2, -4]:
        return False
    for m in (1, 2, 3):
        a, _ = exact.fit_exact(xs, ys, m)
        if any(v != 0 for v in exact.normal_residual(xs, ys, a)):
            return False
        S, _ = exact.power_sums_exact(xs, ys, m)
        for k in range(m + 1):
            ap = list(a)
            ap[k] += Fraction(3, 7)
            if exact.normal_residual(xs, ys, ap) != [-Fraction(3, 7) * S[j + k] for j in range(m + 1)]:
                return False
    return True


def _normal_residual_drops_power(xs, ys, a):
    m = len(a) - 1
    r = [exact.frac(y) - exact.polyval_exact(a, x) for x, y in zip(xs, ys)]
    return [sum(r, Fraction(0)) for _ in range(m + 1)]


def _normal_residual_wrong_sign(xs, ys, a):
    m = len(a) - 1
    r = [exact.polyval_exact(a, x) - exact.frac(y) for x, y in zip(xs, ys)]
    return [sum((exact.frac(x) ** k * ri for x, ri in zip(xs, r)), Fraction(0)) for k in range(m + 1)]


def _normal_residual_shifted_power(xs, ys, a):
    m = len(a) - 1
    r = [exact.frac(y) - exact.polyval_exact(a, x) for x, y in zip(xs, ys)]
    return [sum((exact.frac(x) ** (k + 1) * ri for x, ri in zip(xs, r)), Fraction(0)) for k in range(m + 1)]


def test_unmodified_normal_residual_passes():
    assert _normal_residual_pins_hold()


@pytest.mark.parametrize("replacement", [_normal_residual_drops_power, _normal_residual_wrong_sign,
                                         _normal_residual_shifted_power])
def test_planted_normal_residual_mistake_is_caught(monkeypatch, replacement):
    monkeypatch.setattr(exact, "normal_residual", replacement)
    assert not _normal_residual_pins_hold()
