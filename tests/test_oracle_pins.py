"""Pins of the CPU oracle against what the paper and mathematics fix.

Each test ties the oracle to something other than itself: numbers printed in
the paper (Tables I-V, Sec. III), closed forms, exact rational arithmetic,
library routines of an independent algorithm (LAPACK's SVD least squares and
LU solve), invariants of the least-squares minimiser and brute force on tiny
inputs.  None of these tests needs a GPU.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from conftest import read_golden
from oracle import adjoint, c_oracle, exact, fp64, qr
from paper_1512_08017_amd import workloads as W


def table_i():
    rows, _ = read_golden("table_i.txt")
    xs = [r[0] for r in rows]
    ys = [r[1] for r in rows]
    return xs, ys


def polyfit_columns():
    rows, _ = read_golden("polyfit_coefficients.txt")
    out = {}
    for m, k, v, d in rows:
        out.setdefault(int(m), {})[int(k)] = (float(v), int(d))
    return out


def relerr(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


# --- the worked example of Sec. III ------------------------------------------

def test_table_i_fixture_matches_workload_module():
    xs, ys = table_i()
    assert xs == list(W.TABLE_I_X) and ys == list(W.TABLE_I_Y)


@pytest.mark.parametrize("m", [1, 2, 3])
def test_fp64_reproduces_polyfit_columns(m):
    """Tables II-IV: the exact minimiser rounds to the printed polyfit() values."""
    xs, ys = table_i()
    res = fp64.fit(np.array(xs, float), np.array(ys, float), m)
    assert res["status"] == fp64.OK
    for k, (v, d) in polyfit_columns()[m].items():
        assert abs(res["a"][k] - v) <= 0.5 * 10.0 ** -d + 1e-12, (m, k, res["a"][k], v)


@pytest.mark.parametrize("m", [1, 2, 3])
def test_exact_reproduces_polyfit_columns(m):
    xs, ys = table_i()
    a, _ = exact.fit_exact(xs, ys, m)
    for k, (v, d) in polyfit_columns()[m].items():
        assert abs(float(a[k]) - v) <= 0.5 * 10.0 ** -d, (m, k)


def test_table_v_sse_bounds():
    """Table V: the minimum SSE is below both printed sums and close to the
    paper's own elimination result (whose coefficients differ in the 4th decimal)."""
    xs, ys = table_i()
    _, notes = read_golden("table_v.txt")
    a, _ = exact.fit_exact(xs, ys, 3)
    sse_star = float(exact.sse_exact(xs, ys, a))
    assert sse_star <= notes["sum_e_f2"]
    assert sse_star <= notes["sum_e_p2"]
    assert abs(sse_star - notes["sum_e_f2"]) < 1e-3
    res = fp64.fit(np.array(xs, float), np.array(ys, float), 3)
    assert abs(fp64.sse(np.array(xs, float), np.array(ys, float), res["a"]) - sse_star) < 1e-9 * sse_star


def test_table_v_polyfit_rows_from_printed_coefficients():
    """Table V's y_p column and sum e_p^2 follow from evaluating the Table IV
    polyfit() coefficients as printed; this pins polyval and sse."""
    xs, ys = table_i()
    rows, notes = read_golden("table_v.txt")
    ap = [v for _, (v, _) in sorted(polyfit_columns()[3].items())]
    x = np.array(xs, float)
    yp = fp64.polyval(ap, x)
    for row, v in zip(rows, yp):
        assert abs(float(row[2]) - v) < 1e-3
    assert abs(fp64.sse(x, np.array(ys, float), ap) - notes["sum_e_p2"]) < 1e-3


@pytest.mark.parametrize("m", [1, 2, 3])
def test_fp64_matches_exact_on_table_i(m):
    xs, ys = table_i()
    a, _ = exact.fit_exact(xs, ys, m)
    res = fp64.fit(np.array(xs, float), np.array(ys, float), m)
    # exact on the decimal inputs vs float64 on their rounded values: cond(A) ~ 3e9
    assert relerr(res["a"], [float(v) for v in a]) < 1e-9


@pytest.mark.parametrize("m", [1, 2, 3])
def test_exact_normal_residual_is_zero(m):
    """First-order conditions of Sec. II: V^T r = 0 at the minimiser, exactly."""
    xs, ys = table_i()
    a, _ = exact.fit_exact(xs, ys, m)
    assert all(v == 0 for v in exact.normal_residual(xs, ys, a))


def test_normal_residual_hand_worked():
    """V^T r on three points, worked by hand: (x, y) = (0, 1), (1, 2), (2, 2).
    At a = 0, r = y: [sum y, sum x y, sum x^2 y] = [5, 6, 10].  At a = (1, 1),
    r = y - 1 - x = (0, 0, -1): [-1, -2, -4]."""
    xs, ys = [0, 1, 2], [1, 2, 2]
    assert exact.normal_residual(xs, ys, [0, 0, 0]) == [5, 6, 10]
    assert exact.normal_residual(xs, ys, [1, 1, 0]) == [-1, -2, -4]


@pytest.mark.parametrize("m,k", [(m, k) for m in (1, 2, 3) for k in range(m + 1)])
def test_normal_residual_off_the_minimiser(m, k):
    """Away from the minimiser: with a = a* + delta e_k, r = r* - delta x^k, so
    V^T r = -delta V^T V e_k = -delta (S_k, S_(k+1), .., S_(k+m)), the k-th
    column of the Hankel matrix of Sec. II, exactly (Table I points)."""
    xs, ys = table_i()
    a, _ = exact.fit_exact(xs, ys, m)
    S, _ = exact.power_sums_exact(xs, ys, m)
    delta = Fraction(3, 7)
    ap = list(a)
    ap[k] += delta
    assert exact.normal_residual(xs, ys, ap) == [-delta * S[j + k] for j in range(m + 1)]


def test_gepp_many_is_gepp_per_system():
    """The batched elimination gives every system the bits of fp64.gepp (same
    pivots, same operations), singular systems included."""
    rng = np.random.default_rng(44)
    for n in (1, 2, 3, 5):
        A = rng.standard_normal((40, n, n))
        B = rng.standard_normal((40, n))
        A[3] = 0.0                      # singular
        if n > 1:
            A[5, 1] = A[5, 0]           # singular (two equal rows)
            A[7, :, 0] = 1.0            # ties in the first column: first row wins
        X, ok = fp64.gepp_many(A, B)
        for i in range(40):
            x1, st = fp64.gepp(A[i].tolist(), B[i].tolist())
            assert ok[i] == (st == fp64.OK)
            if ok[i]:
                assert np.array_equal(X[i], np.array(x1))


def test_printed_matrix_a00_reading():
    """The printed A_00 = 1 does not reproduce Table II; A_00 = n does (reading of Sec. II)."""
    xs, ys = table_i()
    S, T = exact.power_sums_exact(xs, ys, 1)
    A = [[Fraction(1), S[1]], [S[1], S[2]]]
    b, _ = exact.gepp_exact(A, T[:2])
    v, d = polyfit_columns()[1][0]
    assert abs(float(b[0]) - v) > 0.5 * 10.0 ** -d
    A[0][0] = S[0]
    b, _ = exact.gepp_exact(A, T[:2])
    assert abs(float(b[0]) - v) <= 0.5 * 10.0 ** -d


# --- closed forms -------------------------------------------------------------

def test_degree_zero_is_mean():
    fit = W.random_small(37, 0, seed=1)
    res = fp64.fit(fit.x, fit.y, 0)
    assert abs(res["a"][0] - math.fsum(fit.y.tolist()) / 37) < 1e-15


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_linear_textbook_formula(seed):
    """m = 1: a_1 = (n Sxy - Sx Sy)/(n Sxx - Sx^2), a_0 = (Sy - a_1 Sx)/n, in exact rationals."""
    fit = W.random_small(50, 1, seed=seed, lo=0.0, hi=10.0)
    xs = [Fraction(float(v)) for v in fit.x]
    ys = [Fraction(float(v)) for v in fit.y]
    n = len(xs)
    sx, sy = sum(xs), sum(ys)
    sxx = sum(v * v for v in xs)
    sxy = sum(u * v for u, v in zip(xs, ys))
    a1 = (n * sxy - sx * sy) / (n * sxx - sx * sx)
    a0 = (sy - a1 * sx) / n
    res = fp64.fit(fit.x, fit.y, 1)
    assert relerr(res["a"], [float(a0), float(a1)]) < 1e-13
    ae, _ = exact.fit_exact(fit.x, fit.y, 1)
    assert ae == [a0, a1]
    co = c_oracle.fit(fit.x, fit.y, 1)
    assert relerr(co["a"], [float(a0), float(a1)]) < 1e-13


def test_faulhaber_power_sums():
    """x = 1..N: sum x = N(N+1)/2, sum x^2 = N(N+1)(2N+1)/6, sum x^3 = (N(N+1)/2)^2,
    sum x^4 = N(N+1)(2N+1)(3N^2+3N-1)/30 -- exact integers below 2^53."""
    N = 1000
    x = np.arange(1, N + 1, dtype=np.float64)
    y = np.ones(N)
    closed = [N, N * (N + 1) // 2, N * (N + 1) * (2 * N + 1) // 6, (N * (N + 1) // 2) ** 2,
              N * (N + 1) * (2 * N + 1) * (3 * N * N + 3 * N - 1) // 30]
    S, T = fp64.power_sums(x, y, 2)
    assert [int(v) for v in S] == closed
    assert [int(v) for v in T] == closed[:3]
    Sc, Tc = c_oracle.power_sums(x, y, 2)
    assert [int(v) for v in Sc] == closed
    assert [int(v) for v in Tc] == closed[:3]
    Sf, _ = c_oracle.power_sums(x.astype(np.float32), y.astype(np.float32), 2)
    assert [int(v) for v in Sf] == closed


@pytest.mark.parametrize("m", [1, 2, 3, 4])
def test_noiseless_recovery(m):
    """Integer coefficients on dyadic x: y is exact, and so is the recovered polynomial."""
    rng = np.random.default_rng(m)
    coef = rng.integers(-5, 6, m + 1).astype(float)
    x = rng.integers(-64, 65, 200) / 16.0
    y = np.zeros_like(x)
    for c in coef[::-1]:
        y = y * x + c
    a, _ = exact.fit_exact(x, y, m)
    assert [float(v) for v in a] == list(coef)
    res = fp64.fit(x, y, m)
    assert np.max(np.abs(res["a"] - coef)) < 1e-11
    assert np.max(np.abs(c_oracle.fit(x, y, m)["a"] - coef)) < 1e-11
    assert np.max(np.abs(qr.lstsq_qr(x, y, m) - coef)) < 1e-11


@pytest.mark.parametrize("m", [1, 2, 3])
def test_interpolation_when_n_equals_m_plus_1(m):
    """n = m+1 distinct points: the fit interpolates (zero residual); compare a
    Lagrange-form interpolant evaluated exactly."""
    x = [Fraction(k, 3) - 1 for k in range(m + 1)]
    y = [Fraction((-1) ** k * (k + 2), 7) for k in range(m + 1)]
    a, _ = exact.fit_exact(x, y, m)
    for xi, yi in zip(x, y):
        assert exact.polyval_exact(a, xi) == yi
    z = Fraction(5, 11)
    lag = sum(yi * math.prod((z - xj) / (xi - xj) for j, xj in enumerate(x) if xj != xi)
              for xi, yi in zip(x, y))
    assert exact.polyval_exact(a, z) == lag


# --- agreement with independent library routines ------------------------------

@pytest.mark.parametrize("seed,m", [(0, 1), (1, 2), (2, 3), (3, 5), (4, 8)])
def test_fp64_vs_lapack_svd_lstsq(seed, m):
    """LAPACK gelsd (SVD) solves the same least-squares problem another way."""
    fit = W.random_small(300, m, seed=seed)
    V = np.vander(fit.x, m + 1, increasing=True)
    ref = np.linalg.lstsq(V, fit.y, rcond=None)[0]
    res = fp64.fit(fit.x, fit.y, m)
    tol = 1e-12 if m <= 3 else 1e-8
    assert relerr(res["a"], ref) < tol
    assert relerr(qr.lstsq_qr(fit.x, fit.y, m), ref) < tol
    assert relerr(c_oracle.fit(fit.x, fit.y, m)["a"], ref) < tol


@pytest.mark.parametrize("n", [2, 3, 5, 9])
def test_gepp_vs_lapack_gesv(n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n))
    B = rng.standard_normal(n)
    X, st = fp64.gepp(A.tolist(), B.tolist())
    assert st == fp64.OK
    assert relerr(X, np.linalg.solve(A, B)) < 1e-12


def test_gepp_pivots_on_first_largest():
    """A zero leading entry forces a row swap; ties choose the first row."""
    A = [[0.0, 1.0], [2.0, 3.0]]
    X, st = fp64.gepp(A, [1.0, 5.0])
    assert st == fp64.OK and X == [1.0, 1.0]
    X, st = fp64.gepp([[1.0, 2.0], [-1.0, 1.0]], [3.0, 0.0])  # |1| == |-1|: keep row 0
    assert st == fp64.OK and np.allclose(X, [1.0, 1.0])


def test_householder_factorisation():
    fit = W.random_small(40, 3, seed=7)
    V = qr.vandermonde(fit.x, 3)
    Q, R = qr.householder_qr(V)
    assert np.allclose(Q.T @ Q, np.eye(4), atol=1e-14)
    assert np.allclose(np.tril(R, -1), 0.0)
    assert np.allclose(Q @ R, V, atol=1e-13)
    Rn = np.linalg.qr(V, mode="r")
    assert np.allclose(np.abs(R), np.abs(Rn), atol=1e-12)


def test_tsqr_equals_single_qr():
    fit = W.random_small(5000, 3, seed=8)
    b1 = qr.lstsq_qr(fit.x, fit.y, 3, block=1 << 20)
    b2 = qr.lstsq_qr(fit.x, fit.y, 3, block=333)
    assert relerr(b1, b2) < 1e-13


# --- invariants of the minimiser -----------------------------------------------

def test_normal_residual_fp64_bound():
    fit = W.random_small(2000, 3, seed=9)
    res = fp64.fit(fit.x, fit.y, 3)
    r = fit.y - fp64.polyval(res["a"], fit.x)
    for k in range(4):
        terms = fit.x ** k * r
        assert abs(math.fsum(terms.tolist())) <= 10 * 2000 * 2.0 ** -52 * np.sum(np.abs(terms)) + 1e-300


def test_affine_change_of_variable_invariance():
    """The minimiser does not depend on (c, s); the oracle's unscale must agree."""
    fit = W.random_small(500, 3, seed=10, lo=3.0, hi=5.0)
    a_ex, _ = exact.fit_exact(fit.x, fit.y, 3)
    a_ex = [float(v) for v in a_ex]
    r0 = fp64.fit(fit.x, fit.y, 3)
    r1 = fp64.fit(fit.x, fit.y, 3, center=4.0, scale=0.5)
    r2 = fp64.fit(fit.x, fit.y, 3, center=3.5, scale=2.0)
    assert relerr(r0["a"], a_ex) < 1e-8          # raw basis: cond(A) ~ 1e10 on [3, 5]
    assert relerr(r1["a"], a_ex) < 1e-10          # unscale to the x-basis cancels on [3, 5]
    assert relerr(r2["a"], a_ex) < 1e-10
    # t-basis coefficients describe the same polynomial
    t = (fit.x - 4.0) / 0.5
    assert np.allclose(fp64.polyval(r1["b"], t), fp64.polyval(r0["a"], fit.x), rtol=0, atol=1e-9)


def test_unscale_exact_vs_float():
    b = [Fraction(3, 7), Fraction(-2, 5), Fraction(1, 3), Fraction(5, 9)]
    c, s = Fraction(1001, 2), Fraction(1, 2)
    a = exact.unscale_exact(b, c, s)
    af = fp64.unscale([float(v) for v in b], float(c), float(s))
    for u, v in zip(af, a):
        assert abs(u - float(v)) <= 1e-14 * abs(float(v))
    # the polynomials agree at a point
    x = Fraction(10007, 10)
    assert exact.polyval_exact(a, x) == exact.polyval_exact(b, (x - c) / s)


def test_permutation_duplication_and_linearity():
    fit = W.random_small(300, 2, seed=11)
    base = fp64.fit(fit.x, fit.y, 2)["a"]
    perm = np.random.default_rng(0).permutation(300)
    assert relerr(fp64.fit(fit.x[perm], fit.y[perm], 2)["a"], base) < 1e-13
    assert relerr(fp64.fit(np.tile(fit.x, 3), np.tile(fit.y, 3), 2)["a"], base) < 1e-13
    y2 = np.random.default_rng(1).standard_normal(300)
    lin = fp64.fit(fit.x, 2.0 * fit.y - 3.0 * y2, 2)["a"]
    comb = 2.0 * base - 3.0 * fp64.fit(fit.x, y2, 2)["a"]
    assert relerr(lin, comb) < 1e-12


def test_sse_non_increasing_in_degree():
    fit = W.random_small(200, 4, seed=12)
    sses = [fp64.sse(fit.x, fit.y, fp64.fit(fit.x, fit.y, m)["a"]) for m in range(0, 7)]
    assert all(b <= a * (1 + 1e-12) for a, b in zip(sses, sses[1:]))


def test_singular_when_too_few_distinct_x():
    x = np.array([1.0, 1.0, 2.0, 2.0, 2.0])
    y = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    assert fp64.fit(x, y, 2)["status"] == fp64.SINGULAR
    assert c_oracle.fit(x, y, 2)["status"] == "singular"
    assert exact.fit_exact(x, y, 2) == (None, None)
    assert fp64.fit(x, y, 1)["status"] == fp64.OK


def test_nonfinite_inputs():
    x = np.array([1.0, 2.0, np.nan, 4.0])
    y = np.array([1.0, 2.0, 3.0, 4.0])
    assert fp64.fit(x, y, 1)["status"] == fp64.NONFINITE
    assert c_oracle.fit(x, y, 1)["status"] == "nonfinite"


# --- exact truth for large shifted inputs -------------------------------------

def test_grid_power_sums_equal_brute_force():
    fit = W.shifted_quintic(n=300, seed=5)
    S, T = exact.grid_power_sums(fit.x, fit.y, 5, 1000.5, 0.5, 2.0 ** -14)
    Sb, Tb = exact.power_sums_exact(fit.x, fit.y, 5, Fraction(2001, 2), Fraction(1, 2))
    assert S == Sb and T == Tb
    a, b = exact.fit_exact_grid(fit.x, fit.y, 5, 1000.5, 0.5, 2.0 ** -14)
    a2, b2 = exact.fit_exact(fit.x, fit.y, 5, Fraction(2001, 2), Fraction(1, 2))
    assert a == a2 and b == b2


def test_grid_rejects_off_grid_points():
    with pytest.raises(ValueError):
        exact.grid_power_sums(np.array([1000.0, 1000.3]), np.array([1.0, 2.0], np.float32),
                              1, 1000.5, 0.5, 2.0 ** -14)


def test_shifted_quintic_oracles_agree_and_raw_basis_fails():
    """On x in [1000, 1001] the shifted float64 routes match the exact minimiser;
    the raw x-basis normal equations do not (documented failure)."""
    fit = W.shifted_quintic(n=20000, seed=6)
    a_ex, b_ex = exact.fit_exact_grid(fit.x, fit.y, 5, 1000.5, 0.5, 2.0 ** -14)
    b_ex = np.array([float(v) for v in b_ex])
    a_ex = np.array([float(v) for v in a_ex])
    sh = c_oracle.fit(fit.x, fit.y, 5, center=1000.5, scale=0.5)
    per_coef_b = np.abs(sh["b"] - b_ex) / np.abs(b_ex)
    per_coef_a = np.abs(sh["a"] - a_ex) / np.abs(a_ex)
    assert per_coef_b.max() < 1e-9 and per_coef_a.max() < 1e-9
    bq = qr.lstsq_qr(fit.x, fit.y, 5, center=1000.5, scale=0.5)
    assert (np.abs(bq - b_ex) / np.abs(b_ex)).max() < 1e-9
    raw = c_oracle.fit(fit.x, fit.y, 5)
    assert raw["status"] != "ok" or (np.abs(raw["a"] - a_ex) / np.abs(a_ex)).max() > 1e-3


# --- the C oracle --------------------------------------------------------------

@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_c_oracle_matches_python_oracle(dtype):
    fit = W.random_small(200_003, 3, seed=13, dtype=dtype)
    py = fp64.fit(fit.x, fit.y, 3)
    c1 = c_oracle.fit(fit.x, fit.y, 3, threads=1)
    c4 = c_oracle.fit(fit.x, fit.y, 3, threads=4)
    assert np.array_equal(c1["a"], c4["a"])       # chunk order fixed: thread count irrelevant
    assert relerr(c1["a"], py["a"]) < 1e-13
    assert np.max(np.abs(c1["S"] - py["S"]) / np.abs(py["S"])) < 1e-15


def test_c_oracle_batched_equals_single():
    bf = W.random_batch([1, 5, 100, 7, 0, 2000], [1, 2, 3, 3, 1, 2], seed=14)
    a, st = c_oracle.fit_batched(bf.x, bf.y, bf.offsets, bf.degrees, stride=4)
    for f in range(bf.batch):
        lo, hi = bf.offsets[f], bf.offsets[f + 1]
        m = int(bf.degrees[f])
        single = c_oracle.fit(bf.x[lo:hi], bf.y[lo:hi], m)
        assert c_oracle.STATUS[int(st[f])] == single["status"]
        if single["status"] == "ok":
            assert relerr(a[f, : m + 1], single["a"]) < 1e-13
    assert c_oracle.STATUS[int(st[0])] == "singular" and c_oracle.STATUS[int(st[4])] == "singular"


# --- adjoint --------------------------------------------------------------------

def _loss_factory(target):
    return lambda a: np.sum((a - target) ** 2, axis=-1)


@pytest.mark.parametrize("center,scale", [(0.0, 1.0), (0.25, 0.5)])
def test_adjoint_vs_finite_differences(center, scale):
    fit = W.random_small(60, 2, seed=15)
    target = np.random.default_rng(3).standard_normal(3)
    a = fp64.fit(fit.x, fit.y, 2)["a"]
    g = adjoint.gradients(fit.x, fit.y, 2, 2.0 * (a - target), center, scale)
    fd = adjoint.fd_gradients(fit.x, fit.y, 2, _loss_factory(target), h=1e-6, center=center, scale=scale)
    assert relerr(g["dx"], fd["dx"]) < 1e-6
    assert relerr(g["dy"], fd["dy"]) < 1e-6


def test_adjoint_vs_torch_autograd():
    """Independent library pin: float64 autograd through a dense solve of V^T V a = V^T y."""
    torch = pytest.importorskip("torch")
    fit = W.random_small(80, 3, seed=16)
    target = np.random.default_rng(4).standard_normal(4)
    xt = torch.tensor(fit.x, dtype=torch.float64, requires_grad=True)
    yt = torch.tensor(fit.y, dtype=torch.float64, requires_grad=True)
    V = torch.stack([xt ** k for k in range(4)], dim=1)
    a = torch.linalg.solve(V.T @ V, V.T @ yt)
    loss = ((a - torch.tensor(target)) ** 2).sum()
    loss.backward()
    ao = fp64.fit(fit.x, fit.y, 3)["a"]
    g = adjoint.gradients(fit.x, fit.y, 3, 2.0 * (ao - target), 0.1, 0.5)
    assert relerr(g["dx"], xt.grad.numpy()) < 1e-9
    assert relerr(g["dy"], yt.grad.numpy()) < 1e-9


def test_adjoint_identities():
    """V^T dL/dy = gbar; sum y dL/dy = gbar.a; translation and dilation identities."""
    fit = W.random_small(500, 3, seed=17, lo=-2.0, hi=3.0)
    gbar = np.random.default_rng(5).standard_normal(4)
    g = adjoint.gradients(fit.x, fit.y, 3, gbar, 0.5, 2.0)
    a = g["a"]
    V = np.vander(fit.x, 4, increasing=True)
    assert relerr(V.T @ g["dy"], gbar) < 1e-10
    assert abs(np.dot(fit.y, g["dy"]) - np.dot(gbar, a)) < 1e-9 * np.abs(gbar * a).sum()
    trans = -sum(gbar[k] * (k + 1) * a[k + 1] for k in range(3))
    assert abs(np.sum(g["dx"]) - trans) < 1e-9 * (np.abs(g["dx"]).sum())
    dil = -sum(k * gbar[k] * a[k] for k in range(4))
    assert abs(np.dot(fit.x, g["dx"]) - dil) < 1e-9 * (np.abs(fit.x * g["dx"]).sum())


@pytest.mark.parametrize("lo,hi", [(0, 3000), (1234, 4321), (1024 * 1021 - 700, 1024 * 1021 + 900)])
def test_periodic_power_sums_match_brute_force(lo, hi):
    """The closed form of the periodic pattern's sums (the reference of the
    beyond-2^31 checks) equals the exact sums over the points themselves,
    also across a joint period of the two residues."""
    x, y = W.periodic_points_np(lo, hi)
    S, T = exact.periodic_power_sums(lo, hi, 3)
    S2, T2 = exact.power_sums_exact(x, y, 3)
    assert S == S2 and T == T2
    assert S[0] == hi - lo


def test_periodic_power_sums_are_additive_and_symmetric():
    """Sums over [a, c) are the sums over [a, b) plus [b, c); over whole
    periods of x the odd power sums vanish (x takes +-v equally often)."""
    a, b, c = 5, (1 << 31) - 3, (1 << 31) + 1_000_003
    S1, T1 = exact.periodic_power_sums(a, b, 3)
    S2, T2 = exact.periodic_power_sums(b, c, 3)
    S, T = exact.periodic_power_sums(a, c, 3)
    assert S == [u + v for u, v in zip(S1, S2)] and T == [u + v for u, v in zip(T1, T2)]
    Sp, _ = exact.periodic_power_sums(0, 1024 * 4096, 3)
    assert Sp[1] == Sp[3] == Sp[5] == 0 and Sp[0] == 1024 * 4096
