"""Pins of the Chebyshev-basis oracle (CPU only)."""
from fractions import Fraction

import numpy as np
import pytest

from oracle import cheb, exact, fp64
from paper_1512_08017_amd import workloads as W


def test_cheb_values_closed_form():
    """T_k(cos th) = cos(k th)."""
    th = np.linspace(0.1, 3.0, 50)
    T = cheb.cheb_values(np.cos(th), 12)
    for k in range(13):
        assert np.max(np.abs(T[k] - np.cos(k * th))) < 1e-13


def test_cheb_to_monomial_known_polynomials():
    """T_2 = 2t^2 - 1, T_3 = 4t^3 - 3t, T_4 = 8t^4 - 8t^2 + 1 (exact)."""
    F = Fraction
    assert cheb.cheb_to_monomial([F(0), F(0), F(1)]) == [-1, 0, 2]
    assert cheb.cheb_to_monomial([F(0), F(0), F(0), F(1)]) == [0, -3, 0, 4]
    assert cheb.cheb_to_monomial([F(0), F(0), F(0), F(0), F(1)]) == [1, 0, -8, 0, 8]


@pytest.mark.parametrize("m", [1, 2, 3, 5])
def test_same_minimiser_as_monomial_route(m):
    """The basis does not change the least-squares minimiser (exact arithmetic)."""
    fit = W.random_small(40, m, seed=30 + m)
    c = cheb.fit_cheb_exact(fit.x, fit.y, m, Fraction(1, 4), 2)
    a_mono, _ = exact.fit_exact(fit.x, fit.y, m)
    b = cheb.cheb_to_monomial(c)
    assert exact.unscale_exact(b, Fraction(1, 4), 2) == a_mono


@pytest.mark.parametrize("m", [4, 8, 12, 16])
def test_fp64_vs_exact_and_numpy_chebfit(m):
    fit = W.random_small(2000, m, seed=40 + m)
    res = cheb.fit_cheb(fit.x, fit.y, m)
    ce = cheb.fit_cheb_exact(fit.x[:300], fit.y[:300], m) if m <= 8 else None
    if ce is not None:
        r300 = cheb.fit_cheb(fit.x[:300], fit.y[:300], m)
        assert np.max(np.abs(r300["c"] - np.array([float(v) for v in ce]))) < 1e-11 * np.max(np.abs(r300["c"]))
    ref = np.polynomial.chebyshev.chebfit(fit.x, fit.y, m)   # LAPACK least squares on the Chebyshev matrix
    assert np.max(np.abs(res["c"] - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_monomial_route_fails_where_chebyshev_holds():
    """At degree 20 on [-1, 1] the monomial normal matrix is numerically
    singular in float64 even with correctly rounded sums; the Chebyshev route
    keeps full precision (against numpy's chebfit)."""
    fit = W.random_small(20000, 20, seed=60)
    ref = np.polynomial.chebyshev.chebfit(fit.x, fit.y, 20)
    res = cheb.fit_cheb(fit.x, fit.y, 20)
    assert np.max(np.abs(res["c"] - ref)) <= 1e-10 * np.max(np.abs(ref))
    mono = fp64.fit(fit.x, fit.y, 20)
    if mono["status"] == fp64.OK:
        c_from_mono = np.polynomial.chebyshev.poly2cheb(mono["b"])
        assert np.max(np.abs(c_from_mono - ref)) > 1e-6 * np.max(np.abs(ref))
    else:
        assert mono["status"] == fp64.SINGULAR


@pytest.mark.parametrize("m", [1, 4, 9, 16])
def test_c_oracle_matches_python_oracle(m):
    """The plain-C Chebyshev route (entrywise compensated sums, chunked) agrees
    with the fsum route, and its Gram matrix is the definition's."""
    from oracle import c_oracle
    wl = W.runge(n=3000, seed=40 + m, dtype=np.float64, lo=-2.0, hi=3.0)
    r = c_oracle.cheb_fit(wl.x, wl.y, m, 0.5, 2.5)
    p = cheb.fit_cheb(wl.x, wl.y, m, 0.5, 2.5)
    assert r["status"] == "ok"
    assert np.max(np.abs(r["c"] - p["c"])) <= 1e-12 * np.max(np.abs(p["c"]))
    t = (wl.x - 0.5) / 2.5
    V = np.polynomial.chebyshev.chebvander(t, m)
    assert np.allclose(r["G"], V.T @ V, rtol=1e-12, atol=1e-12 * wl.x.size)
    assert r["G"][0, 0] == wl.x.size


def test_c_oracle_batched_matches_single():
    from oracle import c_oracle
    lengths = [0, 3, 17, 500, 2000]
    degrees = [2, 3, 16, 9, 12]
    bf = W.random_batch(lengths, degrees, seed=9, dtype=np.float64)
    out, st = c_oracle.cheb_fit_batched(bf.x, bf.y, bf.offsets, bf.degrees, stride=17)
    assert list(st) == [2, 2, 0, 0, 0]
    assert np.isnan(out[0, :3]).all() and np.isnan(out[1, :4]).all()
    for f in (2, 3, 4):
        lo, hi = bf.offsets[f], bf.offsets[f + 1]
        r = c_oracle.cheb_fit(bf.x[lo:hi], bf.y[lo:hi], int(degrees[f]))
        assert np.array_equal(out[f, : degrees[f] + 1], r["c"])


def test_cheb_range_maps_extent_onto_unit_interval():
    rng = np.random.default_rng(5)
    for lo, hi in [(-1.0, 1.0), (1000.0, 1001.0), (-7.25, 3.5), (0.0, 1e-3)]:
        x = rng.uniform(lo, hi, 1000).astype(np.float32)
        x[[3, 17]] = [np.nan, np.inf]                 # skipped
        c, s = cheb.cheb_range(x)
        f = x[np.isfinite(x)].astype(np.float64)
        assert (f.min() - c) / s == -1.0 and (f.max() - c) / s == 1.0
    assert cheb.cheb_range(np.full(5, 2.5)) == (2.5, 1.0)
    assert cheb.cheb_range(np.array([np.nan, np.inf])) == (0.0, 1.0)


def test_cheb_derivative_values_closed_form():
    """T_j'(cos th) = j sin(j th) / sin(th)."""
    th = np.linspace(0.1, 3.0, 23)
    dT = cheb.cheb_derivative_values(np.cos(th), 9)
    for j in range(10):
        assert np.allclose(dT[j], j * np.sin(j * th) / np.sin(th), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("m", [1, 4, 9])
def test_cheb_gradients_against_autograd(m):
    """The closed-form adjoint equals torch's float64 reverse mode through the
    fit's definition (Gram matrix V^T V, right side V^T y, linear solve)."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(20 + m)
    n = 300
    x = rng.uniform(-2.0, 3.0, n)
    y = np.cos(x) + 0.1 * rng.standard_normal(n)
    gbar = rng.standard_normal(m + 1)
    c0, s0 = 0.5, 2.5
    got = cheb.cheb_gradients(x, y, m, gbar, c0, s0)
    xt = torch.tensor(x, dtype=torch.float64, requires_grad=True)
    yt = torch.tensor(y, dtype=torch.float64, requires_grad=True)
    t = (xt - c0) / s0
    cols = [torch.ones_like(t), t]
    for k in range(1, m):
        cols.append(2 * t * cols[k] - cols[k - 1])
    V = torch.stack(cols[: m + 1], dim=1)
    c = torch.linalg.solve(V.T @ V, V.T @ yt)
    (c @ torch.tensor(gbar, dtype=torch.float64)).backward()
    assert np.allclose(got["c"], c.detach().numpy(), rtol=1e-10, atol=1e-12)
    for g, ref in ((got["gx"], xt.grad.numpy()), (got["gy"], yt.grad.numpy())):
        assert np.max(np.abs(g - ref)) <= 1e-9 * np.max(np.abs(ref))


def test_cheb_gradients_against_finite_differences():
    """Central differences of L(c(x, y)) on a few inputs."""
    rng = np.random.default_rng(31)
    n, m = 120, 6
    x = rng.uniform(-1.0, 1.0, n)
    y = x ** 3 - x + 0.05 * rng.standard_normal(n)
    gbar = rng.standard_normal(m + 1)
    got = cheb.cheb_gradients(x, y, m, gbar)

    def loss(xx, yy):
        return float(np.dot(gbar, cheb.fit_cheb(xx, yy, m)["c"]))
    h = 1e-6
    for i in (0, 17, 63, 119):
        for arr, g in ((x, got["gx"]), (y, got["gy"])):
            up, dn = arr.copy(), arr.copy()
            up[i] += h
            dn[i] -= h
            num = (loss(up, y) - loss(dn, y)) / (2 * h) if arr is x else (loss(x, up) - loss(x, dn)) / (2 * h)
            assert abs(num - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, num, g[i])
