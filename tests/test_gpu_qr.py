"""GPU parity of the streaming QR route (fit_qr) against the oracle's
Householder QR (the comparator of Sec. III, in its tall-skinny tree form).

Both are backward-stable least-squares solvers, so their difference is
bounded by the perturbation bound of the problem:
    |db| / |b| <= C eps (kappa + kappa^2 eta),  eta = |r| / (|V| |b|),
with kappa = cond(V) of the t-basis Vandermonde matrix, r the residual and
C = 1e3 (row updates per lane, the merge tree and the change of basis).  The
gate is that bound, and never looser than 1e-9 normwise where it is smaller.
The same bound makes the QR route usable where the power sums are not: on
[0, 1] without centring at m = 8, cond(V)^2 ~ 1e13.
"""
import numpy as np
import pytest

from gpu_common import announce, normwise, to_dev, torch
from oracle import c_oracle, fp64, qr
from paper_1512_08017_amd import workloads as W

pytestmark = pytest.mark.gpu

lf = pytest.importorskip("paper_1512_08017_amd")
EPS = np.finfo(np.float64).eps


def qr_bound(x, y, m, c, s, b_ref):
    V = qr.vandermonde(x, m, c, s)
    sv = np.linalg.svd(V, compute_uv=False)
    kappa = sv[0] / sv[-1]
    r = np.asarray(y, np.float64) - V @ b_ref
    eta = np.linalg.norm(r) / (sv[0] * np.linalg.norm(b_ref))
    return max(1e-9, 1e3 * EPS * (kappa + kappa * kappa * eta)), kappa


def run(x, y, m, **kw):
    res = lf.fit_qr(to_dev(x), to_dev(y), m, **kw)
    torch.cuda.synchronize()
    return res


@pytest.mark.parametrize("m", range(1, 9))
def test_every_degree_given_range(m):
    announce(f"qr m={m} given range")
    wl = W.random_small(60_007, m, seed=800 + m, dtype=np.float64)
    res = run(wl.x, wl.y, m, center=0.0, scale=1.0)
    b_ref = qr.lstsq_qr(wl.x, wl.y, m, 0.0, 1.0)
    tol, kappa = qr_bound(wl.x, wl.y, m, 0.0, 1.0, b_ref)
    assert int(res.status.cpu()[0]) == 0
    e = normwise(res.coef_t.cpu().numpy(), b_ref)
    announce(f"  t-basis error {e:.2e} (gate {tol:.1e}, cond(V) {kappa:.1e})")
    assert e <= tol
    assert res.center == 0.0 and res.scale == 1.0


# A lane takes the first-column reciprocal of a data row from a 1024-entry
# table while its factor holds fewer rows, and computes it past that.  On a
# 64-wave grid (4,096 lanes) these sizes give every lane about 1,000 and about
# 1,150 rows: the lanes cross the table's end inside the sweep, at degrees 3 and 8.
@pytest.mark.parametrize("m,rows", [(3, 1000), (3, 1150), (8, 1150)])
def test_rows_past_reciprocal_table(m, rows):
    n = 4096 * rows + 7
    announce(f"qr m={m}: n={n} on 64 waves ({rows} rows per lane)")
    wl = W.random_small(n + 1, m, seed=870 + m + rows, dtype=np.float32)
    x, y = wl.x[1:], wl.y[1:]
    old = lf.default_schedule().as_dict()
    try:
        lf.set_default_schedule({"waves": 64, "waves_per_block": 1, "tile": 2048, "unroll": 1})
        res = lf.fit_qr(to_dev(wl.x)[1:], to_dev(wl.y)[1:], m, center=0.0, scale=1.0)
        torch.cuda.synchronize()
    finally:
        lf.set_default_schedule(old)
    b_ref = qr.lstsq_qr(x, y, m, 0.0, 1.0)
    tol, kappa = qr_bound(x, y, m, 0.0, 1.0, b_ref)
    assert int(res.status.cpu()[0]) == 0
    e = normwise(res.coef_t.cpu().numpy(), b_ref)
    announce(f"  t-basis error {e:.2e} (gate {tol:.1e}, cond(V) {kappa:.1e})")
    assert e <= tol


@pytest.mark.parametrize("n,dtype", [(2, np.float64), (9, np.float64), (4097, np.float32), (1_000_003, np.float32)])
def test_sizes_automatic_range(n, dtype):
    m = 1 if n < 4 else 3
    announce(f"qr n={n} {np.dtype(dtype).name} m={m}")
    wl = W.random_small(n, m, seed=n, dtype=dtype, lo=-3.0, hi=5.0)
    res = run(wl.x, wl.y, m)
    ref = c_oracle.fit(wl.x, wl.y, m)
    assert int(res.status.cpu()[0]) == 0
    assert normwise(res.coef.cpu().numpy(), ref["a"]) <= 1e-9


def test_ill_conditioned_where_power_sums_fail():
    """x on [0, 1] with c = 0, s = 1 (no centring), m = 8, nearly noiseless
    (cond(V) ~ 7e5, so cond(V)^2 eps ~ 1e-4): the QR route stays inside its
    bound, the power sums lose about cond(V) times more."""
    m = 8
    wl = W.random_small(200_003, m, seed=900, dtype=np.float64, lo=0.0, hi=1.0, noise_sd=1e-9)
    res = run(wl.x, wl.y, m, center=0.0, scale=1.0)
    mom = lf.fit(to_dev(wl.x), to_dev(wl.y), m, center=0.0, scale=1.0)
    torch.cuda.synchronize()
    b_ref = qr.lstsq_qr(wl.x, wl.y, m, 0.0, 1.0)
    tol, kappa = qr_bound(wl.x, wl.y, m, 0.0, 1.0, b_ref)
    e_qr = normwise(res.coef_t.cpu().numpy(), b_ref)
    e_mom = normwise(mom.coef_t.cpu().numpy(), b_ref)
    announce(f"  cond(V) {kappa:.1e}: QR route {e_qr:.2e} (gate {tol:.1e}), power sums {e_mom:.2e}")
    assert int(res.status.cpu()[0]) == 0
    assert e_qr <= tol
    assert e_qr * 100 < e_mom


def test_residual_sum_of_squares():
    m = 4
    wl = W.random_small(123_457, m, seed=901, dtype=np.float32, lo=-2.0, hi=2.0)
    x, y = to_dev(wl.x), to_dev(wl.y)
    res = lf.fit_qr(x, y, m)
    sse_pass, _ = lf.residuals(x, y, res)
    torch.cuda.synchronize()
    ref = c_oracle.fit(wl.x, wl.y, m)
    sse_ref = fp64.sse(wl.x, wl.y, ref["a"])
    assert abs(res.sse - sse_ref) <= 1e-9 * sse_ref
    assert abs(float(sse_pass.cpu()[0]) - sse_ref) <= 1e-9 * sse_ref


def test_degenerate_inputs():
    x = to_dev(np.full(50, 0.25))
    y = to_dev(np.linspace(0.0, 1.0, 50))
    r = lf.fit_qr(x, y, 2)
    torch.cuda.synchronize()
    assert int(r.status.cpu()[0]) == 2 and np.isnan(r.coef.cpu().numpy()).all()
    wl = W.random_small(1000, 3, seed=902, dtype=np.float64)
    yb = wl.y.copy()
    yb[500] = np.nan
    r = lf.fit_qr(to_dev(wl.x), to_dev(yb), 3)
    torch.cuda.synchronize()
    assert int(r.status.cpu()[0]) == 3 and np.isnan(r.coef.cpu().numpy()).all()
    # exactly determined: m + 1 distinct points are interpolated
    xi = np.array([-1.0, -0.25, 0.5, 1.0])
    yi = np.array([2.0, -1.0, 0.5, 3.0])
    r = lf.fit_qr(to_dev(xi), to_dev(yi), 3, center=0.0, scale=1.0)
    torch.cuda.synchronize()
    a = r.coef.cpu().numpy()
    assert int(r.status.cpu()[0]) == 0
    assert np.max(np.abs(np.polynomial.polynomial.polyval(xi, a) - yi)) <= 1e-12


def test_misaligned_and_reproducible():
    wl = W.random_small(300_001, 3, seed=903, dtype=np.float32)
    x, y = to_dev(wl.x), to_dev(wl.y)
    ref = c_oracle.fit(wl.x[1:], wl.y[1:], 3)
    r1 = lf.fit_qr(x[1:], y[1:], 3)
    r2 = lf.fit_qr(x[1:], y[1:], 3)
    r3 = lf.fit_qr(x[1:], y[:-1], 3)   # x and y misaligned differently: scalar loads
    torch.cuda.synchronize()
    assert normwise(r1.coef.cpu().numpy(), ref["a"]) <= 1e-9
    assert np.array_equal(r1.coef.cpu().numpy(), r2.coef.cpu().numpy())
    ref3 = c_oracle.fit(wl.x[1:], wl.y[:-1], 3)
    assert normwise(r3.coef.cpu().numpy(), ref3["a"]) <= 1e-9


# ---------------------------------------------------------------------------
# batches (fit_qr_batched)
# ---------------------------------------------------------------------------
RAGGED = [0, 1, 2, 5, 9, 17, 63, 64, 65, 255, 257, 1000, 4097, 70_001, 0, 30_000, 12_345, 40]


@pytest.mark.parametrize("maxdeg,dtype", [(3, np.float32), (8, np.float64), (6, np.float32)])
def test_batched_given_range_against_householder(maxdeg, dtype):
    """t = x / 8 for every fit (given range), so b_k = 8^k a_k exactly; each
    fit's b against the oracle's Householder QR, gated by its own bound."""
    announce(f"qr batched maxdeg={maxdeg} {np.dtype(dtype).name}")
    rng = np.random.default_rng(20 + maxdeg)
    deg = rng.integers(1, maxdeg + 1, len(RAGGED)).astype(np.int32)
    bf = W.random_batch(RAGGED, deg, seed=21 + maxdeg, lo=-5.0, hi=5.0, dtype=dtype)
    coef, status, sse, _ = lf.fit_qr_batched(to_dev(bf.x), to_dev(bf.y), to_dev(bf.offsets), to_dev(bf.degrees),
                                             maxdeg, center=0.0, scale=8.0)
    torch.cuda.synchronize()
    coef, status, sse = coef.cpu().numpy(), status.cpu().numpy(), sse.cpu().numpy()
    for f in range(bf.batch):
        m = int(bf.degrees[f])
        lo, hi = bf.offsets[f], bf.offsets[f + 1]
        if hi - lo < m + 1:
            assert status[f] == 2 and np.isnan(coef[f, : m + 1]).all() and np.isnan(sse[f])
            continue
        assert status[f] == 0, (f, status[f])
        xf, yf = bf.x[lo:hi].astype(np.float64), bf.y[lo:hi].astype(np.float64)
        b_ref = qr.lstsq_qr(xf, yf, m, 0.0, 8.0)
        tol, kappa = qr_bound(xf, yf, m, 0.0, 8.0, b_ref)
        b_gpu = coef[f, : m + 1] * 8.0 ** np.arange(m + 1)
        e = normwise(b_gpu, b_ref)
        assert e <= tol, (f, m, hi - lo, e, tol, kappa)
        r = yf - qr.vandermonde(xf, m, 0.0, 8.0) @ b_ref
        ssr = float(r @ r)
        assert abs(sse[f] - ssr) <= 1e-9 * max(ssr, 1e-300) + 1e3 * EPS * float(yf @ yf), (f, sse[f], ssr)


def test_batched_automatic_range_and_residual_pass():
    rng = np.random.default_rng(30)
    lengths = rng.integers(50, 20_000, 300)
    deg = rng.integers(1, 4, 300).astype(np.int32)
    bf = W.random_batch(lengths, deg, seed=31, lo=-5.0, hi=5.0)
    x, y, off, dg = to_dev(bf.x), to_dev(bf.y), to_dev(bf.offsets), to_dev(bf.degrees)
    coef, status, sse, ws = lf.fit_qr_batched(x, y, off, dg, 3)
    sse_pass, _ = lf.residuals_batched(x, y, off, dg, 3, ws=ws)
    torch.cuda.synchronize()
    ref, rst = c_oracle.fit_batched(bf.x, bf.y, bf.offsets, bf.degrees, stride=4)
    coef, status, sse, sse_pass = coef.cpu().numpy(), status.cpu().numpy(), sse.cpu().numpy(), sse_pass.cpu().numpy()
    assert (status == 0).all() and (rst == 0).all()
    for f in range(bf.batch):
        m = int(bf.degrees[f])
        assert normwise(coef[f, : m + 1], ref[f, : m + 1]) <= 1e-9
    assert np.max(np.abs(sse - sse_pass) / sse_pass) <= 1e-9


def test_batched_degenerate_fits_stay_local():
    bf = W.random_batch([100, 100, 100, 100], [3, 0, 9, 2], seed=32)
    y = bf.y.copy()
    y[350] = np.nan                      # inside the fourth fit
    coef, status, sse, _ = lf.fit_qr_batched(to_dev(bf.x), to_dev(y), to_dev(bf.offsets), to_dev(bf.degrees), 8,
                                             coef_stride=9)
    torch.cuda.synchronize()
    coef, status = coef.cpu().numpy(), status.cpu().numpy()
    assert list(status) == [0, 1, 1, 3]
    assert np.isnan(coef[1]).all() and np.isnan(coef[2]).all() and np.isnan(coef[3, :3]).all()
    ref = c_oracle.fit(bf.x[:100], bf.y[:100], 3)
    assert normwise(coef[0, :4], ref["a"]) <= 1e-9
