"""GPU parity of the single-fit path (fit_moments + fit_solve) against the oracle.

Sizes span several tiles and a ragged tail; both the float64 and the
compensated-float32 forms, both range modes, every degree up to the maximum,
odd alignments and the degenerate cases.  Gates: float64 form <= 1e-9 and
compensated float32 form with one refinement <= 1e-6, normwise relative to
the oracle's coefficients; power sums <= 1e-12 relative per sum.
"""
import ctypes

import numpy as np
import pytest

from gpu_common import announce, normwise, to_dev, torch
from oracle import adjoint, c_oracle, fp64
from paper_1512_08017_amd import _lib, api, workloads as W

pytestmark = pytest.mark.gpu

lf = pytest.importorskip("paper_1512_08017_amd")


def run_fit(fit, degree, precision="f64", **kw):
    x, y = to_dev(fit.x), to_dev(fit.y)
    res = lf.fit(x, y, degree, precision=precision, **kw)
    torch.cuda.synchronize()
    return res


@pytest.mark.parametrize("n", [2, 3, 5, 63, 64, 65, 255, 257, 1000, 4097, 65_537, 1_000_003])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_f64_form_sizes(n, dtype):
    m = 1 if n < 4 else 3
    announce(f"f64 form n={n} dtype={np.dtype(dtype).name} m={m}")
    fit = W.random_small(n, m, seed=n, dtype=dtype)
    res = run_fit(fit, m)
    ref = c_oracle.fit(fit.x, fit.y, m)
    assert int(res.status.cpu()[0]) == 0
    assert normwise(res.coef.cpu().numpy(), ref["a"]) <= 1e-9


# block counts of the streaming grid: 16 (fewer than a wave's lanes); 64; 500
# (a partial chunk of the finish's 512 blocks per round); 1,024; 8,192
# (sixteen rounds)
SINGLE_SCHEDULES = [
    {"waves": 64, "waves_per_block": 4, "tile": 2048, "unroll": 2},
    {"waves": 64, "waves_per_block": 1, "tile": 2048, "unroll": 1},
    {"waves": 1000, "waves_per_block": 2, "tile": 2048, "unroll": 2},
    {"waves": 4096, "waves_per_block": 4, "tile": 2048, "unroll": 4},
    {"waves": 8192, "waves_per_block": 1, "tile": 2048, "unroll": 2},
]


@pytest.mark.parametrize("schedule", SINGLE_SCHEDULES)
@pytest.mark.parametrize("m,precision", [(3, "f64"), (3, "f32c"), (8, "f64")])
def test_single_fit_under_schedules(schedule, m, precision):
    """The finish adds the block partials of any grid: a few blocks, a partial
    round, several rounds; each against the oracle and with its power sums."""
    announce(f"single fit m={m} {precision} under {schedule}")
    fit = W.random_small(2_000_003, m, seed=300 + m, lo=-1.0, hi=1.0, dtype=np.float32)
    old = lf.default_schedule().as_dict()
    try:
        lf.set_default_schedule(schedule)
        res = run_fit(fit, m, precision=precision, center=0.0, scale=1.0)
    finally:
        lf.set_default_schedule(old)
    ref = c_oracle.fit(fit.x, fit.y, m, center=0.0, scale=1.0)
    assert int(res.status.cpu()[0]) == 0
    mom = res.moments.cpu().numpy()
    S = mom[2:3 + 2 * m]
    assert S[0] == fit.n
    if precision == "f64":
        T = mom[3 + 2 * m:]
        assert np.max(np.abs(S - ref["S"]) / np.abs(ref["S"]).max()) <= 1e-12
        assert np.max(np.abs(T - ref["T"]) / np.abs(ref["T"]).max()) <= 1e-12
    tol = (1e-9 if m <= 5 else 1e-7) if precision == "f64" else 1e-6
    assert normwise(res.coef_t.cpu().numpy(), ref["b"]) <= tol


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6, 7, 8])
def test_every_degree_given_range(m):
    """Given (c, s): compare power sums and t-basis solution in the same basis."""
    announce(f"degree {m} given range")
    fit = W.random_small(200_001, m, seed=100 + m, lo=2.0, hi=4.0, dtype=np.float32)
    c, s = 3.0, 1.0
    res = run_fit(fit, m, center=c, scale=s)
    ref = c_oracle.fit(fit.x, fit.y, m, center=c, scale=s)
    mom = res.moments.cpu().numpy()
    assert mom[0] == c and mom[1] == s
    S, T = mom[2:3 + 2 * m], mom[3 + 2 * m:]
    assert S[0] == fit.n
    assert np.max(np.abs(S - ref["S"]) / np.abs(ref["S"]).max()) <= 1e-12
    assert np.max(np.abs(T - ref["T"]) / np.abs(ref["T"]).max()) <= 1e-12
    assert int(res.status.cpu()[0]) == 0
    # cond of the monomial Hankel matrix grows quickly with m: the gate follows it
    tol = 1e-9 if m <= 5 else 1e-7
    assert normwise(res.coef_t.cpu().numpy(), ref["b"]) <= tol
    # a = M b amplifies a relative error of b by kappa = max|M||b| / max|a|
    Mx = adjoint.basis_map(m, c, s)
    kappa = np.max(np.abs(Mx) @ np.abs(ref["b"])) / np.max(np.abs(ref["a"]))
    assert normwise(res.coef.cpu().numpy(), ref["a"]) <= tol * max(1.0, kappa)


@pytest.mark.parametrize("m", [1, 3, 5])
def test_auto_range_matches_plain_minimiser(m):
    announce(f"auto range m={m}")
    fit = W.random_small(300_007, m, seed=200 + m, lo=-3.0, hi=7.0, dtype=np.float32)
    res = run_fit(fit, m)
    mom = res.moments.cpu().numpy()
    # the auto range is a power-of-two scale and a float32 centre
    assert np.log2(mom[1]) == np.round(np.log2(mom[1]))
    assert float(np.float32(mom[0])) == mom[0]
    ref = c_oracle.fit(fit.x, fit.y, m, center=2.0, scale=4.0)
    assert normwise(res.coef.cpu().numpy(), ref["a"]) <= 1e-9


@pytest.mark.parametrize("n", [5, 1000, 65_536, 1_000_001])
@pytest.mark.parametrize("m", [1, 3, 5])
def test_f32c_form_with_refinement(n, m):
    announce(f"f32c n={n} m={m}")
    fit = W.random_small(n, m, seed=300 + n + m, lo=-1.0, hi=1.0, noise_sd=0.01, dtype=np.float32)
    if n < m + 1:
        # fewer points than coefficients: rejected on the host, nothing launched
        with pytest.raises(lf.LsefitError):
            run_fit(fit, m, precision="f32c", refine=1)
        return
    res = run_fit(fit, m, precision="f32c", refine=1)
    ref = c_oracle.fit(fit.x, fit.y, m)
    assert int(res.status.cpu()[0]) == 0
    assert normwise(res.coef.cpu().numpy(), ref["a"]) <= 1e-6


def test_f32c_without_refinement_is_close():
    fit = W.random_small(1_000_000, 3, seed=41, dtype=np.float32)
    res = run_fit(fit, 3, precision="f32c", refine=0)
    ref = c_oracle.fit(fit.x, fit.y, 3)
    assert normwise(res.coef.cpu().numpy(), ref["a"]) <= 1e-4


def test_bitwise_deterministic():
    fit = W.random_small(3_000_017, 3, seed=42, dtype=np.float32)
    x, y = to_dev(fit.x), to_dev(fit.y)
    for prec in ("f64", "f32c"):
        outs = []
        for _ in range(3):
            r = lf.fit(x, y, 3, precision=prec)
            torch.cuda.synchronize()
            outs.append((r.coef.cpu().numpy().tobytes(), r.moments.cpu().numpy().tobytes()))
        assert outs[0] == outs[1] == outs[2], prec


@pytest.mark.parametrize("shift_x,shift_y", [(1, 1), (2, 2), (3, 3), (1, 2), (0, 3)])
def test_misaligned_pointers(shift_x, shift_y):
    """Slices that start off the 16-byte grid (same or different offsets for x and y)."""
    announce(f"misaligned {shift_x} {shift_y}")
    fit = W.random_small(100_003, 3, seed=43, dtype=np.float32)
    xf = np.concatenate([np.zeros(4, np.float32), fit.x])
    yf = np.concatenate([np.zeros(4, np.float32), fit.y])
    n = fit.n - 4
    xh, yh = xf[shift_x:shift_x + n], yf[shift_y:shift_y + n]
    x = to_dev(xf)[shift_x:shift_x + n]
    y = to_dev(yf)[shift_y:shift_y + n]
    assert x.is_contiguous() and y.is_contiguous()
    res = lf.fit(x, y, 3)
    torch.cuda.synchronize()
    ref = c_oracle.fit(xh, yh, 3)
    assert normwise(res.coef.cpu().numpy(), ref["a"]) <= 1e-9


def test_duplicate_x_is_singular():
    x = np.repeat(np.array([1.0, 2.0, 3.0], np.float32), 1000)
    y = np.random.default_rng(0).standard_normal(3000).astype(np.float32)
    for m, expect in ((2, 0), (3, 2), (4, 2)):
        res = lf.fit(to_dev(x), to_dev(y), m)
        torch.cuda.synchronize()
        assert int(res.status.cpu()[0]) == expect, m
        assert fp64.fit(x, y, m)["status"] == ("ok" if expect == 0 else "singular")
        if expect:
            assert torch.isnan(res.coef).all()


@pytest.mark.parametrize("where", ["x", "y"])
@pytest.mark.parametrize("value", [np.nan, np.inf])
def test_nonfinite_input(where, value):
    fit = W.random_small(10_000, 2, seed=44, dtype=np.float32)
    getattr(fit, where)[1234] = value
    for prec in ("f64", "f32c"):
        res = run_fit(fit, 2, precision=prec, center=0.0, scale=1.0)
        assert int(res.status.cpu()[0]) == 3
        assert torch.isnan(res.coef).all()


def test_constant_x_auto_range():
    x = np.full(1000, 5.0, np.float32)
    y = np.arange(1000, dtype=np.float32)
    res = run_fit(W.SingleFit("c", x, y, 1, np.zeros(2)), 1)
    assert int(res.status.cpu()[0]) == 2


def test_minimum_points_interpolates():
    """n = m + 1 distinct points: zero residual (interpolation)."""
    x = np.array([-1.0, -0.25, 0.5, 1.0], np.float64)
    y = np.array([2.0, -1.0, 0.5, 3.0], np.float64)
    res = run_fit(W.SingleFit("i", x, y, 3, np.zeros(4)), 3)
    a = res.coef.cpu().numpy()
    assert np.max(np.abs(fp64.polyval(a, x) - y)) <= 1e-12


def test_host_errors_raise():
    x = to_dev(np.zeros(3, np.float32))
    with pytest.raises(lf.LsefitError):
        lf.fit(x, x, 3)                       # n < m + 1
    with pytest.raises(lf.LsefitError):
        lf.fit(x.double(), x.double(), 1, precision="f32c")   # unsupported
    with pytest.raises((lf.LsefitError, ValueError)):
        lf.fit(to_dev(np.zeros(100, np.float32)), to_dev(np.zeros(100, np.float32)), 9)


def test_c_abi_workspace_check_on_device():
    from paper_1512_08017_amd import _lib, api
    L = _lib.load()
    x = to_dev(np.zeros(100, np.float32))
    ws = torch.empty(64, dtype=torch.uint8, device=x.device)
    mom = torch.empty(13, dtype=torch.float64, device=x.device)
    o = api.options(3)
    rc = L.fit_moments(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(x.data_ptr()), 100, _lib.F32,
                       ctypes.byref(o), ctypes.c_void_p(ws.data_ptr()), 64, ctypes.c_void_p(mom.data_ptr()), None)
    assert rc == _lib.WORKSPACE


def test_linear_f64_workload():
    """The m = 1, n = 1e6 float64 workload (x ~ U[0,10], y = 2 + 3x + noise)."""
    fit = W.linear_f64()
    res = run_fit(fit, 1)
    ref = c_oracle.fit(fit.x, fit.y, 1)
    assert normwise(res.coef.cpu().numpy(), ref["a"]) <= 1e-9
    assert abs(res.coef.cpu().numpy()[1] - 3.0) < 1e-2


@pytest.mark.parametrize("precision", ["f64", "f32c"])
def test_split_calls_match_fused_call(precision):
    """fit_moments + fit_solve and the fused fit_single give the same numbers."""
    fit = W.random_small(500_009, 3, seed=45, dtype=np.float32)
    x, y = to_dev(fit.x), to_dev(fit.y)
    fused = lf.fit(x, y, 3, precision=precision)
    split = lf.fit_split(x, y, 3, precision=precision)
    torch.cuda.synchronize()
    assert np.array_equal(fused.moments.cpu().numpy(), split.moments.cpu().numpy())
    assert normwise(fused.coef.cpu().numpy(), split.coef.cpu().numpy()) <= 1e-13
    assert int(fused.status.cpu()[0]) == int(split.status.cpu()[0]) == 0


@pytest.mark.parametrize("solver", ["gepp", "cholesky"])
@pytest.mark.parametrize("m", range(1, 9))
def test_finish_forms_match_the_one_thread_solve(m, solver):
    """The fused call's finish solves in registers by one lane up to degree 4
    and by a wave, a row per lane, above it; fit_solve solves by one thread.
    All do the same operations in the same order, so on the same power sums
    (equal bit for bit) the coefficients in both bases are equal bit for bit."""
    fit = W.random_small(200_003, m, seed=70 + m, dtype=np.float32)
    x, y = to_dev(fit.x), to_dev(fit.y)
    fused = lf.fit(x, y, m, solver=solver)
    split = lf.fit_split(x, y, m, solver=solver)
    torch.cuda.synchronize()
    st = int(fused.status.cpu()[0])
    assert st == int(split.status.cpu()[0]) and (st == 0 or solver == "cholesky")
    assert np.array_equal(fused.moments.cpu().numpy(), split.moments.cpu().numpy())
    assert np.array_equal(fused.coef.cpu().numpy(), split.coef.cpu().numpy(), equal_nan=True)
    assert np.array_equal(fused.coef_t.cpu().numpy(), split.coef_t.cpu().numpy(), equal_nan=True)


def test_reuse_across_calls_and_workspaces():
    """Nothing in the workspace has to start at zero: many calls on one
    workspace that first holds arbitrary bytes give identical results."""
    fit = W.random_small(2_000_003, 2, seed=46, dtype=np.float32)
    x, y = to_dev(fit.x), to_dev(fit.y)
    ws = torch.full((lf.workspace_bytes(1, 2),), 0x5A, dtype=torch.uint8, device=x.device)
    first = lf.fit(x, y, 2, ws=ws).coef.cpu().numpy()
    for _ in range(5):
        assert np.array_equal(lf.fit(x, y, 2, ws=ws).coef.cpu().numpy(), first)
    ref = c_oracle.fit(fit.x, fit.y, 2)
    assert normwise(first, ref["a"]) <= 1e-9


# --- Cholesky solver and the residual pass -------------------------------------

@pytest.mark.parametrize("m", [1, 3, 5, 8])
@pytest.mark.parametrize("precision", ["f64", "f32c"])
def test_cholesky_matches_oracle(m, precision):
    fit = W.random_small(300_001, m, seed=500 + m, dtype=np.float32)
    res = run_fit(fit, m, precision=precision, solver="cholesky", center=0.0, scale=1.0)
    ref = c_oracle.fit(fit.x, fit.y, m)
    assert int(res.status.cpu()[0]) == 0
    tol = (1e-9 if m <= 5 else 1e-7) if precision == "f64" else 1e-6
    assert normwise(res.coef_t.cpu().numpy(), ref["b"]) <= tol


def test_cholesky_flags_singular():
    x = np.repeat(np.array([1.0, 2.0, 3.0], np.float32), 100)
    y = np.arange(300, dtype=np.float32)
    assert int(lf.fit(to_dev(x), to_dev(y), 3, solver="cholesky").status.cpu()[0]) == 2
    assert int(lf.fit(to_dev(x), to_dev(y), 2, solver="cholesky").status.cpu()[0]) == 0


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_residuals_single(dtype):
    fit = W.random_small(1_000_003, 3, seed=510, dtype=dtype)
    x, y = to_dev(fit.x), to_dev(fit.y)
    res = lf.fit(x, y, 3)
    sse, e = lf.residuals(x, y, res, store=True)
    torch.cuda.synchronize()
    a = c_oracle.fit(fit.x, fit.y, 3)["a"]
    sse_ref = fp64.sse(fit.x, fit.y, a)
    assert abs(float(sse.cpu()[0]) - sse_ref) <= 1e-10 * sse_ref
    e_ref = fit.y.astype(np.float64) - fp64.polyval(a, fit.x)
    assert np.max(np.abs(e.cpu().numpy().astype(np.float64) - e_ref)) <= 1e-6 * np.max(np.abs(e_ref)) + (
        0 if dtype == np.float64 else 1e-7 * np.max(np.abs(e_ref)))


def test_residuals_table_v():
    """Table V (Sec. III): the sum of squared errors of the order-3 fit of Table I
    is the exact minimum 128.19957537..., below the printed 128.199937."""
    from conftest import read_golden
    rows, notes = read_golden("table_i.txt")
    x = np.array([float(r[0]) for r in rows])
    y = np.array([float(r[1]) for r in rows])
    xd, yd = to_dev(x), to_dev(y)
    res = lf.fit(xd, yd, 3)
    sse, e = lf.residuals(xd, yd, res, store=True)
    torch.cuda.synchronize()
    from oracle import exact
    a_ex, _ = exact.fit_exact(x, y, 3)
    sse_exact = float(exact.sse_exact(x, y, a_ex))
    _, tv = read_golden("table_v.txt")
    s = float(sse.cpu()[0])
    assert abs(s - sse_exact) <= 1e-9 * sse_exact
    assert s <= tv["sum_e_f2"] and s <= tv["sum_e_p2"]
    # the residuals themselves (e = y - f(x)) against the exact fitted values
    fe = np.array([float(exact.polyval_exact(a_ex, xv)) for xv in x])
    assert np.max(np.abs(e.cpu().numpy() - (y - fe))) <= 1e-8


# --- streams, graph capture and long runs of single fits --------------------------

def test_single_fits_on_several_streams():
    """Fits on three streams at once, each with its own workspace: each result
    equals the same fit run alone, bit for bit."""
    fits = [W.random_small(n, 3, seed=s, dtype=np.float32) for n, s in ((3_000_001, 61), (700_003, 62),
                                                                          (5_000_011, 63))]
    data = [(to_dev(f.x), to_dev(f.y)) for f in fits]
    alone = []
    for x, y in data:
        r = lf.fit(x, y, 3)
        torch.cuda.synchronize()
        alone.append(r.coef.cpu().numpy())
    streams = [torch.cuda.Stream() for _ in data]
    outs = []
    for _ in range(3):
        res = []
        for (x, y), s in zip(data, streams):
            with torch.cuda.stream(s):
                res.append(lf.fit(x, y, 3))
        torch.cuda.synchronize()
        outs.append([r.coef.cpu().numpy() for r in res])
    for rep in outs:
        for got, ref in zip(rep, alone):
            assert np.array_equal(got, ref)
    for f, ref in zip(fits, alone):
        assert normwise(ref[:4], c_oracle.fit(f.x, f.y, 3)["a"]) <= 1e-9


@pytest.mark.parametrize("precision", ["f64", "f32c"])
def test_captured_single_fit_matches_eager(precision):
    """fit_single captured into a HIP graph: replays, with eager calls between
    them, give the eager bits."""
    fit = W.random_small(1_500_007, 3, seed=64, dtype=np.float32)
    x, y = to_dev(fit.x), to_dev(fit.y)
    L = _lib.load()
    vp = ctypes.c_void_p
    opt = api.options(3, precision, 1)
    ws = torch.zeros(api.workspace_bytes(1, 3), dtype=torch.uint8, device=x.device)
    coef = torch.zeros(8, dtype=torch.float64, device=x.device)
    status = torch.zeros(1, dtype=torch.int32, device=x.device)
    er = lf.fit(x, y, 3, precision=precision)
    torch.cuda.synchronize()
    eager = np.concatenate([er.coef.cpu().numpy(), er.coef_t.cpu().numpy()])   # a, then b
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        args = (vp(x.data_ptr()), vp(y.data_ptr()), x.numel(), _lib.F32, ctypes.byref(opt), vp(ws.data_ptr()),
                ws.numel(), vp(coef.data_ptr()), vp(status.data_ptr()), None, vp(s.cuda_stream))
        _lib.check(L.fit_single(*args), "fit_single")     # eager call on the capture stream first
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=s):
            _lib.check(L.fit_single(*args), "fit_single")
    for i in range(3):
        coef.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(coef.cpu().numpy(), eager), i
        assert int(status.cpu()[0]) == 0
        lf.fit(x, y, 3, precision=precision)                  # eager work between replays
        torch.cuda.synchronize()


def test_single_fit_stress_against_split():
    """Many fits in a row of changing size and degree on one stream: fit_single
    gives, every time, the power sums of fit_moments bit for bit."""
    rng = np.random.default_rng(65)
    base = W.random_small(4_000_037, 4, seed=65, dtype=np.float32)
    x, y = to_dev(base.x), to_dev(base.y)
    for i in range(120):
        n = int(rng.integers(50_000, 4_000_037))
        m = int(rng.integers(1, 5))
        xs, ys = x[:n], y[:n]
        fused = lf.fit(xs, ys, m)
        split_mom, _ = lf.fit_moments(xs, ys, m)
        torch.cuda.synchronize()
        assert int(fused.status.cpu()[0]) == 0, i
        assert np.array_equal(fused.moments.cpu().numpy(), split_mom.cpu().numpy()), (i, n, m)
