"""GPU parity of the batched path (one persistent launch over CSR segments)
and of the adjoint, against the oracle."""
import numpy as np
import pytest

from gpu_common import announce, normwise, to_dev, torch
from oracle import adjoint, c_oracle
from paper_1512_08017_amd import workloads as W

pytestmark = pytest.mark.gpu

lf = pytest.importorskip("paper_1512_08017_amd")


def run_batched(bf, max_degree, precision="f64", plan=None, **kw):
    x, y = to_dev(bf.x), to_dev(bf.y)
    off, deg = to_dev(bf.offsets), to_dev(bf.degrees)
    coef, status, ws = lf.fit_batched(x, y, off, deg, max_degree, precision=precision, plan=plan, **kw)
    torch.cuda.synchronize()
    return coef.cpu().numpy(), status.cpu().numpy()


def check_against_oracle(bf, coef, status, tol):
    ref, rst = c_oracle.fit_batched(bf.x, bf.y, bf.offsets, bf.degrees, stride=coef.shape[1])
    worst = 0.0
    for f in range(bf.batch):
        m = int(bf.degrees[f])
        assert int(status[f]) == int(rst[f]), (f, status[f], rst[f])
        if rst[f] == 0:
            e = normwise(coef[f, : m + 1], ref[f, : m + 1])
            worst = max(worst, e)
        else:
            assert np.isnan(coef[f, : m + 1]).all()
    assert worst <= tol, worst
    return worst


RAGGED = [0, 1, 2, 3, 4, 5, 15, 16, 17, 63, 64, 65, 255, 256, 257, 1000, 4097, 70_001, 0, 7, 300_000, 2, 12_345]


@pytest.mark.parametrize("precision,tol", [("f64", 1e-9), ("f32c", 1e-6)])
def test_ragged_mixed_degrees(precision, tol):
    announce(f"ragged batch {precision}")
    rng = np.random.default_rng(1)
    deg = rng.integers(1, 4, len(RAGGED))
    bf = W.random_batch(RAGGED, deg, seed=2, lo=-5.0, hi=5.0)
    coef, status = run_batched(bf, 3, precision)
    check_against_oracle(bf, coef, status, tol)
    assert status[0] == 2 and status[1] == 2     # empty and one-point fits are singular


@pytest.mark.parametrize("schedule", [
    {"waves": 64, "waves_per_block": 1, "tile": 64, "unroll": 1},
    {"waves": 1024, "waves_per_block": 2, "tile": 512, "unroll": 2},
    {"waves": 4096, "waves_per_block": 4, "tile": 4096, "unroll": 4},
    {"waves": 8192, "waves_per_block": 4, "tile": 256, "unroll": 2},
    {"waves": 2048, "waves_per_block": 2, "tile": 1000, "unroll": 2},   # not a power of two: two plan launches
])
def test_schedules_agree(schedule):
    announce(f"schedule {schedule}")
    rng = np.random.default_rng(3)
    L = W.ragged_lengths(500, 16, 20_000, rng)
    deg = rng.integers(1, 4, 500)
    bf = W.random_batch(L, deg, seed=4, lo=-5.0, hi=5.0)
    old = lf.default_schedule().as_dict()
    try:
        lf.set_default_schedule(schedule)
        coef, status = run_batched(bf, 3)
    finally:
        lf.set_default_schedule(old)
    check_against_oracle(bf, coef, status, 1e-9)


@pytest.mark.parametrize("batch,dtype", [(b, np.float32) for b in (256, 257, 1024, 1025, 2048, 2049, 4096, 4097,
                                                                  8192, 8193)]
                         + [(b, np.float64) for b in (300, 1025, 4097, 8193)])
def test_tile_table_one_launch_and_two(batch, dtype):
    """Up to 32 blocks of 256 fits (8,192) the tile table takes one launch, in
    which every block also counts the tiles before its own, with a loop sized
    for 0, 3, 7, 15 or 31 earlier blocks (each size at its first and last block
    count here); from 8,193 fits on it takes two.  Short fits, some empty and
    some across tile boundaries."""
    announce(f"tile table, {batch} fits, {np.dtype(dtype).name}")
    rng = np.random.default_rng(batch)
    L = rng.integers(0, 600, batch)
    L[::97] = 0
    deg = rng.integers(1, 4, batch)
    bf = W.random_batch(L, deg, seed=batch + 1, lo=-5.0, hi=5.0, dtype=dtype)
    old = lf.default_schedule().as_dict()
    try:
        lf.set_default_schedule({"waves": 4096, "waves_per_block": 2, "tile": 256, "unroll": 2})
        coef, status = run_batched(bf, 3)
    finally:
        lf.set_default_schedule(old)
    check_against_oracle(bf, coef, status, 1e-9)
    assert (status[L < deg + 1] == 2).all()      # too few points (empty fits included)


def _documented_auto_range(xs):
    """(c, s) of a batched fit with the automatic range, as include/lsefit.h
    states the rule: the first 8 and the last 8 points (all of a shorter fit),
    s = 2^ceil(log2(half-range)), c = mid-range rounded to a multiple of s/8 (0
    below 2^-6 half-ranges), then to float32; (0, 1) without a finite sample."""
    import math
    v = xs if xs.size <= 16 else np.concatenate([xs[:8], xs[-8:]])
    v = v.astype(np.float64)
    v = v[np.isfinite(v)]
    if v.size == 0:
        return 0.0, 1.0
    lo, hi = float(v.min()), float(v.max())
    half, mid = 0.5 * hi - 0.5 * lo, 0.5 * hi + 0.5 * lo
    s, c = 1.0, mid
    if half > 0.0:
        fr, e = math.frexp(half)
        s = math.ldexp(1.0, e - 1 if fr == 0.5 else e)
        q = s / 8
        c = 0.0 if abs(mid) < math.ldexp(half, -6) else float(np.rint(mid / q)) * q
    return float(np.float32(c)), s


@pytest.mark.parametrize("batch,dtype", [(300, np.float32), (9000, np.float32), (300, np.float64), (9000, np.float64)])
def test_batched_auto_range_follows_the_documented_rule(batch, dtype):
    """The (c, s) each fit of a batch gets from its own x: bit for bit the
    documented sample rule, with the tile table in one launch (300 fits) and in
    two (9,000 fits), for empty, single-point, short (up to 16 points, all
    sampled) and long fits of unsorted x, a constant fit and fits near zero."""
    announce(f"batched automatic range, {batch} fits, {np.dtype(dtype).name}")
    rng = np.random.default_rng(batch + 7)
    L = rng.integers(0, 40, batch)
    L[::53] = rng.integers(100, 3000, L[::53].size)
    L[:6] = [0, 1, 2, 16, 17, 5000]
    deg = rng.integers(1, 4, batch)
    bf = W.random_batch(L, deg, seed=batch + 11, lo=-7.0, hi=13.0, dtype=dtype)
    # a constant fit and a fit whose mid-range is near zero
    bf.x[bf.offsets[4]:bf.offsets[5]] = dtype(3.25)
    bf.x[bf.offsets[5]:bf.offsets[6]] = np.linspace(-1.0, 1.0001, L[5]).astype(dtype)
    M = 3
    x, y = to_dev(bf.x), to_dev(bf.y)
    off, dg = to_dev(bf.offsets), to_dev(bf.degrees)
    coef, status, _ = lf.fit_batched(x, y, off, dg, M, output_basis="x_and_t")
    torch.cuda.synchronize()
    coef = coef.cpu().numpy()
    for f in range(batch):
        lo, hi = bf.offsets[f], bf.offsets[f + 1]
        c, s = _documented_auto_range(bf.x[lo:hi])
        assert coef[f, 2 * M + 2] == c and coef[f, 2 * M + 3] == s, (f, hi - lo, coef[f, 2 * M + 2:], c, s)


def test_degree_out_of_range_is_flagged():
    bf = W.random_batch([100, 100, 100], [1, 3, 2], seed=5)
    coef, status = run_batched(bf, 2)      # fit 1 asks for more than max_degree
    assert list(status) == [0, 1, 0]
    assert np.isnan(coef[1]).all()         # every entry of an out-of-range fit


def test_decreasing_segment_is_flagged():
    """A fit whose end offset lies before its start (a bad segment) is flagged
    INVALID_ARG with NaN coefficients and no tiles; its neighbours, which then
    overlap in x, are fitted on their own ranges as usual."""
    bf = W.random_batch([2000], [3], seed=41)
    x, y = bf.x, bf.y
    offsets = np.array([0, 1000, 500, 2000], dtype=np.int64)
    degrees = np.array([3, 2, 3], dtype=np.int32)
    coef, status, _ = lf.fit_batched(to_dev(x), to_dev(y), to_dev(offsets), to_dev(degrees), 3)
    torch.cuda.synchronize()
    coef, status = coef.cpu().numpy(), status.cpu().numpy()
    assert list(status) == [0, 1, 0]
    assert np.isnan(coef[1, :3]).all() and coef[1, 3] == 0.0   # its m + 1 coefficients; the row's rest untouched
    # the two valid fits, laid out one after the other for the oracle
    x2 = np.concatenate([x[0:1000], x[500:2000]])
    y2 = np.concatenate([y[0:1000], y[500:2000]])
    ref, rst = c_oracle.fit_batched(x2, y2, np.array([0, 1000, 2500]), np.array([3, 3], dtype=np.int32), stride=4)
    assert list(rst) == [0, 0]
    assert normwise(coef[0], ref[0]) <= 1e-9 and normwise(coef[2], ref[1]) <= 1e-9


def test_nonfinite_fit_does_not_touch_neighbours():
    bf = W.random_batch([1000, 1000, 1000], [2, 2, 2], seed=6)
    bf.y[1500] = np.nan
    coef, status = run_batched(bf, 2)
    assert list(status) == [0, 3, 0]
    ref, _ = c_oracle.fit_batched(bf.x, bf.y, bf.offsets, bf.degrees, stride=3)
    assert normwise(coef[0], ref[0]) <= 1e-9 and normwise(coef[2], ref[2]) <= 1e-9


def test_batched_equals_single_fits():
    bf = W.random_batch([5000, 70_000, 333], [3, 2, 1], seed=7)
    coef, status = run_batched(bf, 3)
    for f in range(3):
        lo, hi = bf.offsets[f], bf.offsets[f + 1]
        m = int(bf.degrees[f])
        r = lf.fit(to_dev(bf.x[lo:hi]), to_dev(bf.y[lo:hi]), m)
        assert normwise(coef[f, : m + 1], r.coef.cpu().numpy()) <= 1e-12


def test_plan_graph_replays_match_eager():
    announce("plan + graph")
    rng = np.random.default_rng(8)
    L = W.ragged_lengths(2000, 16, 30_000, rng)
    deg = rng.integers(1, 4, 2000)
    bf = W.random_batch(L, deg, seed=9, lo=-5.0, hi=5.0)
    x, y = to_dev(bf.x), to_dev(bf.y)
    off, dg = to_dev(bf.offsets), to_dev(bf.degrees)
    eager, est, _ = lf.fit_batched(x, y, off, dg, 3)
    plan = lf.Plan(bf.batch, 3)
    plan.set_graph(True)           # a form set by the caller survives tuning
    best = plan.tune(x, y, off, dg, reps=1)
    assert best > 0 and plan.graph
    coef = torch.zeros_like(eager)
    status = torch.zeros_like(est)
    outs = []
    for _ in range(4):
        coef.zero_()
        lf.fit_batched(x, y, off, dg, 3, plan=plan, out=(coef, status))
        torch.cuda.synchronize()
        outs.append(coef.cpu().numpy().copy())
        _ = (x * 2).sum().item()    # eager work between replays
    for o in outs:
        assert np.array_equal(o, outs[0])
    check_against_oracle(bf, outs[0], status.cpu().numpy(), 1e-9)
    plan.close()


def test_plan_tune_cache(tmp_path):
    announce("plan tune cache")
    rng = np.random.default_rng(12)
    L = W.ragged_lengths(500, 16, 20_000, rng)
    deg = rng.integers(1, 4, 500)
    bf = W.random_batch(L, deg, seed=13, lo=-5.0, hi=5.0)
    x, y = to_dev(bf.x), to_dev(bf.y)
    off, dg = to_dev(bf.offsets), to_dev(bf.degrees)
    cache = tmp_path / "schedules.txt"
    # a miss tunes and appends one line keyed by the call's shape
    p1 = lf.Plan(bf.batch, 3)
    p1.set_tune_cache(str(cache))
    ms1 = p1.tune(x, y, off, dg, reps=1)
    lines = cache.read_text().splitlines()
    assert len(lines) == 1
    key, vals = lines[0].split("\t")
    assert f"B={bf.batch} " in key and " m=3 " in key
    w, wpb, tile, unroll, ms, form = vals.split()
    assert p1.schedule == {"waves": int(w), "waves_per_block": int(wpb), "tile": int(tile), "unroll": int(unroll)}
    assert float(ms) == pytest.approx(ms1, abs=5.1e-7)   # written with six decimals
    assert form in ("0", "1") and p1.graph == (form == "1")   # the replay form the tuning kept
    # a hit installs the cached schedule and form without timing or appending
    p2 = lf.Plan(bf.batch, 3)
    p2.set_graph(form == "0")
    p2.set_tune_cache(str(cache))
    p2b = lf.Plan(bf.batch, 3)
    p2b.set_tune_cache(str(cache))
    assert p2.tune(x, y, off, dg, reps=1) == pytest.approx(ms1, abs=5.1e-7)
    assert p2b.tune(x, y, off, dg, reps=1) == pytest.approx(ms1, abs=5.1e-7)
    assert p2.schedule == p1.schedule and p2b.schedule == p1.schedule
    assert p2b.graph == p1.graph and p2.graph != p1.graph   # a form the caller set is kept
    assert len(cache.read_text().splitlines()) == 1
    # the last line of a key wins (a line of five fields leaves the form as it
    # is); the plan then fits with that schedule
    cus = lf.device_cus()
    with open(cache, "a") as fh:
        fh.write(f"{key}\t{cus * 4} 2 256 1 0.5\n")
    p3 = lf.Plan(bf.batch, 3)
    p3.set_tune_cache(str(cache))
    assert p3.tune(x, y, off, dg, reps=1) == 0.5
    assert p3.schedule == {"waves": cus * 4, "waves_per_block": 2, "tile": 256, "unroll": 1}
    assert p3.graph                                          # a new plan's form
    coef, status = run_batched(bf, 3, plan=p3)
    check_against_oracle(bf, coef, status, 1e-9)
    # another shape misses the cache and adds its own line
    p4 = lf.Plan(bf.batch - 1, 3)
    p4.set_tune_cache(str(cache))
    p4.tune(x, y, off[:-1].contiguous(), dg[:-1].contiguous(), reps=1)
    assert len(cache.read_text().splitlines()) == 3
    p4.set_tune_cache(None)
    for p in (p1, p2, p2b, p3, p4):
        p.close()


@pytest.mark.parametrize("chosen", [None, False, True])
def test_tuned_replay_form(chosen):
    """tune() keeps the faster of eager launches and graph replays unless the
    caller chose a form; either form gives the same bits as eager calls with
    the tuned schedule, call after call."""
    announce(f"tuned replay form (caller's choice {chosen})")
    rng = np.random.default_rng(21)
    L = W.ragged_lengths(3000, 16, 8_000, rng)
    deg = rng.integers(1, 4, 3000)
    bf = W.random_batch(L, deg, seed=22, lo=-5.0, hi=5.0)
    x, y = to_dev(bf.x), to_dev(bf.y)
    off, dg = to_dev(bf.offsets), to_dev(bf.degrees)
    plan = lf.Plan(bf.batch, 3)
    if chosen is not None:
        plan.set_graph(chosen)
    plan.tune(x, y, off, dg, reps=2)
    if chosen is not None:
        assert plan.graph == chosen
    announce(f"  form: {'graph' if plan.graph else 'eager'}, schedule {plan.schedule}")
    ref = lf.Plan(bf.batch, 3)
    ref.set_schedule(plan.schedule)
    ref.set_graph(False)
    want, wst = run_batched(bf, 3, plan=ref)
    coef = torch.zeros(bf.batch, 4, dtype=torch.float64, device=x.device)
    status = torch.zeros(bf.batch, dtype=torch.int32, device=x.device)
    for _ in range(3):
        coef.zero_()                # entries past a fit's degree stay as they are
        status.fill_(-1)
        lf.fit_batched(x, y, off, dg, 3, plan=plan, out=(coef, status))
        torch.cuda.synchronize()
        assert np.array_equal(coef.cpu().numpy(), want, equal_nan=True)
        assert np.array_equal(status.cpu().numpy(), wst)
        _ = (x * 2).sum().item()    # eager work between calls
    check_against_oracle(bf, want, wst, 1e-9)
    plan.close()
    ref.close()


def test_graph_recaptures_when_pointers_change():
    plan = lf.Plan(3, 2)
    for seed in (10, 11):
        bf = W.random_batch([500, 600, 700], [2, 2, 1], seed=seed)
        coef, status = run_batched(bf, 2, plan=plan)
        check_against_oracle(bf, coef, status, 1e-9)
    plan.close()


# --- adjoint -------------------------------------------------------------------

# largest degree 3: the walk solves for lambda itself; 6: a separate solve launch first
@pytest.mark.parametrize("maxd,lengths,degrees", [(3, [4096, 1000, 257, 33], [2, 3, 1, 2]),
                                                  (6, [4096, 1000, 257, 33, 3000, 5000], [2, 3, 1, 2, 5, 6])])
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_adjoint_against_oracle(dtype, maxd, lengths, degrees):
    announce(f"adjoint {np.dtype(dtype).name}, largest degree {maxd}")
    bf = W.random_batch(lengths, degrees, seed=12, dtype=dtype, with_target=True)
    x = to_dev(bf.x).requires_grad_(True)
    y = to_dev(bf.y).requires_grad_(True)
    off, dg = to_dev(bf.offsets), to_dev(bf.degrees)
    target = torch.from_numpy(bf.target).to(x.device)
    coef = lf.lsefit(x, y, off, dg, maxd, center=0.0, scale=1.0)
    mask = torch.zeros_like(coef)
    for f in range(bf.batch):
        mask[f, : int(bf.degrees[f]) + 1] = 1.0
    loss = (((coef - target) * mask) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    gx, gy = x.grad.cpu().numpy(), y.grad.cpu().numpy()
    tol = 1e-5 if dtype == np.float32 else 1e-10
    a_all = coef.detach().cpu().numpy()
    for f in range(bf.batch):
        lo, hi = bf.offsets[f], bf.offsets[f + 1]
        m = int(bf.degrees[f])
        gbar = 2.0 * (a_all[f, : m + 1] - bf.target[f, : m + 1])
        ref = adjoint.gradients(bf.x[lo:hi], bf.y[lo:hi], m, gbar)
        # the float32 gradients are rounded on store; compare against the rounded oracle too
        assert normwise(gx[lo:hi], ref["dx"]) <= tol, f
        assert normwise(gy[lo:hi], ref["dy"]) <= tol, f


@pytest.mark.parametrize("precision,tol", [("f64", 1e-9), ("f32c", 1e-6)])
def test_batched_t_basis_output(precision, tol):
    """output_basis="x_and_t": rows [a | b | c | s]; b is the fit in t = (x - c)/s
    (the oracle's fit with the same c and s), a is the plain call's output bit
    for bit, and a fit with too few points has NaN a and b but its (c, s)."""
    announce(f"batched t-basis output {precision}")
    from oracle import fp64
    bf = W.random_batch([5000, 20_000, 2, 777, 65_537], [5, 3, 2, 4, 5], seed=33, lo=1000.0, hi=1001.0)
    x, y = to_dev(bf.x), to_dev(bf.y)
    off, dg = to_dev(bf.offsets), to_dev(bf.degrees)
    M = 5
    coef, status, _ = lf.fit_batched(x, y, off, dg, M, precision=precision, output_basis="x_and_t")
    plain, pstatus, _ = lf.fit_batched(x, y, off, dg, M, precision=precision)
    torch.cuda.synchronize()
    coef, status = coef.cpu().numpy(), status.cpu().numpy()
    plain = plain.cpu().numpy()
    assert coef.shape == (bf.batch, 2 * M + 4)
    assert np.array_equal(status, pstatus.cpu().numpy())
    for f in range(bf.batch):
        m = int(bf.degrees[f])
        lo, hi = bf.offsets[f], bf.offsets[f + 1]
        c, s = coef[f, 2 * M + 2], coef[f, 2 * M + 3]
        assert np.isfinite(c) and s > 0 and abs(c - 1000.5) <= 0.5
        a, b = coef[f, : m + 1], coef[f, M + 1: M + 2 + m]
        assert np.array_equal(a, plain[f, : m + 1], equal_nan=True)
        if status[f] != 0:
            assert np.isnan(a).all() and np.isnan(b).all()
            continue
        ref = fp64.fit(bf.x[lo:hi], bf.y[lo:hi], m, float(c), float(s))
        assert normwise(b, ref["b"]) <= tol, f
    assert status[2] == 2


def test_adjoint_after_compensated_forward():
    """Backward after a compensated-float32 forward: the adjoint solves with the
    sums and refined coefficients that forward left in the workspace."""
    announce("adjoint after an f32c forward")
    bf = W.random_batch([4096, 1000, 257, 3000], [2, 3, 1, 3], seed=31, lo=-2.0, hi=3.0, with_target=True)
    x = to_dev(bf.x).requires_grad_(True)
    y = to_dev(bf.y).requires_grad_(True)
    off, dg = to_dev(bf.offsets), to_dev(bf.degrees)
    target = torch.from_numpy(bf.target).to(x.device)
    coef = lf.lsefit(x, y, off, dg, 3, precision="f32c")
    mask = torch.zeros_like(coef)
    for f in range(bf.batch):
        mask[f, : int(bf.degrees[f]) + 1] = 1.0
    (((coef - target) * mask) ** 2).sum().backward()
    torch.cuda.synchronize()
    gx, gy = x.grad.cpu().numpy(), y.grad.cpu().numpy()
    a_all = coef.detach().cpu().numpy()
    for f in range(bf.batch):
        lo, hi = bf.offsets[f], bf.offsets[f + 1]
        m = int(bf.degrees[f])
        ref = adjoint.gradients(bf.x[lo:hi], bf.y[lo:hi], m, 2.0 * (a_all[f, : m + 1] - bf.target[f, : m + 1]))
        assert normwise(gx[lo:hi], ref["dx"]) <= 1e-5, f
        assert normwise(gy[lo:hi], ref["dy"]) <= 1e-5, f


@pytest.mark.parametrize("maxd,degrees", [(3, [2, 3, 1, 2]), (6, [2, 3, 1, 6])])
def test_adjoint_with_cholesky(maxd, degrees):
    """The adjoint solve with the Cholesky factorisation (in the walk up to
    degree 3, in its own launch above) against the float64 adjoint oracle."""
    announce(f"adjoint, Cholesky, largest degree {maxd}")
    bf = W.random_batch([4096, 1000, 257, 3001], degrees, seed=14, dtype=np.float64, with_target=True)
    x, y = to_dev(bf.x), to_dev(bf.y)
    off, dg = to_dev(bf.offsets), to_dev(bf.degrees)
    coef, status, ws = lf.fit_batched(x, y, off, dg, maxd, center=0.0, scale=1.0, solver="cholesky")
    torch.cuda.synchronize()
    assert (status.cpu().numpy() == 0).all()
    a_all = coef.cpu().numpy()
    gbar = np.zeros_like(a_all)
    for f in range(bf.batch):
        m = int(bf.degrees[f])
        gbar[f, : m + 1] = 2.0 * (a_all[f, : m + 1] - bf.target[f, : m + 1])
    gx, gy = lf.fit_backward(x, y, off, dg, maxd, torch.from_numpy(gbar).to(x.device), ws=ws,
                             center=0.0, scale=1.0, solver="cholesky")
    torch.cuda.synchronize()
    gx, gy = gx.cpu().numpy(), gy.cpu().numpy()
    for f in range(bf.batch):
        lo, hi = bf.offsets[f], bf.offsets[f + 1]
        m = int(bf.degrees[f])
        ref = adjoint.gradients(bf.x[lo:hi], bf.y[lo:hi], m, gbar[f, : m + 1])
        assert normwise(gx[lo:hi], ref["dx"]) <= 1e-9, f
        assert normwise(gy[lo:hi], ref["dy"]) <= 1e-9, f


def test_adjoint_lambda_in_stream_matches_separate_solve():
    """Up to degree 3 the adjoint walk solves for lambda itself; above, a
    separate launch solves first.  The same fits (degrees 1-3) run with
    largest degree 3 and 4: when the forward gives the same bits under both,
    so do the gradients; otherwise they agree to rounding."""
    announce("adjoint: lambda in the walk against the separate solve")
    bf = W.random_batch([5000, 70_001, 1, 12_345, 999, 2048, 4096], [2, 3, 1, 2, 3, 1, 2], seed=41)
    x, y = to_dev(bf.x), to_dev(bf.y)
    off, dg = to_dev(bf.offsets), to_dev(bf.degrees)
    g = torch.from_numpy(np.random.default_rng(42).standard_normal((bf.batch, 5))).to(x.device)
    out = []
    for maxd in (3, 4):
        coef, status, ws = lf.fit_batched(x, y, off, dg, maxd)
        gx, gy = lf.fit_backward(x, y, off, dg, maxd, g[:, : maxd + 1].contiguous(), ws=ws)
        torch.cuda.synchronize()
        out.append((coef.cpu().numpy()[:, :4], status.cpu().numpy(), gx.cpu().numpy(), gy.cpu().numpy()))
    (c3, s3, gx3, gy3), (c4, s4, gx4, gy4) = out
    assert np.array_equal(s3, s4) and s3[2] != 0 and (np.delete(s3, 2) == 0).all()
    lo, hi = bf.offsets[2], bf.offsets[3]
    assert np.isnan(gx3[lo:hi]).all() and np.isnan(gx4[lo:hi]).all()
    same_forward = np.array_equal(c3, c4, equal_nan=True)
    announce(f"  forward bits equal under both: {same_forward}")
    if same_forward:
        assert np.array_equal(gx3, gx4, equal_nan=True) and np.array_equal(gy3, gy4, equal_nan=True)
    else:
        keep = np.isfinite(gx4)
        assert normwise(gx3[keep], gx4[keep]) <= 1e-6 and normwise(gy3[keep], gy4[keep]) <= 1e-6


def test_batched_workspace_need_not_be_cleared():
    """A batch fitted, differentiated and its residuals summed on a workspace
    that starts with arbitrary bytes gives the same bits as on a cleared one."""
    announce("batched calls on an uncleared workspace")
    bf = W.random_batch([5000, 70_001, 1, 12_345, 999, 0, 4096], [2, 3, 1, 2, 3, 1, 2], seed=43,
                        with_target=True)
    x, y = to_dev(bf.x), to_dev(bf.y)
    off, dg = to_dev(bf.offsets), to_dev(bf.degrees)
    g = torch.from_numpy(np.nan_to_num(bf.target)).to(x.device)
    nbytes = lf.workspace_bytes(bf.batch, 3)
    out = []
    for fill in (0x00, 0x5A, 0xFF):
        ws = torch.full((nbytes,), fill, dtype=torch.uint8, device=x.device)
        coef, status, _ = lf.fit_batched(x, y, off, dg, 3, ws=ws)
        gx, gy = lf.fit_backward(x, y, off, dg, 3, g, ws=ws)
        sse, _ = lf.residuals_batched(x, y, off, dg, 3, ws=ws)
        torch.cuda.synchronize()
        out.append([t.cpu().numpy() for t in (coef, status, gx, gy, sse)])
    for other in out[1:]:
        for a, b in zip(out[0], other):
            assert np.array_equal(a, b, equal_nan=True)
    assert out[0][1][2] == 2 and out[0][1][5] == 2      # the one-point and the empty fit


def test_backward_and_residuals_after_schedule_change():
    """The adjoint and the residual pass read the tile size from the forward's
    tile table, so a default schedule changed between forward and backward
    (other tile, other grid) gives the same gradients, bit for bit, and the
    same sums of squared residuals up to their summation order."""
    announce("schedule change between forward and backward")
    bf = W.random_batch([5000, 70_001, 3, 12_345, 999], [2, 3, 1, 2, 3], seed=32, with_target=True)
    x, y = to_dev(bf.x), to_dev(bf.y)
    off, dg = to_dev(bf.offsets), to_dev(bf.degrees)
    g = torch.from_numpy(np.nan_to_num(bf.target)).to(x.device)
    base = lf.default_schedule().as_dict()
    other = {"waves": 1024, "waves_per_block": 2, "tile": 256, "unroll": 1}
    assert other["tile"] != base["tile"] and other["waves"] != base["waves"]
    coef, status, ws = lf.fit_batched(x, y, off, dg, 3)
    gx0, gy0 = lf.fit_backward(x, y, off, dg, 3, g, ws=ws)
    sse0, _ = lf.residuals_batched(x, y, off, dg, 3, ws=ws)
    torch.cuda.synchronize()
    try:
        lf.set_default_schedule(other)
        gx1, gy1 = lf.fit_backward(x, y, off, dg, 3, g, ws=ws)
        sse1, _ = lf.residuals_batched(x, y, off, dg, 3, ws=ws)
        torch.cuda.synchronize()
    finally:
        lf.set_default_schedule(None)
    assert torch.equal(gx0, gx1) and torch.equal(gy0, gy1)
    st = status.cpu().numpy()
    s0, s1 = sse0.cpu().numpy(), sse1.cpu().numpy()
    ok = st == 0
    assert np.isnan(s1[~ok]).all() and np.isfinite(s1[ok]).all()
    assert np.max(np.abs(s1[ok] - s0[ok]) / s0[ok]) <= 1e-12


def test_adjoint_against_finite_differences():
    bf = W.random_batch([300], [2], seed=13, dtype=np.float64, with_target=True)
    x = to_dev(bf.x).requires_grad_(True)
    y = to_dev(bf.y).requires_grad_(True)
    off, dg = to_dev(bf.offsets), to_dev(bf.degrees)
    target = bf.target[0, :3]
    coef = lf.lsefit(x, y, off, dg, 2)
    loss = ((coef[0] - torch.from_numpy(target).to(x.device)) ** 2).sum()
    loss.backward()
    fd = adjoint.fd_gradients(bf.x, bf.y, 2, lambda a: np.sum((a - target) ** 2, axis=-1), h=1e-6)
    assert normwise(x.grad.cpu().numpy(), fd["dx"]) <= 1e-4
    assert normwise(y.grad.cpu().numpy(), fd["dy"]) <= 1e-4


def test_adjoint_nan_for_failed_fits():
    bf = W.random_batch([100, 2, 100], [2, 2, 2], seed=14)
    x = to_dev(bf.x).requires_grad_(True)
    y = to_dev(bf.y).requires_grad_(True)
    coef = lf.lsefit(x, y, to_dev(bf.offsets), to_dev(bf.degrees), 2)
    torch.nan_to_num(coef).sum().backward()
    g = x.grad.cpu().numpy()
    assert np.isfinite(g[:100]).all() and np.isnan(g[100:102]).all() and np.isfinite(g[102:]).all()


def test_batched_cholesky_and_residuals():
    rng = np.random.default_rng(20)
    L = W.ragged_lengths(300, 16, 40_000, rng)
    deg = rng.integers(1, 4, 300)
    L[5] = 2          # singular
    bf = W.random_batch(L, deg, seed=21, lo=-5.0, hi=5.0)
    x, y = to_dev(bf.x), to_dev(bf.y)
    off, dg = to_dev(bf.offsets), to_dev(bf.degrees)
    for solver in ("gepp", "cholesky"):
        coef, status, ws = lf.fit_batched(x, y, off, dg, 3, solver=solver)
        torch.cuda.synchronize()
        check_against_oracle(bf, coef.cpu().numpy(), status.cpu().numpy(), 1e-9)
    sse, e = lf.residuals_batched(x, y, off, dg, 3, ws=ws, store=True)
    torch.cuda.synchronize()
    sse = sse.cpu().numpy()
    e = e.cpu().numpy()
    ref, rst = c_oracle.fit_batched(bf.x, bf.y, bf.offsets, bf.degrees, stride=4)
    from oracle import fp64
    for f in range(bf.batch):
        lo, hi = bf.offsets[f], bf.offsets[f + 1]
        if rst[f] != 0:
            assert np.isnan(sse[f]) and np.isnan(e[lo:hi]).all()
            continue
        m = int(bf.degrees[f])
        s_ref = fp64.sse(bf.x[lo:hi], bf.y[lo:hi], ref[f, : m + 1])
        assert abs(sse[f] - s_ref) <= 1e-9 * s_ref + 1e-300, f
        e_ref = bf.y[lo:hi].astype(np.float64) - fp64.polyval(ref[f, : m + 1], bf.x[lo:hi])
        assert np.max(np.abs(e[lo:hi] - e_ref)) <= 1e-5 * max(np.max(np.abs(e_ref)), 1e-30), f
