"""The kernel clock of lsefit_timing_*: every timed launch stamps its own start
and end, the durations fit inside the region of events around the same
launches, and nothing is counted while timing is off or for the entry point
that allocates nothing."""
import ctypes

import numpy as np
import pytest

from gpu_common import announce, to_dev, torch
from paper_1512_08017_amd import _lib, api, workloads as W

pytestmark = pytest.mark.gpu


def _read(L, kind):
    tot, cnt = ctypes.c_double(0.0), ctypes.c_int64(0)
    _lib.check(L.lsefit_timing_read(kind, ctypes.byref(tot), ctypes.byref(cnt)), "lsefit_timing_read")
    return tot.value, cnt.value


def test_kernel_clock_durations_fit_the_region():
    L = _lib.load()
    n, m, K = 20_000_000, 3, 6
    announce(f"kernel clock: fit_single n={n} m={m}, {K} timed steps")
    fit = W.random_small(n, m, seed=31, dtype=np.float32)
    x, y = to_dev(fit.x), to_dev(fit.y)
    vp = ctypes.c_void_p
    opt = api.options(m)
    ws = torch.zeros(api.workspace_bytes(1, m), dtype=torch.uint8, device=x.device)
    coef = torch.empty(2 * (m + 1), dtype=torch.float64, device=x.device)
    status = torch.empty(1, dtype=torch.int32, device=x.device)
    st = vp(torch.cuda.current_stream().cuda_stream)
    args = (vp(x.data_ptr()), vp(y.data_ptr()), n, _lib.F32, ctypes.byref(opt), vp(ws.data_ptr()), ws.numel(),
            vp(coef.data_ptr()), vp(status.data_ptr()), None, st)
    step = lambda: _lib.check(L.fit_single(*args), "fit_single")
    for _ in range(2):
        step()
    _lib.check(L.lsefit_timing_reset(), "lsefit_timing_reset")
    _lib.check(L.lsefit_timing_enable(1), "lsefit_timing_enable")
    try:
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(K):
            step()
        b.record()
        torch.cuda.synchronize()
    finally:
        L.lsefit_timing_enable(0)
    region = a.elapsed_time(b)
    mom, nm = _read(L, 0)
    fin, nf = _read(L, 3)
    announce(f"  region {region / K:.4f} ms/step, moments {mom / max(nm, 1):.4f} ms, finish {fin / max(nf, 1):.4f} ms")
    assert nm == K and nf == K
    assert 0.0 < mom and 0.0 < fin
    # the two kernels of a step run one after the other inside the region
    assert mom + fin <= region * 1.02
    # 160 MB read: the pass takes at least 160 MB / 8 TB/s, and most of the step
    assert mom / K >= 0.160 / 8000 * 1e3
    assert mom >= 0.5 * region
    assert int(status.cpu()[0]) == 0
    # off: nothing more is counted; reset clears the totals
    step()
    torch.cuda.synchronize()
    assert _read(L, 0)[1] == K
    _lib.check(L.lsefit_timing_reset(), "lsefit_timing_reset")
    assert _read(L, 0) == (0.0, 0)


def test_noalloc_launches_are_not_timed():
    L = _lib.load()
    n, m = 100_003, 2
    fit = W.random_small(n, m, seed=32, dtype=np.float32)
    x, y = to_dev(fit.x), to_dev(fit.y)
    vp = ctypes.c_void_p
    opt = api.options(m)
    coef = torch.empty(2 * (m + 1), dtype=torch.float64, device=x.device)
    status = torch.empty(1, dtype=torch.int32, device=x.device)
    _lib.check(L.lsefit_timing_reset(), "lsefit_timing_reset")
    _lib.check(L.lsefit_timing_enable(1), "lsefit_timing_enable")
    try:
        _lib.check(L.fit_single_noalloc(vp(x.data_ptr()), vp(y.data_ptr()), n, _lib.F32, ctypes.byref(opt),
                                        vp(coef.data_ptr()), vp(status.data_ptr()), None,
                                        vp(torch.cuda.current_stream().cuda_stream)), "fit_single_noalloc")
        torch.cuda.synchronize()
    finally:
        L.lsefit_timing_enable(0)
    assert _read(L, 0)[1] == 0 and _read(L, 3)[1] == 0
    assert int(status.cpu()[0]) == 0


@pytest.mark.parametrize("batch", [300, 9000])
def test_batched_call_times_its_tile_table(batch):
    """A batched call is timed as one tile table (kind 7: its first launch, in
    the one-launch form up to 8,192 fits and the two-launch form above), one
    power-sum pass (kind 0) and one combine (kind 3)."""
    import paper_1512_08017_amd as lf
    announce(f"kernel clock: batched call of {batch} fits")
    rng = np.random.default_rng(batch)
    bf = W.random_batch(rng.integers(20, 400, batch), rng.integers(1, 4, batch), seed=batch)
    x, y = to_dev(bf.x), to_dev(bf.y)
    off, dg = to_dev(bf.offsets), to_dev(bf.degrees)
    lf.fit_batched(x, y, off, dg, 3)
    torch.cuda.synchronize()
    L = _lib.load()
    _lib.check(L.lsefit_timing_reset(), "lsefit_timing_reset")
    _lib.check(L.lsefit_timing_enable(1), "lsefit_timing_enable")
    try:
        for _ in range(3):
            _, status, _ = lf.fit_batched(x, y, off, dg, 3)
        torch.cuda.synchronize()
    finally:
        L.lsefit_timing_enable(0)
    for kind in (7, 0, 3):
        tot, cnt = _read(L, kind)
        assert cnt == 3 and tot > 0.0, (kind, tot, cnt)
    assert (status.cpu().numpy() == 0).all()
