"""fit_single_noalloc (workspace in the library's static device array) against
fit_single (caller workspace) through the C ABI: two calls in a row, the second
on a smaller input, each checked bit for bit against fit_single on the same
data and against the float64 oracle within the single-fit bounds (1e-9 for the
float64 form, 1e-6 for the compensated float32 form after refinement)."""
import ctypes

import numpy as np
import pytest

from gpu_common import announce, normwise, to_dev, torch
from oracle import c_oracle
from paper_1512_08017_amd import _lib, api, workloads as W

pytestmark = pytest.mark.gpu


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _run_both(L, x, y, m, prec):
    """(coef, status, moments) of fit_single and of fit_single_noalloc on x, y."""
    vp = ctypes.c_void_p
    dt = _lib.F32 if x.dtype == torch.float32 else _lib.F64
    opt = api.options(m, prec, 1)
    out = []
    for noalloc in (False, True):
        coef = torch.full((2 * (m + 1),), -7.0, dtype=torch.float64, device=x.device)
        status = torch.full((1,), -1, dtype=torch.int32, device=x.device)
        mom = torch.full((3 * m + 4,), -7.0, dtype=torch.float64, device=x.device)
        if noalloc:
            rc = L.fit_single_noalloc(vp(x.data_ptr()), vp(y.data_ptr()), x.numel(), dt, ctypes.byref(opt),
                                      vp(coef.data_ptr()), vp(status.data_ptr()), vp(mom.data_ptr()), _stream())
        else:
            ws = torch.zeros(api.workspace_bytes(1, m), dtype=torch.uint8, device=x.device)
            rc = L.fit_single(vp(x.data_ptr()), vp(y.data_ptr()), x.numel(), dt, ctypes.byref(opt),
                              vp(ws.data_ptr()), ws.numel(), vp(coef.data_ptr()), vp(status.data_ptr()),
                              vp(mom.data_ptr()), _stream())
        _lib.check(rc, "fit_single_noalloc" if noalloc else "fit_single")
        torch.cuda.synchronize()
        out.append((coef.cpu().numpy(), int(status.cpu()[0]), mom.cpu().numpy()))
    return out


@pytest.mark.parametrize("prec,tol", [("f64", 1e-9), ("f32c", 1e-6)])
def test_noalloc_matches_fit_single_on_two_calls(prec, tol):
    L = _lib.load()
    m = 3
    # the second call is smaller: the array keeps the first call's contents,
    # which the second must not see
    for n, seed in ((1_000_003, 11), (20_011, 12)):
        announce(f"noalloc {prec}: n={n} m={m} seed={seed}")
        fit = W.random_small(n, m, seed=seed, dtype=np.float32)
        x, y = to_dev(fit.x), to_dev(fit.y)
        (ca, sa, ma), (cb, sb, mb) = _run_both(L, x, y, m, prec)
        assert sa == 0 and sb == 0
        assert np.array_equal(ca, cb) and np.array_equal(ma, mb)
        ref = c_oracle.fit(fit.x, fit.y, m)["a"]
        assert normwise(cb[: m + 1], ref) <= tol


def test_noalloc_float64_data_and_other_degrees():
    L = _lib.load()
    for m, n, seed in ((8, 300_007, 21), (1, 2_001, 22)):
        announce(f"noalloc f64 data: n={n} m={m} seed={seed}")
        fit = W.random_small(n, m, seed=seed, dtype=np.float64)
        x, y = to_dev(fit.x), to_dev(fit.y)
        (ca, sa, _), (cb, sb, _) = _run_both(L, x, y, m, "f64")
        assert sa == sb
        assert np.array_equal(ca, cb, equal_nan=True)


def test_noalloc_rejects_a_schedule_beyond_the_array():
    L = _lib.load()
    x = torch.zeros(64, dtype=torch.float32, device="cuda:0")
    coef = torch.zeros(8, dtype=torch.float64, device="cuda:0")
    status = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    vp = ctypes.c_void_p
    opt = api.options(3, "f64", 1)
    big = _lib.Schedule(1 << 16, 4, 2048, 2)   # 65,536 waves: the single-fit workspace exceeds 4 MiB
    assert L.lsefit_workspace_bytes(1, 3, ctypes.byref(big)) > _lib.NOALLOC_SCRATCH_BYTES
    _lib.check(L.lsefit_set_default_schedule(ctypes.byref(big)), "lsefit_set_default_schedule")
    try:
        rc = L.fit_single_noalloc(vp(x.data_ptr()), vp(x.data_ptr()), 64, _lib.F32, ctypes.byref(opt),
                                  vp(coef.data_ptr()), vp(status.data_ptr()), None, _stream())
    finally:
        _lib.check(L.lsefit_set_default_schedule(None), "lsefit_set_default_schedule")
    assert rc == _lib.WORKSPACE
