"""The C ABI loads on a machine without a GPU, exports every symbol that
include/lsefit.h declares, and rejects bad arguments on the host before any
device work (no compute call is made here)."""
import ctypes
import os
import re

import pytest

from paper_1512_08017_amd import _lib

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "lsefit.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s+\*?([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_expected_entry_points():
    assert set(declared_functions()) == set(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = _lib.load()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_status_strings():
    L = _lib.load()
    assert L.lsefit_status_string(_lib.OK) == b"ok"
    assert L.lsefit_status_string(_lib.SINGULAR) == b"singular normal system"
    assert L.lsefit_status_string(99) == b"unknown status"


def _opt(**kw):
    o = _lib.Options()
    o.degree, o.precision, o.refine_steps, o.range_mode, o.center, o.scale = 3, 0, 0, 1, 0.0, 1.0
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def test_workspace_bytes_grows_with_batch_and_degree():
    L = _lib.load()
    s = _lib.Schedule(4096, 4, 256, 2)
    a = L.lsefit_workspace_bytes(1, 3, ctypes.byref(s))
    b = L.lsefit_workspace_bytes(1000, 3, ctypes.byref(s))
    c = L.lsefit_workspace_bytes(1000, 8, ctypes.byref(s))
    assert 0 < a < b < c
    assert L.lsefit_workspace_bytes(0, 3, ctypes.byref(s)) == 0
    assert L.lsefit_workspace_bytes(1, 16, ctypes.byref(s)) > a      # Chebyshev-basis fits go to 16
    assert L.lsefit_workspace_bytes(1, 17, ctypes.byref(s)) == 0
    bad = _lib.Schedule(4096, 3, 256, 2)
    assert L.lsefit_workspace_bytes(1, 3, ctypes.byref(bad)) == 0


FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails validation first


@pytest.mark.parametrize("kw,n,dt,expect", [
    ({"degree": 0}, 100, _lib.F32, _lib.INVALID_ARG),
    ({"degree": 9}, 100, _lib.F32, _lib.INVALID_ARG),
    ({}, 3, _lib.F32, _lib.INVALID_ARG),                       # n < m + 1
    ({"precision": 1}, 100, _lib.F64, _lib.UNSUPPORTED),       # compensated FP32 needs FP32 data
    ({"range_mode": 0, "scale": 0.0}, 100, _lib.F32, _lib.INVALID_ARG),
    ({"range_mode": 0, "scale": float("nan")}, 100, _lib.F32, _lib.INVALID_ARG),
    ({"refine_steps": 2}, 100, _lib.F32, _lib.INVALID_ARG),
    ({}, 100, 7, _lib.INVALID_ARG),
    ({"basis": 2}, 100, _lib.F32, _lib.INVALID_ARG),
    ({"basis": 1, "degree": 17}, 100, _lib.F32, _lib.INVALID_ARG),
    ({"basis": 1, "degree": 16}, 16, _lib.F32, _lib.INVALID_ARG),    # n < m + 1
    ({"basis": 1, "precision": 1}, 100, _lib.F32, _lib.UNSUPPORTED),  # Chebyshev sums are float64 only
])
def test_fit_moments_host_validation(kw, n, dt, expect):
    L = _lib.load()
    o = _opt(**kw)
    assert L.fit_moments(FAKE, FAKE, n, dt, ctypes.byref(o), FAKE, 1 << 30, FAKE, None) == expect


@pytest.mark.parametrize("kw,expect", [
    ({"degree": 9}, _lib.INVALID_ARG),
    ({"precision": 1}, _lib.UNSUPPORTED),            # the QR route accumulates in float64 only
    ({"basis": 1}, _lib.UNSUPPORTED),                # monomial basis only
])
def test_fit_qr_host_validation(kw, expect):
    L = _lib.load()
    o = _opt(**kw)
    assert L.fit_qr(FAKE, FAKE, 100, _lib.F32, ctypes.byref(o), FAKE, 1 << 30, FAKE, FAKE, None, None) == expect
    assert L.fit_qr(FAKE, FAKE, 100, _lib.F32, ctypes.byref(_opt()), FAKE, 16, FAKE, FAKE, None, None) == _lib.WORKSPACE
    assert L.fit_qr(FAKE, FAKE, 100, _lib.F32, ctypes.byref(_opt()), FAKE, 1 << 30, None, FAKE, None,
                    None) == _lib.INVALID_ARG


def test_fit_qr_batched_host_validation():
    L = _lib.load()
    o = _opt()
    args = (FAKE, FAKE, FAKE, FAKE, 10, _lib.F32)
    assert L.fit_qr_batched(*args, ctypes.byref(o), FAKE, 1 << 30, FAKE, 3, FAKE, None, None) == _lib.INVALID_ARG
    assert L.fit_qr_batched(*args, ctypes.byref(_opt(precision=1)), FAKE, 1 << 30, FAKE, 4, FAKE, None,
                            None) == _lib.UNSUPPORTED
    assert L.fit_qr_batched(*args, ctypes.byref(o), FAKE, 8, FAKE, 4, FAKE, None, None) == _lib.WORKSPACE
    assert L.fit_qr_batched(FAKE, FAKE, FAKE, FAKE, 0, _lib.F32, ctypes.byref(o), None, 0, None, 4, None, None,
                            None) == _lib.OK


def test_fit_moments_workspace_too_small():
    L = _lib.load()
    o = _opt()
    assert L.fit_moments(FAKE, FAKE, 100, _lib.F32, ctypes.byref(o), FAKE, 16, FAKE, None) == _lib.WORKSPACE


def test_null_pointers_rejected():
    L = _lib.load()
    o = _opt()
    assert L.fit_moments(None, FAKE, 100, _lib.F32, ctypes.byref(o), FAKE, 1 << 30, FAKE, None) == _lib.INVALID_ARG
    assert L.fit_solve(None, ctypes.byref(o), None, None, 0, _lib.F32, FAKE, 1 << 30, FAKE, FAKE,
                       None) == _lib.INVALID_ARG
    assert L.fit_batched(FAKE, FAKE, None, FAKE, 10, _lib.F32, ctypes.byref(o), None, FAKE, 1 << 30, FAKE, 4,
                         FAKE, None) == _lib.INVALID_ARG
    assert L.fit_batched(FAKE, FAKE, FAKE, FAKE, 10, _lib.F32, ctypes.byref(o), None, FAKE, 1 << 30, FAKE, 3,
                         FAKE, None) == _lib.INVALID_ARG           # coef_stride < m + 1
    assert L.fit_batched(FAKE, FAKE, FAKE, FAKE, 10, _lib.F32, ctypes.byref(o), None, FAKE, 8, FAKE, 4,
                         FAKE, None) == _lib.WORKSPACE
    assert L.fit_batched(FAKE, FAKE, FAKE, FAKE, 0, _lib.F32, ctypes.byref(o), None, None, 0, None, 4,
                         None, None) == _lib.OK                    # empty batch: nothing to do
    assert L.fit_backward(FAKE, FAKE, FAKE, FAKE, 10, _lib.F32, ctypes.byref(o), None, FAKE, 1 << 30, None, 4,
                          FAKE, FAKE, None) == _lib.INVALID_ARG
    assert L.fit_plan_create(None, 10, 3, _lib.F32, 0) == _lib.INVALID_ARG
    cheb = _opt(basis=1)
    assert L.fit_backward(FAKE, FAKE, FAKE, FAKE, 10, _lib.F32, ctypes.byref(cheb), None, FAKE, 1 << 30, FAKE, 4,
                          FAKE, FAKE, None) == _lib.UNSUPPORTED     # no adjoint for the Chebyshev basis
    assert L.fit_residuals(FAKE, FAKE, None, None, 1, 100, _lib.F32, ctypes.byref(cheb), None, FAKE, 8,
                           FAKE, None, None) == _lib.WORKSPACE      # Chebyshev residuals are taken; ws too small
    assert L.fit_residuals(FAKE, FAKE, None, None, 1, 12, _lib.F32, ctypes.byref(_opt(basis=1, degree=12)), None,
                           FAKE, 1 << 30, FAKE, None, None) == _lib.INVALID_ARG   # n < m + 1
    h = ctypes.c_void_p()
    assert L.fit_plan_create(ctypes.byref(h), 10, 17, _lib.F32, 0) == _lib.INVALID_ARG
    assert L.fit_plan_set_graph(None, 1) == _lib.INVALID_ARG
    assert L.fit_plan_get_graph(None, ctypes.byref(ctypes.c_int32())) == _lib.INVALID_ARG
    L.fit_plan_destroy(None)


def test_fit_single_noalloc_host_validation():
    """The entry point without a workspace argument validates like fit_single
    and refuses a call whose workspace would not fit its static array (here: a
    default schedule of 65,536 waves) before touching any device."""
    L = _lib.load()
    o = _opt()
    assert L.fit_single_noalloc(None, FAKE, 100, _lib.F32, ctypes.byref(o), FAKE, FAKE, None, None) == _lib.INVALID_ARG
    assert L.fit_single_noalloc(FAKE, FAKE, 100, _lib.F32, ctypes.byref(o), None, FAKE, None, None) == _lib.INVALID_ARG
    assert L.fit_single_noalloc(FAKE, FAKE, 3, _lib.F32, ctypes.byref(o), FAKE, FAKE, None, None) == _lib.INVALID_ARG
    assert L.fit_single_noalloc(FAKE, FAKE, 100, _lib.F64, ctypes.byref(_opt(precision=1)), FAKE, FAKE, None,
                                None) == _lib.UNSUPPORTED
    big = _lib.Schedule(1 << 16, 4, 2048, 2)
    assert L.lsefit_workspace_bytes(1, 3, ctypes.byref(big)) > _lib.NOALLOC_SCRATCH_BYTES
    assert L.lsefit_workspace_bytes(1, 8, None) <= _lib.NOALLOC_SCRATCH_BYTES      # the default schedule fits
    assert L.lsefit_workspace_bytes(1, 16, None) <= _lib.NOALLOC_SCRATCH_BYTES
    assert L.lsefit_set_default_schedule(ctypes.byref(big)) == _lib.OK
    try:
        assert L.fit_single_noalloc(FAKE, FAKE, 100, _lib.F32, ctypes.byref(o), FAKE, FAKE, None,
                                    None) == _lib.WORKSPACE
    finally:
        assert L.lsefit_set_default_schedule(None) == _lib.OK


@pytest.mark.gpu
def test_plan_tune_validates_against_the_plan():
    """A degree above the plan's, a short stride or a null pointer never reaches
    the kernels (the plan's workspace is sized for its own maximum degree).
    Every pointer is a real device buffer of the call's shape."""
    import torch
    dev = torch.device("cuda:0")
    x = torch.zeros(100, dtype=torch.float32, device=dev)
    y = torch.zeros(100, dtype=torch.float32, device=dev)
    off = torch.arange(0, 101, 10, dtype=torch.int64, device=dev)
    deg = torch.full((10,), 2, dtype=torch.int32, device=dev)
    coef = torch.zeros(10 * 4, dtype=torch.float64, device=dev)
    status = torch.zeros(10, dtype=torch.int32, device=dev)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    L = _lib.load()
    h = ctypes.c_void_p()
    assert L.fit_plan_create(ctypes.byref(h), 10, 2, _lib.F32, 0) == _lib.OK
    try:
        best = ctypes.c_double(0.0)
        o3 = _opt(degree=3)
        o2 = _opt(degree=2)
        assert L.fit_plan_tune(h, p(x), p(y), p(off), p(deg), 10, ctypes.byref(o3), p(coef), 4, p(status), None, 1,
                               ctypes.byref(best)) == _lib.INVALID_ARG
        assert L.fit_plan_tune(h, p(x), p(y), p(off), p(deg), 10, ctypes.byref(o2), p(coef), 2, p(status), None, 1,
                               ctypes.byref(best)) == _lib.INVALID_ARG
        assert L.fit_plan_tune(h, None, p(y), p(off), p(deg), 10, ctypes.byref(o2), p(coef), 3, p(status), None, 1,
                               ctypes.byref(best)) == _lib.INVALID_ARG
        torch.cuda.synchronize()
    finally:
        L.fit_plan_destroy(h)


def test_output_basis_validation():
    """The t-basis output of batched fits needs its option value known and a
    coefficient row of 2M + 4 entries; both are checked before any device work."""
    L = _lib.load()
    args = (FAKE, FAKE, FAKE, FAKE, 10, _lib.F32)
    assert L.fit_batched(*args, ctypes.byref(_opt(output_basis=2)), None, FAKE, 1 << 30, FAKE, 10,
                         FAKE, None) == _lib.INVALID_ARG
    assert L.fit_batched(*args, ctypes.byref(_opt(output_basis=1)), None, FAKE, 1 << 30, FAKE, 9,
                         FAKE, None) == _lib.INVALID_ARG            # needs 2 * 3 + 4 = 10
    assert L.fit_batched(*args, ctypes.byref(_opt(output_basis=1)), None, FAKE, 8, FAKE, 10,
                         FAKE, None) == _lib.WORKSPACE              # stride accepted, then the workspace
    assert L.fit_batched(*args, ctypes.byref(_opt(output_basis=1, basis=1)), None, FAKE, 8, FAKE, 4,
                         FAKE, None) == _lib.WORKSPACE              # ignored in the Chebyshev basis


def test_copy_probe_validation():
    L = _lib.load()
    odd = ctypes.c_void_p(0x1004)
    assert L.lsefit_copy_probe(FAKE, FAKE, None, FAKE, 1024, None, 0, 1, None) == _lib.INVALID_ARG
    assert L.lsefit_copy_probe(FAKE, FAKE, odd, FAKE, 1024, None, 0, 1, None) == _lib.INVALID_ARG
    assert L.lsefit_copy_probe(FAKE, FAKE, FAKE, FAKE, 1024, None, 3, 1, None) == _lib.INVALID_ARG
    assert L.lsefit_copy_probe(FAKE, FAKE, FAKE, FAKE, 3, None, 0, 1, None) == _lib.INVALID_ARG


def test_default_schedule_setter_validates():
    L = _lib.load()
    bad = _lib.Schedule(0, 4, 256, 2)
    assert L.lsefit_set_default_schedule(ctypes.byref(bad)) == _lib.INVALID_ARG
    s = _lib.Schedule()
    assert L.lsefit_default_schedule(ctypes.byref(s)) == _lib.OK
    assert s.waves > 0 and s.waves_per_block in (1, 2, 4) and s.tile >= 64


def test_package_import_does_not_load_or_fall_back():
    import paper_1512_08017_amd as lf
    assert callable(lf.fit)
    with pytest.raises((ValueError, TypeError)):
        import torch
        lf.fit(torch.zeros(10), torch.zeros(10), 1)   # CPU tensors are refused, never computed
