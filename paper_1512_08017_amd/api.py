"""Python surface of the HIP library: tensors in, tensors out.

Every function here only marshals arguments for the C ABI (include/lsefit.h):
device pointers of torch tensors, the current HIP stream of their device, and
a workspace tensor from torch's caching allocator.  All arithmetic of the fit
runs in the library's kernels; there is no CPU path.
"""
from __future__ import annotations

import os

import ctypes
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import Options, Schedule, check

_DT = {torch.float32: _lib.F32, torch.float64: _lib.F64}
_PREC = {"f64": _lib.PREC_F64, "f32c": _lib.PREC_F32C}
_SOLVER = {"gepp": _lib.SOLVER_GEPP, "cholesky": _lib.SOLVER_CHOLESKY}
_BASIS = {"monomial": _lib.BASIS_MONOMIAL, "chebyshev": _lib.BASIS_CHEBYSHEV}
_OUTPUT = {"x": _lib.OUTPUT_X, "x_and_t": _lib.OUTPUT_X_AND_T}


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def options(degree: int, precision: str = "f64", refine: int = 1, center=None, scale=None,
            solver: str = "gepp", basis: str = "monomial", output_basis: str = "x") -> Options:
    if precision not in _PREC:
        raise ValueError(f"precision must be one of {sorted(_PREC)}")
    if solver not in _SOLVER:
        raise ValueError(f"solver must be one of {sorted(_SOLVER)}")
    if basis not in _BASIS:
        raise ValueError(f"basis must be one of {sorted(_BASIS)}")
    if output_basis not in _OUTPUT:
        raise ValueError(f"output_basis must be one of {sorted(_OUTPUT)}")
    o = Options()
    o.output_basis = _OUTPUT[output_basis]
    o.solver = _SOLVER[solver]
    o.basis = _BASIS[basis]
    o.degree = int(degree)
    o.precision = _PREC[precision]
    o.refine_steps = int(refine) if precision == "f32c" else 0
    if center is None and scale is None:
        o.range_mode = _lib.RANGE_AUTO
        o.center, o.scale = 0.0, 1.0
    else:
        o.range_mode = _lib.RANGE_GIVEN
        o.center = float(0.0 if center is None else center)
        o.scale = float(1.0 if scale is None else scale)
    return o


def _check_points(x, y):
    if not (isinstance(x, torch.Tensor) and isinstance(y, torch.Tensor)):
        raise TypeError("x and y must be tensors")
    if not x.is_cuda or x.device != y.device:
        raise ValueError("x and y must be on the same GPU")
    if x.dtype not in _DT or y.dtype != x.dtype:
        raise TypeError("x and y must both be float32 or both float64")
    if x.dim() != 1 or y.shape != x.shape:
        raise ValueError("x and y must be 1-D of equal length")
    if not (x.is_contiguous() and y.is_contiguous()):
        raise ValueError("x and y must be contiguous")


def workspace_bytes(batch: int, max_degree: int, schedule: Schedule | None = None) -> int:
    L = _lib.load()
    n = L.lsefit_workspace_bytes(int(batch), int(max_degree), ctypes.byref(schedule) if schedule else None)
    if n == 0:
        raise ValueError("invalid batch/degree/schedule")
    return int(n)


def default_schedule() -> Schedule:
    s = Schedule()
    check(_lib.load().lsefit_default_schedule(ctypes.byref(s)), "lsefit_default_schedule")
    return s


def set_default_schedule(schedule: Schedule | dict | None):
    if isinstance(schedule, dict):
        s = Schedule()
        for k, v in schedule.items():
            setattr(s, k, int(v))
        schedule = s
    check(_lib.load().lsefit_set_default_schedule(ctypes.byref(schedule) if schedule is not None else None),
          "lsefit_set_default_schedule")


def device_cus() -> int:
    return int(_lib.load().lsefit_device_cus())


# ---------------------------------------------------------------------------
# single fit
# ---------------------------------------------------------------------------
@dataclass
class FitResult:
    coef: torch.Tensor       # a_0..a_m, x-basis, float64 (device)
    coef_t: torch.Tensor | None   # b_0..b_m, t-basis (monomial basis only)
    status: torch.Tensor     # int32 [1] (device)
    moments: torch.Tensor    # [c, s, S_0..S_2m, T_0..T_m] (Chebyshev: C_k, D_j in their place)
    ws: torch.Tensor | None = None   # the workspace the fit left its records in
    options: Options | None = None
    coef_cheb: torch.Tensor | None = None   # c_0..c_m of sum_j c_j T_j(t) (Chebyshev basis)

    @property
    def center(self):
        return float(self.moments[0])

    @property
    def scale(self):
        return float(self.moments[1])


def fit_moments(x, y, degree, precision="f64", center=None, scale=None, ws=None, solver="gepp",
                basis="monomial"):
    """Power sums [c, s, S_0..S_2m, T_0..T_m] of t = (x - c)/s (one streaming
    pass); for basis="chebyshev" the sums C_k of T_k(t) and D_j of y T_j(t)."""
    _check_points(x, y)
    L = _lib.load()
    o = options(degree, precision, 0, center, scale, solver, basis)
    nbytes = workspace_bytes(1, degree)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
    mom = torch.empty(3 * degree + 4, dtype=torch.float64, device=x.device)
    check(L.fit_moments(_ptr(x), _ptr(y), x.numel(), _DT[x.dtype], ctypes.byref(o), _ptr(ws), ws.numel(),
                        _ptr(mom), _stream(x.device)), "fit_moments")
    return mom, ws


def fit_solve(moments, degree, precision="f64", refine=1, x=None, y=None, ws=None, center=None, scale=None,
              solver="gepp", basis="monomial"):
    """Elimination on the Hankel system, optional refinement, x-basis
    coefficients; returns ([a | b], status) ([c | a] for basis="chebyshev")."""
    L = _lib.load()
    o = options(degree, precision, refine, center, scale, solver, basis)
    dev = moments.device
    nbytes = workspace_bytes(1, degree)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    coef = torch.empty(2 * (degree + 1), dtype=torch.float64, device=dev)
    status = torch.empty(1, dtype=torch.int32, device=dev)
    n = x.numel() if x is not None else 0
    dt = _DT[x.dtype] if x is not None else _lib.F32
    check(L.fit_solve(_ptr(moments), ctypes.byref(o), _ptr(x), _ptr(y), n, dt, _ptr(ws), ws.numel(), _ptr(coef),
                      _ptr(status), _stream(dev)), "fit_solve")
    return coef, status


def fit(x, y, degree: int, precision: str = "f64", refine: int = 1, center=None, scale=None,
        ws=None, solver: str = "gepp", basis: str = "monomial") -> FitResult:
    """Least-squares polynomial fit of degree ``degree`` (coefficients a_0 first), one fused call.

    basis="chebyshev" (degree up to 16): the normal equations are written in
    Chebyshev polynomials of t = (x - center)/scale; ``coef_cheb`` holds their
    coefficients c, ``coef`` the x-basis a, and ``coef_t`` is None."""
    _check_points(x, y)
    L = _lib.load()
    o = options(degree, precision, refine, center, scale, solver, basis)
    nbytes = workspace_bytes(1, degree)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
    m1 = degree + 1
    coef = torch.empty(2 * m1, dtype=torch.float64, device=x.device)
    status = torch.empty(1, dtype=torch.int32, device=x.device)
    mom = torch.empty(3 * degree + 4, dtype=torch.float64, device=x.device)
    check(L.fit_single(_ptr(x), _ptr(y), x.numel(), _DT[x.dtype], ctypes.byref(o), _ptr(ws), ws.numel(),
                       _ptr(coef), _ptr(status), _ptr(mom), _stream(x.device)), "fit_single")
    if basis == "chebyshev":
        return FitResult(coef[m1:], None, status, mom, ws, o, coef_cheb=coef[:m1])
    return FitResult(coef[:m1], coef[m1:], status, mom, ws, o)


@dataclass
class QRResult:
    coef: torch.Tensor       # a_0..a_m, x-basis, float64 (device)
    coef_t: torch.Tensor     # b_0..b_m, t-basis
    status: torch.Tensor     # int32 [1]
    info: torch.Tensor       # [c, s, sum of squared residuals]
    ws: torch.Tensor | None = None
    options: Options | None = None

    @property
    def center(self):
        return float(self.info[0])

    @property
    def scale(self):
        return float(self.info[1])

    @property
    def sse(self):
        return float(self.info[2])


def fit_qr(x, y, degree: int, center=None, scale=None, ws=None) -> QRResult:
    """The same fit through a streaming QR factorisation (error ~ cond(V), not cond(V)^2)."""
    _check_points(x, y)
    L = _lib.load()
    o = options(degree, "f64", 0, center, scale)
    nbytes = workspace_bytes(1, degree)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
    m1 = degree + 1
    coef = torch.empty(2 * m1, dtype=torch.float64, device=x.device)
    status = torch.empty(1, dtype=torch.int32, device=x.device)
    info = torch.empty(3, dtype=torch.float64, device=x.device)
    check(L.fit_qr(_ptr(x), _ptr(y), x.numel(), _DT[x.dtype], ctypes.byref(o), _ptr(ws), ws.numel(), _ptr(coef),
                   _ptr(status), _ptr(info), _stream(x.device)), "fit_qr")
    return QRResult(coef[:m1], coef[m1:], status, info, ws, o)


def fit_qr_batched(x, y, offsets, degrees, max_degree: int, center=None, scale=None, coef_stride=None, ws=None,
                   out=None):
    """Independent fits over CSR segments through the streaming QR route;
    returns (coef [B, stride], status [B], sse [B], ws)."""
    _check_batch(x, y, offsets, degrees)
    L = _lib.load()
    B = degrees.numel()
    o = options(max_degree, "f64", 0, center, scale)
    stride = coef_stride or (max_degree + 1)
    if out is None:
        coef = torch.zeros((B, stride), dtype=torch.float64, device=x.device)
        status = torch.empty(B, dtype=torch.int32, device=x.device)
        sse = torch.empty(B, dtype=torch.float64, device=x.device)
    else:
        coef, status, sse = out
    nbytes = workspace_bytes(max(B, 1), max_degree)
    if ws is None or ws.numel() < nbytes:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
    check(L.fit_qr_batched(_ptr(x), _ptr(y), _ptr(offsets), _ptr(degrees), B, _DT[x.dtype], ctypes.byref(o),
                           _ptr(ws), ws.numel(), _ptr(coef), stride, _ptr(status), _ptr(sse), _stream(x.device)),
          "fit_qr_batched")
    return coef, status, sse, ws


def fit_split(x, y, degree: int, precision: str = "f64", refine: int = 1, center=None, scale=None,
              solver: str = "gepp", basis: str = "monomial") -> FitResult:
    """The same fit through the two-call form (fit_moments, then fit_solve)."""
    mom, ws = fit_moments(x, y, degree, precision, center, scale, solver=solver, basis=basis)
    coef, status = fit_solve(mom, degree, precision, refine, x, y, ws, center, scale, solver=solver, basis=basis)
    m1 = degree + 1
    o = options(degree, precision, refine, center, scale, solver, basis)
    if basis == "chebyshev":
        return FitResult(coef[m1:], None, status, mom, ws, o, coef_cheb=coef[:m1])
    return FitResult(coef[:m1], coef[m1:], status, mom, ws, o)


def residuals(x, y, result: FitResult, store: bool = False):
    """Sum of squared residuals of a single fit (and, with store=True, every
    residual e_i = y_i - f(x_i)); `result` is what fit() returned for x, y."""
    _check_points(x, y)
    L = _lib.load()
    sse = torch.empty(1, dtype=torch.float64, device=x.device)
    res = torch.empty_like(x) if store else None
    check(L.fit_residuals(_ptr(x), _ptr(y), None, None, 1, x.numel(), _DT[x.dtype], ctypes.byref(result.options),
                          None, _ptr(result.ws), result.ws.numel(), _ptr(sse), _ptr(res), _stream(x.device)),
          "fit_residuals")
    return sse, res


def residuals_batched(x, y, offsets, degrees, max_degree: int, ws=None, plan=None, store: bool = False,
                      precision: str = "f64", center=None, scale=None, solver: str = "gepp", basis: str = "monomial"):
    """Per-fit sums of squared residuals after fit_batched on the same workspace or plan."""
    _check_batch(x, y, offsets, degrees)
    L = _lib.load()
    B = degrees.numel()
    o = options(max_degree, precision, 0, center, scale, solver, basis)
    sse = torch.empty(B, dtype=torch.float64, device=x.device)
    res = torch.empty_like(x) if store else None
    check(L.fit_residuals(_ptr(x), _ptr(y), _ptr(offsets), _ptr(degrees), B, x.numel(), _DT[x.dtype],
                          ctypes.byref(o), plan.handle if plan is not None else None,
                          _ptr(ws) if plan is None else None, ws.numel() if (plan is None and ws is not None) else 0,
                          _ptr(sse), _ptr(res), _stream(x.device)), "fit_residuals")
    return sse, res


# ---------------------------------------------------------------------------
# batched fits
# ---------------------------------------------------------------------------
class Plan:
    """A tuned schedule, its own workspace and a captured HIP graph for
    repeated batched calls of one shape (fit_plan_* in the C ABI)."""

    def __init__(self, batch: int, max_degree: int, dtype=torch.float32, precision: str = "f64"):
        self._L = _lib.load()
        h = ctypes.c_void_p()
        check(self._L.fit_plan_create(ctypes.byref(h), int(batch), int(max_degree), _DT[dtype], _PREC[precision]),
              "fit_plan_create")
        self.handle = h
        self.batch, self.max_degree, self.dtype, self.precision = batch, max_degree, dtype, precision

    def close(self):
        if self.handle:
            self._L.fit_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def schedule(self) -> dict:
        s = Schedule()
        check(self._L.fit_plan_get_schedule(self.handle, ctypes.byref(s)), "fit_plan_get_schedule")
        return s.as_dict()

    def set_schedule(self, sched: dict):
        s = Schedule()
        for k, v in sched.items():
            setattr(s, k, int(v))
        check(self._L.fit_plan_set_schedule(self.handle, ctypes.byref(s)), "fit_plan_set_schedule")

    def set_graph(self, enable: bool):
        """Replay a captured graph (True) or launch eagerly (False); tune() then keeps this form."""
        check(self._L.fit_plan_set_graph(self.handle, 1 if enable else 0), "fit_plan_set_graph")

    @property
    def graph(self) -> bool:
        """Whether calls replay a captured graph (tune() picks the faster form unless set_graph chose)."""
        e = ctypes.c_int32(0)
        check(self._L.fit_plan_get_graph(self.handle, ctypes.byref(e)), "fit_plan_get_graph")
        return bool(e.value)

    def set_tune_cache(self, path):
        """Schedule cache file of tune() (None turns it off); see fit_plan_set_tune_cache."""
        check(self._L.fit_plan_set_tune_cache(self.handle, None if path is None else os.fsencode(path)),
              "fit_plan_set_tune_cache")

    def tune(self, x, y, offsets, degrees, max_degree=None, precision=None, refine=1, center=None, scale=None,
             reps=3, solver="gepp", basis="monomial") -> float:
        _check_batch(x, y, offsets, degrees)
        m = self.max_degree if max_degree is None else max_degree
        o = options(m, precision or self.precision, refine, center, scale, solver, basis)
        B = degrees.numel()
        coef = torch.empty(B * (m + 1), dtype=torch.float64, device=x.device)
        status = torch.empty(B, dtype=torch.int32, device=x.device)
        best = ctypes.c_double(0.0)
        check(self._L.fit_plan_tune(self.handle, _ptr(x), _ptr(y), _ptr(offsets), _ptr(degrees), B, ctypes.byref(o),
                                    _ptr(coef), m + 1, _ptr(status), _stream(x.device), int(reps),
                                    ctypes.byref(best)), "fit_plan_tune")
        return best.value


def _check_batch(x, y, offsets, degrees):
    _check_points(x, y)
    if offsets.dtype != torch.int64 or degrees.dtype != torch.int32:
        raise TypeError("offsets must be int64 and degrees int32")
    if offsets.device != x.device or degrees.device != x.device:
        raise ValueError("offsets and degrees must be on the device of x")
    if offsets.dim() != 1 or degrees.dim() != 1 or offsets.numel() != degrees.numel() + 1:
        raise ValueError("offsets must have one more entry than degrees")
    if not (offsets.is_contiguous() and degrees.is_contiguous()):
        raise ValueError("offsets and degrees must be contiguous")


def fit_batched(x, y, offsets, degrees, max_degree: int, precision: str = "f64", refine: int = 1,
                center=None, scale=None, plan: Plan | None = None, coef_stride: int | None = None,
                ws: torch.Tensor | None = None, out=None, solver: str = "gepp", basis: str = "monomial",
                output_basis: str = "x"):
    """Independent fits over CSR segments; returns (coef [B, stride], status [B], ws).

    output_basis="x_and_t" (monomial basis): each row is [a_0..a_M | b_0..b_M | c | s]
    (M = max_degree, stride 2M + 4 by default): the x-basis coefficients, the
    t-basis coefficients of t = (x - c)/s and the fit's c and s."""
    _check_batch(x, y, offsets, degrees)
    L = _lib.load()
    B = degrees.numel()
    o = options(max_degree, precision, refine, center, scale, solver, basis, output_basis)
    t_out = output_basis == "x_and_t" and basis == "monomial"
    stride = coef_stride or (2 * max_degree + 4 if t_out else max_degree + 1)
    if out is None:
        coef = torch.zeros((B, stride), dtype=torch.float64, device=x.device)
        status = torch.empty(B, dtype=torch.int32, device=x.device)
    else:
        coef, status = out
    if plan is None:
        nbytes = workspace_bytes(max(B, 1), max_degree)
        if ws is None or ws.numel() < nbytes:
            ws = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
    check(L.fit_batched(_ptr(x), _ptr(y), _ptr(offsets), _ptr(degrees), B, _DT[x.dtype], ctypes.byref(o),
                        plan.handle if plan is not None else None, _ptr(ws) if plan is None else None,
                        ws.numel() if plan is None else 0, _ptr(coef), stride, _ptr(status), _stream(x.device)),
          "fit_batched")
    return coef, status, ws


def fit_backward(x, y, offsets, degrees, max_degree, grad_coef, ws=None, plan=None, precision="f64",
                 center=None, scale=None, solver="gepp", basis="monomial"):
    """dL/dx, dL/dy from dL/da (grad_coef [B, stride] float64) after fit_batched; for
    basis="chebyshev" (given center and scale) grad_coef is dL/dc of the Chebyshev coefficients."""
    _check_batch(x, y, offsets, degrees)
    L = _lib.load()
    B = degrees.numel()
    o = options(max_degree, precision, 0, center, scale, solver, basis)
    grad_coef = grad_coef.to(torch.float64).contiguous()
    gx = torch.empty_like(x)
    gy = torch.empty_like(y)
    check(L.fit_backward(_ptr(x), _ptr(y), _ptr(offsets), _ptr(degrees), B, _DT[x.dtype], ctypes.byref(o),
                         plan.handle if plan is not None else None, _ptr(ws) if plan is None else None,
                         ws.numel() if (plan is None and ws is not None) else 0, _ptr(grad_coef),
                         grad_coef.shape[-1], _ptr(gx), _ptr(gy), _stream(x.device)), "fit_backward")
    return gx, gy


class LseFit(torch.autograd.Function):
    """Differentiable batched fit: coef = LseFit.apply(x, y, offsets, degrees, max_degree, precision,
    center, scale, basis).  The backward is the library's adjoint kernel (the Chebyshev basis
    needs a given center and scale)."""

    @staticmethod
    def forward(ctx, x, y, offsets, degrees, max_degree, precision="f64", center=None, scale=None,
                basis="monomial"):
        coef, status, ws = fit_batched(x, y, offsets, degrees, max_degree, precision, 1, center, scale,
                                       basis=basis)
        ctx.save_for_backward(x, y, offsets, degrees)
        ctx.ws = ws
        ctx.cfg = (max_degree, precision, center, scale, basis)
        ctx.status = status
        return coef

    @staticmethod
    def backward(ctx, grad_coef):
        x, y, offsets, degrees = ctx.saved_tensors
        max_degree, precision, center, scale, basis = ctx.cfg
        gx, gy = fit_backward(x, y, offsets, degrees, max_degree, grad_coef, ws=ctx.ws, precision=precision,
                              center=center, scale=scale, basis=basis)
        return gx, gy, None, None, None, None, None, None, None


def lsefit(x, y, offsets, degrees, max_degree: int, precision: str = "f64", center=None, scale=None,
           basis: str = "monomial"):
    """Differentiable batched fit (autograd through the hand-written adjoint)."""
    return LseFit.apply(x, y, offsets, degrees, max_degree, precision, center, scale, basis)
