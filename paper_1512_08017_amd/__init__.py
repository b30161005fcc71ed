"""MI355X-native moment-pass least-squares polynomial fit (gfx950 HIP + C ABI).

Importing the package loads nothing; the HIP library ``liblsefit.so`` is
loaded on the first call and its absence is an error (there is no CPU path).
"""
from __future__ import annotations

__all__ = ["fit", "fit_split", "fit_moments", "fit_solve", "fit_qr", "fit_qr_batched", "fit_batched", "fit_backward", "lsefit", "LseFit",
           "Plan", "FitResult", "QRResult", "residuals", "residuals_batched", "default_schedule", "set_default_schedule",
           "workspace_bytes", "device_cus", "LsefitError"]


def __getattr__(name):
    if name in __all__:
        from . import api, _lib
        if name == "LsefitError":
            return _lib.LsefitError
        return getattr(api, name)
    raise AttributeError(name)
