"""Seeded synthetic inputs for the moment-pass least-squares fit.

This module only draws data.  It holds none of the fitting arithmetic
(no power sums, no normal equations, no elimination), so both the HIP path
and the CPU oracle may consume what it produces without sharing any of the
method.  The polynomial evaluation below builds the *noisy observations*
y = p(x) + noise; it is data generation, not the fit.

Every workload draws from three independent PCG64 streams spawned from one
``numpy.random.SeedSequence``: one for the true coefficients, one for x, one
for the noise.  Drawing a stream in chunks yields the same values as drawing
it at once, so large inputs are generated chunk by chunk without changing
them.  Values are computed in float64 and then cast to the storage dtype;
the cast values are the exact inputs of a fit.

The five workloads follow the shapes the method is meant for (a polynomial
of low degree fitted to many points, Sec. I and Sec. II of the paper):

* ``linear_f64``      n = 1e6 FP64, x ~ U[0,10], y = 2 + 3x + N(0, 0.5^2), m = 1
* ``cubic_f32``       n = 1e8 FP32, x ~ U[-1,1], a ~ N(0,1)^4, noise N(0, 0.01^2), m = 3
* ``ragged_batch``    65,536 fits, lengths log-uniform in [16, 65536], degree
                      U{1,2,3}, x ~ U[-5,5] FP32, a ~ N(0,1), noise N(0, 0.1^2)
* ``grad_batch``      4,096 fits x 4,096 points, m = 2, x ~ U[-1,1] FP32,
                      noise N(0, 0.05^2), targets a_target ~ N(0,1) (FP64)
* ``shifted_quintic`` n = 1e7 FP32, x ~ U[1000,1001], y = poly of degree 5 in
                      (x - 1000.5) with coefficients N(0,1), noise N(0, 1e-4^2)

and one for the higher degrees the Chebyshev basis serves (beyond Sec. II's
low orders):

* ``runge``           n = 1e8 FP32, x ~ U[-1,1], y = 1/(1 + 25x^2) + N(0, 1e-3^2),
                      m = 12

Inputs beyond 2^31 points (64-bit indexing) use a deterministic pattern whose
sums have closed forms: ``periodic_points`` (x_i = (2 (i mod 1024) - 1023) /
1024, y_i = (i mod 1021) / 1024, both exact in float32).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

CHUNK = 1 << 22  # points drawn per chunk; does not change the values


def _streams(seed: int, k: int = 3):
    ss = np.random.SeedSequence(int(seed))
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(k)]


def _horner(coef: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Evaluate sum_j coef[j] u^j (ascending order) in float64 -- data generation only."""
    out = np.zeros_like(u)
    for c in coef[::-1]:
        out = out * u + c
    return out


@dataclass
class SingleFit:
    """One fit: x, y of one storage dtype plus the degree and the generating polynomial."""
    name: str
    x: np.ndarray
    y: np.ndarray
    degree: int
    true_coef: np.ndarray          # generating coefficients (ascending), only a sanity check
    true_center: float = 0.0       # the generating polynomial is in (x - true_center)
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


@dataclass
class BatchFit:
    """Ragged fits concatenated in CSR order: fit f owns points offsets[f]:offsets[f+1]."""
    name: str
    x: np.ndarray
    y: np.ndarray
    offsets: np.ndarray            # int64 [B+1]
    degrees: np.ndarray            # int32 [B]
    true_coef: list                # per fit, ascending, only a sanity check
    target: np.ndarray | None = None   # FP64 [B, max_degree+1] for the loss sum ||a - target||^2
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def batch(self) -> int:
        return int(self.degrees.shape[0])

    @property
    def total_points(self) -> int:
        return int(self.offsets[-1])


def _single(name, n, seed, lo, hi, dtype, coef_fn, noise_sd, degree, center=0.0):
    r_coef, r_x, r_noise = _streams(seed)
    coef = coef_fn(r_coef)
    x_out = np.empty(n, dtype=dtype)
    y_out = np.empty(n, dtype=dtype)
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        xs = r_x.uniform(lo, hi, e - s)
        ys = _horner(coef, xs - center) + r_noise.normal(0.0, noise_sd, e - s)
        x_out[s:e] = xs
        y_out[s:e] = ys
    return SingleFit(name, x_out, y_out, degree, np.asarray(coef, dtype=np.float64),
                     center, seed, {"lo": lo, "hi": hi, "noise_sd": noise_sd})


def linear_f64(n: int = 1_000_000, seed: int = 1000) -> SingleFit:
    """m = 1, FP64 storage, y = 2 + 3x + N(0, 0.5^2), x ~ U[0, 10]."""
    return _single("linear_f64", n, seed, 0.0, 10.0, np.float64,
                   lambda r: np.array([2.0, 3.0]), 0.5, 1)


def cubic_f32(n: int = 100_000_000, seed: int = 2000) -> SingleFit:
    """m = 3, FP32 storage, x ~ U[-1, 1], coefficients N(0,1), noise N(0, 0.01^2)."""
    return _single("cubic_f32", n, seed, -1.0, 1.0, np.float32,
                   lambda r: r.standard_normal(4), 0.01, 3)


def shifted_quintic(n: int = 10_000_000, seed: int = 5000) -> SingleFit:
    """m = 5, FP32 storage, x ~ U[1000, 1001], polynomial in (x - 1000.5), noise N(0, 1e-4^2)."""
    return _single("shifted_quintic", n, seed, 1000.0, 1001.0, np.float32,
                   lambda r: r.standard_normal(6), 1e-4, 5, center=1000.5)


def runge(n: int = 100_000_000, seed: int = 6000, degree: int = 12, lo: float = -1.0, hi: float = 1.0,
          dtype=np.float32, noise_sd: float = 1e-3) -> SingleFit:
    """Higher-degree workload: y = 1 / (1 + 25 u^2) + N(0, noise_sd^2), u the
    position of x in [lo, hi] mapped to [-1, 1], x ~ U[lo, hi]; fitted with
    degree ``degree`` (no polynomial generates it: true_coef is empty)."""
    _, r_x, r_noise = _streams(seed)
    x_out = np.empty(n, dtype=dtype)
    y_out = np.empty(n, dtype=dtype)
    mid, half = 0.5 * (lo + hi), 0.5 * (hi - lo)
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        xs = r_x.uniform(lo, hi, e - s)
        u = (xs - mid) / half
        x_out[s:e] = xs
        y_out[s:e] = 1.0 / (1.0 + 25.0 * u * u) + r_noise.normal(0.0, noise_sd, e - s)
    return SingleFit("runge", x_out, y_out, degree, np.zeros(0), 0.0, seed,
                     {"lo": lo, "hi": hi, "noise_sd": noise_sd})


def ragged_lengths(batch: int, lo: int, hi: int, rng) -> np.ndarray:
    """L = floor(exp(U(ln lo, ln hi))) clamped to [lo, hi] (log-uniform lengths)."""
    u = rng.uniform(np.log(lo), np.log(hi), batch)
    return np.clip(np.floor(np.exp(u)), lo, hi).astype(np.int64)


def _batch(name, lengths, degrees, seed, lo, hi, dtype, noise_sd, rngs, with_target=False):
    r_coef, r_x, r_noise = rngs
    B = lengths.shape[0]
    offsets = np.zeros(B + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    total = int(offsets[-1])
    coefs = [r_coef.standard_normal(int(d) + 1) for d in degrees]
    x_out = np.empty(total, dtype=dtype)
    y_out = np.empty(total, dtype=dtype)
    # draw x and noise chunk by chunk over the concatenated point range, then
    # add each fit's polynomial; the fit loop only slices.
    f = 0
    for s in range(0, total, CHUNK):
        e = min(total, s + CHUNK)
        xs = r_x.uniform(lo, hi, e - s)
        ys = r_noise.normal(0.0, noise_sd, e - s)
        while f < B and offsets[f] < e:
            a = max(int(offsets[f]), s)
            b = min(int(offsets[f + 1]), e)
            if b > a:
                ys[a - s:b - s] += _horner(coefs[f], xs[a - s:b - s])
            if offsets[f + 1] <= e:
                f += 1
            else:
                break
        x_out[s:e] = xs
        y_out[s:e] = ys
    target = None
    if with_target:
        target = r_coef.standard_normal((B, int(degrees.max()) + 1))
    return BatchFit(name, x_out, y_out, offsets, degrees.astype(np.int32), coefs, target, seed,
                    {"lo": lo, "hi": hi, "noise_sd": noise_sd})


def ragged_batch(batch: int = 65_536, min_len: int = 16, max_len: int = 65_536,
                 degrees=(1, 2, 3), seed: int = 3000) -> BatchFit:
    """Ragged fits of log-uniform length and degree uniform over ``degrees``."""
    r_coef, r_x, r_noise, r_len = _streams(seed, 4)
    lengths = ragged_lengths(batch, min_len, max_len, r_len)
    deg = r_len.choice(np.asarray(degrees, dtype=np.int32), size=batch)
    return _batch("ragged_batch", lengths, deg, seed, -5.0, 5.0, np.float32, 0.1,
                  (r_coef, r_x, r_noise))


def grad_batch(batch: int = 4096, length: int = 4096, degree: int = 2, seed: int = 4000) -> BatchFit:
    """Equal-length fits with targets for the loss sum_f ||a_f - a_target_f||^2."""
    r_coef, r_x, r_noise = _streams(seed)
    lengths = np.full(batch, length, dtype=np.int64)
    deg = np.full(batch, degree, dtype=np.int32)
    return _batch("grad_batch", lengths, deg, seed, -1.0, 1.0, np.float32, 0.05,
                  (r_coef, r_x, r_noise), with_target=True)


# --- the paper's worked example (Table I, Sec. III) --------------------------
# Six (x, y) pairs printed in Table I; used as a fixed test vector.
TABLE_I_X = ("39.206", "29.74", "21.31", "12.087", "1.812", "0.001")
TABLE_I_Y = ("751.912", "567.121", "403.746", "221.738", "18.8418", "1.88672")


def table_i() -> SingleFit:
    x = np.array([float(v) for v in TABLE_I_X])
    y = np.array([float(v) for v in TABLE_I_Y])
    return SingleFit("table_i", x, y, 3, np.zeros(4), 0.0, 0, {})


def random_small(n: int, degree: int, seed: int, lo=-1.0, hi=1.0, noise_sd=0.1,
                 dtype=np.float64, center=0.0) -> SingleFit:
    """Small random fit for parity and edge cases."""
    return _single("random_small", n, seed, lo, hi, dtype,
                   lambda r: r.standard_normal(degree + 1), noise_sd, degree, center)


def random_batch(lengths, degrees, seed: int, lo=-1.0, hi=1.0, noise_sd=0.1,
                 dtype=np.float32, with_target=False) -> BatchFit:
    """A batch with caller-chosen lengths and degrees."""
    lengths = np.asarray(lengths, dtype=np.int64)
    degrees = np.asarray(degrees, dtype=np.int32)
    return _batch("random_batch", lengths, degrees, seed, lo, hi, dtype, noise_sd,
                  _streams(seed), with_target=with_target)


# --- a deterministic pattern for any size --------------------------------------
PERIOD_X = 1024
PERIOD_Y = 1021


def periodic_points_np(lo: int, hi: int):
    """Points lo..hi-1 of the periodic pattern as float32 numpy arrays."""
    i = np.arange(lo, hi, dtype=np.int64)
    x = ((2 * (i % PERIOD_X) - (PERIOD_X - 1)) / PERIOD_X).astype(np.float32)
    y = ((i % PERIOD_Y) / 1024.0).astype(np.float32)
    return x, y


def periodic_points(n: int, device, chunk: int = 1 << 27):
    """The first n points of the periodic pattern as float32 tensors on `device`,
    written chunk by chunk (64-bit indices, no host copy)."""
    import torch
    x = torch.empty(n, dtype=torch.float32, device=device)
    y = torch.empty(n, dtype=torch.float32, device=device)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        i = torch.arange(lo, hi, dtype=torch.int64, device=device)
        x[lo:hi] = ((2 * (i % PERIOD_X) - (PERIOD_X - 1)).to(torch.float64) / PERIOD_X).to(torch.float32)
        y[lo:hi] = ((i % PERIOD_Y).to(torch.float64) / 1024.0).to(torch.float32)
        del i
    return x, y

