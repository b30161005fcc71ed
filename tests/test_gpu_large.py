"""Sizes beyond 2^31 points: every streaming pass indexes points with 64-bit
integers.  The inputs are the periodic pattern of the workloads module
(x_i = (2 (i mod 1024) - 1023)/1024, y_i = (i mod 1021)/1024, exact in
float32), whose power sums have an exact closed form
(oracle.exact.periodic_power_sums).  Checks: the float64 form's power sums
against that closed form, and the coefficients of each route (power basis in
float64 and compensated float32, Chebyshev basis, streaming QR, single and
batched with a fit across index 2^31) against the exact minimiser of Sec. II
computed from the exact sums.  Launched with the default schedule, as the
benchmark is."""
import numpy as np
import pytest

from gpu_common import announce, normwise, torch
from oracle import exact
from paper_1512_08017_amd import workloads as W

pytestmark = pytest.mark.gpu

lf = pytest.importorskip("paper_1512_08017_amd")

N = (1 << 31) + 777
M = 3
CUTS = [0, (1 << 31) - 1000, (1 << 31) + 5, N]   # the middle fit spans index 2^31
DEGS = [3, 2, 3]


@pytest.fixture(scope="module")
def big():
    announce(f"periodic inputs, n = {N}")
    x, y = W.periodic_points(N, torch.device("cuda:0"))
    torch.cuda.synchronize()
    yield x, y
    del x, y
    torch.cuda.empty_cache()


def exact_fit(lo, hi, m):
    S, T = exact.periodic_power_sums(lo, hi, m)
    b, singular = exact.solve_from_sums(S, T, m)
    assert not singular
    return S, T, np.array([float(v) for v in b])   # c = 0, s = 1: a = b


def test_power_sums_and_fit_beyond_2_31(big):
    announce("float64 form, n > 2^31")
    x, y = big
    S, T, a = exact_fit(0, N, M)
    r = lf.fit(x, y, M, center=0.0, scale=1.0)
    torch.cuda.synchronize()
    assert int(r.status.cpu()[0]) == 0
    mom = r.moments.cpu().numpy()
    assert mom[2] == N
    # float64 sums of 2^31 terms of magnitude <= 1 in lanes of about 2^14 terms:
    # N * 2^-40 bounds their rounding error, while a point counted twice or
    # skipped moves S_2 by x_i^2 (more than 2^-9 for 95% of the points)
    tol = N * 2.0 ** -40
    for k in range(1, 2 * M + 1):
        assert abs(mom[2 + k] - float(S[k])) <= tol, (k, mom[2 + k], float(S[k]))
    for j in range(M + 1):
        assert abs(mom[3 + 2 * M + j] - float(T[j])) <= tol, (j, mom[3 + 2 * M + j], float(T[j]))
    assert normwise(r.coef.cpu().numpy(), a) <= 1e-9


def test_compensated_float32_beyond_2_31(big):
    announce("compensated float32 form + refinement, n > 2^31")
    x, y = big
    _, _, a = exact_fit(0, N, M)
    r = lf.fit(x, y, M, precision="f32c", center=0.0, scale=1.0)
    assert int(r.status.cpu()[0]) == 0
    assert normwise(r.coef.cpu().numpy(), a) <= 1e-6


def test_chebyshev_and_qr_beyond_2_31(big):
    announce("Chebyshev basis and streaming QR, n > 2^31")
    x, y = big
    _, _, a = exact_fit(0, N, M)
    c = lf.fit(x, y, M, center=0.0, scale=1.0, basis="chebyshev")
    assert int(c.status.cpu()[0]) == 0
    assert normwise(c.coef.cpu().numpy(), a) <= 1e-9
    q = lf.fit_qr(x, y, M, center=0.0, scale=1.0)
    assert int(q.status.cpu()[0]) == 0
    assert normwise(q.coef.cpu().numpy(), a) <= 1e-9


def test_batched_across_2_31(big):
    announce("batched fits across index 2^31")
    x, y = big
    off = torch.tensor(CUTS, dtype=torch.int64, device=x.device)
    deg = torch.tensor(DEGS, dtype=torch.int32, device=x.device)
    coef, status, _ = lf.fit_batched(x, y, off, deg, M, center=0.0, scale=1.0)
    qcoef, qstatus, _, _ = lf.fit_qr_batched(x, y, off, deg, M, center=0.0, scale=1.0)
    coef, status = coef.cpu().numpy(), status.cpu().numpy()
    qcoef, qstatus = qcoef.cpu().numpy(), qstatus.cpu().numpy()
    for f, m in enumerate(DEGS):
        _, _, a = exact_fit(CUTS[f], CUTS[f + 1], m)
        assert status[f] == 0 and qstatus[f] == 0
        assert normwise(coef[f, : m + 1], a) <= 1e-9, f
        assert normwise(qcoef[f, : m + 1], a) <= 1e-9, f
