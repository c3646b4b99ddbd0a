"""Host-side checks of the C-ABI library (no GPU needed).

The library must load, export every function include/hpnfft.h declares, and
reject invalid plans before touching the device.  The window and roll-off
tables (host code) are pinned by quadrature and finite differences.
"""
import ctypes
import math

import numpy as np
import pytest

from paper_2001_01583_amd import hpnfft as H


@pytest.fixture(scope="module")
def lib():
    return H._load()


def _create(lib, N=(16, 16, 16), M=100, sigma=2.0, m=4, window=0, prec=0, flags=0, d=3):
    h = ctypes.c_void_p()
    arr = (ctypes.c_int64 * len(N))(*N)
    rc = lib.hpnfft_plan_create(ctypes.byref(h), d, arr, M, sigma, m, window, prec, flags)
    return rc, h


def test_every_declared_symbol_is_exported(lib):
    names = H.declared_symbols()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_strerror_never_null(lib):
    for c in (0, -1, -2, -3, -4, -5, -99, 7):
        assert lib.hpnfft_strerror(c)


@pytest.mark.parametrize("kw", [
    dict(d=2), dict(N=(15, 16, 16)), dict(N=(0, 16, 16)), dict(M=0), dict(m=0), dict(m=9),
    dict(sigma=1.7),            # 1.7 * 16 is not an integer
    dict(sigma=0.5), dict(window=3), dict(prec=2), dict(flags=8),
    dict(N=(20, 16, 16)),       # n = 40 has a factor 5
    dict(N=(2, 16, 16), m=4),   # 2m > n
    dict(N=(1024, 16, 16)),     # n > 1024
])
def test_invalid_plans_rejected(lib, kw):
    rc, h = _create(lib, **kw)
    assert rc == H.EINVAL
    assert not h.value


@pytest.mark.parametrize("N,sigma", [((16, 16, 16), 2.0), ((16, 12, 24), 2.0), ((32, 48, 64), 2.0),
                                     ((16, 16, 16), 1.5), ((32, 32, 32), 3.0)])
def test_valid_plans_created(lib, N, sigma):
    rc, h = _create(lib, N=N, sigma=sigma)
    assert rc == H.OK
    n = (ctypes.c_int64 * 3)()
    M = ctypes.c_int64()
    assert lib.hpnfft_plan_info(h, n, ctypes.byref(M)) == H.OK
    assert tuple(n) == tuple(int(round(sigma * v)) for v in N) and M.value == 100
    sz = ctypes.c_size_t()
    assert lib.hpnfft_workspace_size(h, ctypes.byref(sz)) == H.OK and sz.value > 0
    assert lib.hpnfft_plan_destroy(h) == H.OK


def test_call_order_enforced(lib):
    rc, h = _create(lib)
    assert rc == H.OK
    dummy = ctypes.c_void_p(0x1000)
    # no workspace yet: points cannot be set; no points: transforms refuse
    assert lib.hpnfft_set_points(h, dummy) == H.ESTATE
    assert lib.hpnfft_adjoint(h, dummy, dummy) == H.ESTATE
    assert lib.hpnfft_forward(h, dummy, dummy) == H.ESTATE
    # gradient needs the flag
    assert lib.hpnfft_adjoint_backward(h, dummy, dummy, dummy, dummy) == H.EINVAL
    # null arguments
    assert lib.hpnfft_adjoint(h, None, dummy) == H.EINVAL
    assert lib.hpnfft_set_workspace(h, None, 0) == H.EINVAL
    assert lib.hpnfft_set_workspace(h, ctypes.c_void_p(0x1001), 1 << 30) == H.EINVAL  # misaligned
    assert lib.hpnfft_set_workspace(h, dummy, 16) == H.ENOMEM
    assert lib.hpnfft_batch_launch(h) == H.ESTATE
    assert lib.hpnfft_plan_destroy(h) == H.OK
    assert lib.hpnfft_plan_destroy(None) == H.OK


def test_tiling_limits(lib):
    rc, h = _create(lib, m=8)
    assert rc == H.OK
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    assert lib.hpnfft_get_tiles(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)) == H.OK
    assert 4 <= a.value <= 32 and b.value >= 2 and c.value % 64 == 0
    assert lib.hpnfft_set_tiles(h, 32, 64, 1024) == H.EINVAL   # LDS overflow at m = 8
    assert lib.hpnfft_set_tiles(h, 8, 16, 1000) == H.EINVAL    # not a multiple of 64
    assert lib.hpnfft_set_tiles(h, 8, 8, 512) == H.OK
    lib.hpnfft_plan_destroy(h)


def test_batch_offsets(lib):
    h = ctypes.c_void_p()
    N = (ctypes.c_int64 * 6)(16, 16, 16, 32, 32, 32)
    M = (ctypes.c_int64 * 2)(10, 20)
    assert lib.hpnfft_batch_create(ctypes.byref(h), 2, N, M, 2.0, 4, 0, 1, 0) == H.OK
    po, fo = ctypes.c_int64(), ctypes.c_int64()
    assert lib.hpnfft_batch_offsets(h, 1, ctypes.byref(po), ctypes.byref(fo)) == H.OK
    assert (po.value, fo.value) == (10, 16 ** 3)
    assert lib.hpnfft_batch_offsets(h, 2, ctypes.byref(po), ctypes.byref(fo)) == H.EINVAL
    lib.hpnfft_plan_destroy(h)


@pytest.mark.parametrize("m", [2, 4, 6, 8])
def test_rolloff_is_fourier_coefficient_of_window(m):
    """The Scaling step divides by c_k, the Fourier coefficient of the
    periodised window (Section 2).  Check the host tables against trapezoid
    quadrature of the tabulated window itself.  The I0 pair holds up to the
    truncation of the window at |t| = m, a relative error of order
    b m / sinh(b m) (1.5e-3 at m = 2, 2.5e-7 at m = 4, 3e-15 at m = 8)."""
    sigma, n, N = 2.0, 64, 32
    ro = H.window_rolloff(m, sigma, n, N)
    t = np.linspace(-m, m, 200001)
    phi, _ = H.window_eval(m, sigma, t)
    wts = np.full(t.size, t[1] - t[0])
    wts[0] = wts[-1] = (t[1] - t[0]) / 2
    b = math.pi * (2 - 1 / sigma)
    tol = max(5e-8, b * m / math.sinh(b * m))
    for k in (-N // 2, -5, 0, 3, N // 2 - 1):
        ck = np.sum(wts * phi * np.cos(2 * np.pi * k * t / n))
        assert abs(ck * ro[k + N // 2] - 1.0) < tol


@pytest.mark.parametrize("m", [1, 4, 8])
def test_window_derivative_matches_finite_differences(m):
    t = np.array([-m + 0.3, -1.7, -0.2, 0.0, 0.45, m - 0.01, m - 1e-9])
    t = t[np.abs(t) <= m]
    h = 1e-6
    p1, d = H.window_eval(m, 2.0, t)
    pp, _ = H.window_eval(m, 2.0, t + h)
    pm, _ = H.window_eval(m, 2.0, t - h)
    fd = (pp - pm) / (2 * h)
    ok = np.abs(t) < m - 2 * h
    assert np.allclose(d[ok], fd[ok], rtol=1e-6, atol=1e-8)
    assert abs(H.window_eval(m, 2.0, [0.0])[0][0] - 1.0) < 1e-15  # normalised peak


def test_window_is_kaiser_bessel_closed_form():
    """phi(t) = sinh(b r)/r normalised, b = pi (2 - 1/sigma): one closed-form
    value per m against the library."""
    for m in (2, 5, 8):
        b = math.pi * (2 - 1 / 2.0)
        t = 0.37 * m
        r = math.sqrt(m * m - t * t)
        ref = (math.sinh(b * r) / r) / (math.sinh(b * m) / m)
        got = H.window_eval(m, 2.0, [t])[0][0]
        assert abs(got / ref - 1) < 1e-13
