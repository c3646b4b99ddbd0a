"""The window family of the precision experiment (Section 4, Eq. (9)):
Kaiser-Bessel, Gaussian, cardinal B-spline and sinc-power windows with cut-off
m = 1 .. 15, on the experiment's shape (d = 3, N = 16^3, M = 4096, sigma = 2),
adjoint (Eq. (5)) and forward (Eq. (6)) against the direct FP64 oracle.

Tolerances come from each window's a-priori error bound E(m, sigma) (the
library's hpnfft_window_error_bound; per output |error| <= d E ||input||_1),
turned into a relative l2 bound over the output vector, plus a rounding
floor: the grid's and the FFT's rounding errors (unit roundoff u) reach the
outputs multiplied by the Scaling divisors 1/D(k), so the floor is
2 u A + a base, with A the rms over I_N of prod_t D_t(0)/D_t(k_t).  A grows
with m (the windows are normalised to phi(0) = 1): for Kaiser-Bessel from 34
at m = 8 to 4247 at m = 15, for sinc-power to 83381.  The paper's own curves (its precision figure) carry no numbers, so
they are not compared; the sweep's errors must fall with m until rounding.
"""
import math

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu
WINDOWS = ["kaiser_bessel", "gaussian", "bspline", "sinc_power"]
N = (16, 16, 16)
M = 4096


@pytest.fixture(scope="module")
def H():
    from paper_2001_01583_amd import hpnfft
    hpnfft._load()
    return hpnfft


@pytest.fixture(scope="module")
def case(oracle_mod):
    g = W.rng(12)
    x = W.uniform_points(M, 3, g)
    f = W.complex_normal(M, g)
    fh = W.complex_normal(int(np.prod(N)), g).reshape(N)
    out = {"x": x, "f": f, "fh": fh}
    for prec in ("f64", "f32"):
        fu = f.astype(np.complex64).astype(np.complex128) if prec == "f32" else f
        fhu = fh.astype(np.complex64).astype(np.complex128) if prec == "f32" else fh
        out[prec] = (fu, fhu, oracle_mod.ndft_adjoint(N, x, fu), oracle_mod.ndft_forward(N, x, fhu))
    return out


def _bound_tol(H, window, m, inp, exact, n_out):
    """Relative l2 bound: ||err||_2 <= sqrt(#outputs) * d E ||input||_1."""
    E = H.window_error_bound(m, 2.0, window)
    b = math.sqrt(n_out) * 3 * E * np.abs(inp).sum() / np.linalg.norm(exact)
    return min(b, 1.0)


def _amplification(H, window, m):
    r = H.window_rolloff(m, 2.0, 2 * N[0], N[0], window)
    r = r / r[N[0] // 2]
    return float(np.sqrt(np.mean(r ** 2))) ** 3


def _floor(H, window, m, prec):
    u, base = (2.0 ** -53, 5e-14) if prec == "f64" else (2.0 ** -24, 1e-6)
    return 2 * u * _amplification(H, window, m) + base


def _sweep(H, oracle_mod, case, window, prec):
    x = torch.from_numpy(case["x"]).cuda()
    fu, fhu, ea, ef = case[prec]
    cd = torch.complex128 if prec == "f64" else torch.complex64
    ft = torch.from_numpy(fu).cuda().to(cd)
    fht = torch.from_numpy(fhu).cuda().to(cd)
    errs = []
    for m in range(1, 16):
        plan = H.Plan(N, M, m=m, precision=prec, window=window)
        plan.set_points(x)
        a = plan.adjoint(ft).cpu().numpy().astype(np.complex128)
        b = plan.forward(fht).cpu().numpy().astype(np.complex128)
        e_a = oracle_mod.rel_l2(a, ea)
        e_f = oracle_mod.rel_l2(b, ef)
        floor = _floor(H, window, m, prec)
        tol_a = _bound_tol(H, window, m, fu, ea, ea.size) + floor
        tol_f = _bound_tol(H, window, m, fhu, ef, ef.size) + floor
        print("%s %s m=%2d adjoint %.3e (tol %.1e) forward %.3e (tol %.1e)" % (window, prec, m, e_a, tol_a, e_f,
                                                                              tol_f), flush=True)
        assert e_a <= tol_a and e_f <= tol_f, (window, prec, m, e_a, tol_a, e_f, tol_f)
        errs.append((e_a, e_f))
    return errs


@pytest.mark.parametrize("window", WINDOWS)
def test_window_sweep_f64(H, oracle_mod, case, window):
    errs = _sweep(H, oracle_mod, case, window, "f64")
    # the error falls with m until it reaches rounding
    for m in range(1, 15):
        for d in (0, 1):
            if errs[m - 1][d] > 1e-11:
                assert errs[m][d] < errs[m - 1][d], (window, m, d, errs[m - 1][d], errs[m][d])
    # and reaches the float64 rounding level somewhere in the range (sinc-power
    # the latest: its divisors' dynamic range is the largest)
    assert min(max(e) for e in errs) < 1e-12


@pytest.mark.parametrize("window", WINDOWS)
def test_window_sweep_f32(H, oracle_mod, case, window):
    errs = _sweep(H, oracle_mod, case, window, "f32")
    # float32 reaches the 1e-5 target of the precision extension at some m
    assert min(max(e) for e in errs) < 1e-5


@pytest.mark.parametrize("window,m", [("gaussian", 6), ("bspline", 10), ("kaiser_bessel", 12)])
def test_window_gradient(H, oracle_mod, window, m):
    """Backward of Eq. (5) with other windows and wide cut-offs: grad_f and
    grad_x against the oracle's analytic gradient."""
    Ng = (16, 12, 16)
    Mg = 600
    g = W.rng(77)
    x = W.uniform_points(Mg, 3, g)
    f = W.complex_normal(Mg, g)
    gbar = W.complex_normal(int(np.prod(Ng)), g).reshape(Ng)
    plan = H.Plan(Ng, Mg, m=m, precision="f64", with_grad=True, window=window)
    plan.set_points(torch.from_numpy(x).cuda())
    gf, gx = plan.adjoint_backward(torch.from_numpy(f).cuda(), torch.from_numpy(gbar).cuda())
    rf, rx = oracle_mod.ndft_adjoint_grad(Ng, x, f, gbar)
    ef = oracle_mod.rel_l2(gf.cpu().numpy(), rf)
    ex = np.linalg.norm(gx.cpu().numpy() - rx) / np.linalg.norm(rx)
    E = H.window_error_bound(m, 2.0, window)
    # grad_x carries the factor 2 pi k of the derivative: up to pi N more
    tol = max(1e-12, 3e3 * E)
    print("%s m=%d grad_f %.3e grad_x %.3e (tol %.1e)" % (window, m, ef, ex, tol))
    assert ef <= tol and ex <= tol
