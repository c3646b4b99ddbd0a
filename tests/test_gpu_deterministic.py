"""Deterministic mode (HPNFFT_DETERMINISTIC): the Spreading and
Interpolating steps with every sum in a fixed order.  Repeated transforms,
and a repeated set_points of the same points (whose counting-sort ranks come
from atomics), give bitwise identical results; the results still match the
direct oracle of Eq. (5) / Eq. (6) and the analytic gradient."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_2001_01583_amd import hpnfft
    hpnfft._load()
    return hpnfft


def _points(kind, M, g):
    if kind == "uniform":
        return W.uniform_points(M, 3, g)
    # most points in a few cells: long runs in a few bins
    x = np.floor(g.random((M, 3)) * 4) / 32.0 - 0.5 + 1.0 / 64.0
    x[: M // 3] = W.uniform_points(M // 3, 3, g)
    return x


@pytest.mark.parametrize("prec,m,tol", [("f64", 8, 1e-12), ("f32", 4, 1e-5)])
@pytest.mark.parametrize("kind", ["uniform", "clustered"])
def test_bitwise_repeatable_and_exact(H, oracle_mod, prec, m, tol, kind):
    N = (32, 24, 32)
    M = 20000
    g = W.rng(1200 + m)
    x = _points(kind, M, g)
    f = W.complex_normal(M, g)
    fh = W.complex_normal(int(np.prod(N)), g).reshape(N)
    cd = torch.complex128 if prec == "f64" else torch.complex64
    if prec == "f32":
        f = f.astype(np.complex64).astype(np.complex128)
        fh = fh.astype(np.complex64).astype(np.complex128)
    plan = H.Plan(N, M, m=m, precision=prec, deterministic=True)
    assert plan.method == "boxes"
    xt = torch.from_numpy(x).cuda()
    ft = torch.from_numpy(f).cuda().to(cd)
    fht = torch.from_numpy(fh).cuda().to(cd)
    outs = []
    for rep in range(3):
        plan.set_points(xt)  # re-binned every time: the atomic ranks change
        outs.append((plan.adjoint(ft).cpu().numpy(), plan.forward(fht).cpu().numpy()))
    for a, b in outs[1:]:
        assert np.array_equal(a, outs[0][0]) and np.array_equal(b, outs[0][1])
    ea = oracle_mod.rel_l2(outs[0][0].astype(np.complex128), oracle_mod.ndft_adjoint(N, x, f))
    eb = oracle_mod.rel_l2(outs[0][1].astype(np.complex128), oracle_mod.ndft_forward(N, x, fh))
    print("deterministic %s %s: adjoint %.3e forward %.3e" % (prec, kind, ea, eb))
    assert ea <= tol and eb <= tol


@pytest.mark.parametrize("prec,m,tol", [("f64", 6, 1e-9), ("f32", 4, 1e-5)])  # grad_x carries 2 pi k
def test_bitwise_repeatable_backward(H, oracle_mod, prec, m, tol):
    N = (16, 20, 16)
    M = 3000
    g = W.rng(1300 + m)
    x = W.uniform_points(M, 3, g)
    f = W.complex_normal(M, g)
    gbar = W.complex_normal(int(np.prod(N)), g).reshape(N)
    cd = torch.complex128 if prec == "f64" else torch.complex64
    if prec == "f32":
        f = f.astype(np.complex64).astype(np.complex128)
        gbar = gbar.astype(np.complex64).astype(np.complex128)
    plan = H.Plan(N, M, m=m, precision=prec, with_grad=True, deterministic=True)
    xt = torch.from_numpy(x).cuda()
    ft = torch.from_numpy(f).cuda().to(cd)
    gt = torch.from_numpy(gbar).cuda().to(cd)
    res = []
    for rep in range(2):
        plan.set_points(xt)
        gf, gx = plan.adjoint_backward(ft, gt)
        res.append((gf.cpu().numpy(), gx.cpu().numpy()))
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
    rf, rx = oracle_mod.ndft_adjoint_grad(N, x, f, gbar)
    ef = oracle_mod.rel_l2(res[0][0].astype(np.complex128), rf)
    ex = np.linalg.norm(res[0][1].astype(np.float64) - rx) / np.linalg.norm(rx)
    print("deterministic backward %s: grad_f %.3e grad_x %.3e" % (prec, ef, ex))
    assert ef <= tol and ex <= tol


def test_deterministic_batch(H, oracle_mod):
    Ns = [(16, 16, 16), (24, 16, 32), (8, 8, 8)]
    Ms = [4000, 2500, 1]
    g = W.rng(1400)
    xs = [W.uniform_points(M, 3, g) for M in Ms]
    fs = [W.complex_normal(M, g) for M in Ms]
    plan = H.Plan(Ns, Ms, m=7, precision="f64", deterministic=True)
    xt = torch.from_numpy(np.concatenate(xs)).cuda()
    ft = torch.from_numpy(np.concatenate(fs)).cuda()
    runs = []
    for rep in range(2):
        plan.set_points(xt)
        runs.append(plan.adjoint(ft).cpu().numpy())
    assert np.array_equal(runs[0], runs[1])
    for b, (N, x, f) in enumerate(zip(Ns, xs, fs)):
        _, fo = plan.offsets(b)
        a = runs[0][fo:fo + int(np.prod(N))].reshape(N)
        assert oracle_mod.rel_l2(a, oracle_mod.ndft_adjoint(N, x, f)) <= 1e-12


def test_deterministic_agrees_with_default(H):
    N = (32, 32, 32)
    M = 50000
    g = W.rng(1500)
    x = torch.from_numpy(W.uniform_points(M, 3, g)).cuda()
    f = torch.from_numpy(W.complex_normal(M, g)).cuda()
    a = H.Plan(N, M, m=8, precision="f64")
    b = H.Plan(N, M, m=8, precision="f64", deterministic=True)
    a.set_points(x)
    b.set_points(x)
    ra, rb = a.adjoint(f), b.adjoint(f)
    assert (torch.linalg.norm(ra - rb) / torch.linalg.norm(ra)).item() <= 1e-14
    lib = H._load()
    assert lib.hpnfft_set_method(b._h, H.METHOD_LINES) == H.EINVAL
