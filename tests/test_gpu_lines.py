"""The interpolation by groups of single lines (the Interpolating step of
Algorithm 5, Section 3) for windows of 2m = 16 cells on grids whose n0 is a
multiple of 2m: groups of 2 x 2 lines (a row of three in float64), slabs of
64 planes, each point evaluated once by the slab of its first tap plane, the
planes passing through an LDS ring of 2m planes.  Checked against the
direct FP64 oracle (Eqs. (5) and (6)) on one slab and several (the last one
short), sigma = 1.5, clustered points, a single point, batches, gradient
plans and repeated calls; m = 5, 6, 7 (which keep the staged sweep) and
grids whose n0 is no multiple of 2m run the same checks through it."""
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


# accuracy of the Kaiser-Bessel window at sigma = 2 (the window error, with a
# margin), and a floor for float32 rounding
TOL64 = {5: 1e-8, 6: 1e-10, 7: 2e-12, 8: 1e-12}
TOL32 = 3e-6


def _forward(H, N, x, fh, m, prec, sigma=2.0, with_grad=False):
    cd = torch.complex128 if prec == "f64" else torch.complex64
    plan = H.Plan(N, x.shape[0], sigma=sigma, m=m, precision=prec, with_grad=with_grad)
    plan.set_points(torch.from_numpy(x).cuda())
    out = plan.forward(torch.from_numpy(fh).cuda().to(cd)).cpu().numpy().astype(np.complex128)
    return plan, out


def _fh(seed, N, prec):
    fh = W.complex_normal(int(np.prod(N)), W.rng(seed)).reshape(N)
    if prec == "f32":
        fh = fh.astype(np.complex64).astype(np.complex128)
    return fh


# N, M, m: one slab (n0 = 32), two (n0 = 128), a short last slab (n0 = 80:
# 64 + 16 planes), a single point, n0 = 24 (no multiple of 16: staged);
# m = 5, 6, 7 run the staged sweep
CASES = [
    ((16, 16, 16), 4096, 8),
    ((64, 16, 16), 20000, 8),
    ((40, 12, 20), 6000, 8),
    ((20, 16, 16), 3000, 5),
    ((36, 12, 12), 3000, 6),
    ((28, 16, 16), 3000, 7),
    ((16, 16, 16), 1, 8),
    ((12, 16, 16), 4000, 8),
]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("N,M,m", CASES)
def test_lines_against_oracle(H, oracle_mod, N, M, m, prec):
    g = W.rng(1300 + M + m)
    x = W.uniform_points(M, 3, g)
    f = W.complex_normal(M, g)
    if prec == "f32":
        f = f.astype(np.complex64).astype(np.complex128)
    fh = _fh(1400 + m, N, prec)
    plan, out = _forward(H, N, x, fh, m, prec)
    err = oracle_mod.rel_l2(out, oracle_mod.ndft_forward(N, x, fh))
    a = plan.adjoint(torch.from_numpy(f).cuda().to(plan.cdtype)).cpu().numpy().astype(np.complex128)
    erra = oracle_mod.rel_l2(a, oracle_mod.ndft_adjoint(N, x, f))
    print("lines N=%s M=%d m=%d %s: forward rel-l2 %.3e adjoint %.3e" % (N, M, m, prec, err, erra))
    tol = TOL64[m] if prec == "f64" else TOL32
    assert err <= tol and erra <= tol


def test_lines_sigma(H, oracle_mod):
    """sigma = 1.5: n = (48, 18, 30), tiles of the counting sort that do not
    divide the grid, a radix-5 FFT edge."""
    N, M = (32, 12, 20), 5000
    g = W.rng(1501)
    x = W.uniform_points(M, 3, g)
    fh = _fh(1502, N, "f64")
    plan, out = _forward(H, N, x, fh, 8, "f64", sigma=1.5)
    assert plan.info()[0] == (48, 18, 30)
    err = oracle_mod.rel_l2(out, oracle_mod.ndft_forward(N, x, fh))
    print("lines sigma=1.5 n=(48,18,30): forward rel-l2 %.3e" % err)
    assert err <= 1e-9


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_lines_clustered(H, oracle_mod, prec):
    """Half the points in four tight clusters: lines with hundreds of
    points per slab (several 64-point batches per line)."""
    N = (32, 32, 32)
    g = W.rng(1601)
    x = W.clustered_points(6000, 4, 1500, 0.01, 3, g)
    fh = _fh(1602, N, prec)
    _, out = _forward(H, N, x, fh, 8, prec)
    err = oracle_mod.rel_l2(out, oracle_mod.ndft_forward(N, x, fh))
    print("lines clustered %s: forward rel-l2 %.3e" % (prec, err))
    assert err <= (1e-12 if prec == "f64" else TOL32)


def test_lines_gradient_plan_and_repeat(H, oracle_mod):
    """A gradient plan's forward runs the line interpolation (its backward
    keeps the staged sweep); a second call on the same points gives the
    same result to rounding (the work queue resets itself; the output
    receives one atomic sum per row group)."""
    N, M = (32, 16, 24), 8000
    g = W.rng(1701)
    x = W.uniform_points(M, 3, g)
    fh = _fh(1702, N, "f64")
    plan, out = _forward(H, N, x, fh, 8, "f64", with_grad=True)
    err = oracle_mod.rel_l2(out, oracle_mod.ndft_forward(N, x, fh))
    again = plan.forward(torch.from_numpy(fh).cuda()).cpu().numpy()
    print("lines gradient plan: forward rel-l2 %.3e, repeat diff %.3e" % (err, np.abs(again - out).max()))
    assert err <= 1e-12
    assert np.abs(again - out).max() <= 1e-13 * np.abs(out).max()
    # the backward (staged interpolation with derivatives) is unchanged
    f = W.complex_normal(M, g)
    gf = torch.from_numpy(W.complex_normal(int(np.prod(N)), g).reshape(N)).cuda()
    res = plan.adjoint_backward(torch.from_numpy(f).cuda(), gf)
    assert all(torch.isfinite(torch.view_as_real(r) if r.is_complex() else r).all() for r in res if r is not None)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", TOL32)])
def test_lines_batch(H, oracle_mod, prec, tol):
    """A batch of transforms of several sizes (every n0 a multiple of 16):
    one launch per transform."""
    sizes = [((16, 16, 16), 900), ((24, 16, 8), 1), ((32, 24, 16), 4000)]
    g = W.rng(1801)
    xs = [W.uniform_points(M, 3, g) for _, M in sizes]
    cd = np.complex128 if prec == "f64" else np.complex64
    plan = H.Plan([n for n, _ in sizes], [M for _, M in sizes], m=8, precision=prec)
    plan.set_points(torch.from_numpy(np.concatenate(xs)).cuda())
    fhs = [_fh(1810 + b, n, prec) for b, (n, _) in enumerate(sizes)]
    fh = np.concatenate([v.reshape(-1) for v in fhs]).astype(cd)
    out = plan.forward(torch.from_numpy(fh).cuda()).cpu().numpy().astype(np.complex128)
    for b, (n, M) in enumerate(sizes):
        po, _ = plan.offsets(b)
        err = oracle_mod.rel_l2(out[po:po + M], oracle_mod.ndft_forward(n, xs[b], fhs[b]))
        print("lines batch %s b=%d N=%s M=%d: forward rel-l2 %.3e" % (prec, b, n, M, err))
        assert err <= tol


def test_lines_in_mixed_batch(H, oracle_mod):
    """A batch whose dense transforms take the line sweeps (their forward: the
    line interpolation) and whose sparse ones take boxes: each forward output
    against the oracle."""
    Ns = [(16, 16, 16), (32, 32, 32), (16, 16, 16)]
    Ms = [20000, 200, 3]
    g = W.rng(1901)
    xs = [W.uniform_points(M, 3, g) for M in Ms]
    plan = H.Plan(Ns, Ms, m=8, precision="f64")
    assert plan.method == "mixed"
    plan.set_points(torch.from_numpy(np.concatenate(xs)).cuda())
    fhs = [_fh(1910 + b, n, "f64") for b, n in enumerate(Ns)]
    out = plan.forward(torch.from_numpy(np.concatenate([v.reshape(-1) for v in fhs])).cuda()).cpu().numpy()
    for b, (n, M) in enumerate(zip(Ns, Ms)):
        po, _ = plan.offsets(b)
        err = oracle_mod.rel_l2(out[po:po + M], oracle_mod.ndft_forward(n, xs[b], fhs[b]))
        print("lines mixed batch b=%d N=%s M=%d: forward rel-l2 %.3e" % (b, n, M, err))
        assert err <= 1e-12
