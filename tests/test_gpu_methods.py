"""Both sweep methods of the spread and the interpolation (the Spreading and
Interpolating steps, Algorithms 2 and 5): the line sweeps (register windows
along dim 0, LDS tiles with halos) and the box method (each workgroup owns an
output box and writes it once).  Each case runs under both, against the
direct FP64 oracle, with the backward, batches, clustered and degenerate
point sets and the widest window."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu
METHODS = ["lines", "boxes"]


@pytest.fixture(scope="module")
def H():
    from paper_2001_01583_amd import hpnfft
    hpnfft._load()
    return hpnfft


def _run(H, oracle_mod, N, x, f, fh, m, prec, method, sigma=2.0, window="kaiser_bessel", tiles=None):
    cd = torch.complex128 if prec == "f64" else torch.complex64
    plan = H.Plan(N, x.shape[0], sigma=sigma, m=m, precision=prec, method=method, window=window, tiles=tiles)
    assert plan.method == method
    plan.set_points(torch.from_numpy(x).cuda())
    a = plan.adjoint(torch.from_numpy(f).cuda().to(cd)).cpu().numpy().astype(np.complex128)
    b = plan.forward(torch.from_numpy(fh).cuda().to(cd)).cpu().numpy().astype(np.complex128)
    ea = oracle_mod.rel_l2(a, oracle_mod.ndft_adjoint(N, x, f))
    eb = oracle_mod.rel_l2(b, oracle_mod.ndft_forward(N, x, fh))
    return ea, eb, a, b


CASES = [
    # N, M, m, prec, sigma, tol
    ((16, 16, 16), 4096, 8, "f64", 2.0, 1e-12),
    ((32, 24, 40), 20000, 4, "f32", 2.0, 1e-5),
    ((24, 24, 24), 3000, 5, "f64", 1.5, 2e-7),     # sigma = 1.5: bound 9.5e-7 per unit of ||f||_1
    ((16, 16, 16), 2000, 15, "f64", 2.0, 2e-12),
    ((48, 16, 30), 7777, 7, "f32", 2.0, 1e-5),
    ((64, 8), 3000, 6, "f64", 2.0, 1e-10),
    ((8, 8, 8), 1, 3, "f64", 2.0, 1e-4),
]


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("N,M,m,prec,sigma,tol", CASES)
def test_methods_against_oracle(H, oracle_mod, N, M, m, prec, sigma, tol, method):
    g = W.rng(700 + M + m)
    d = len(N)
    x = W.uniform_points(M, d, g)
    f = W.complex_normal(M, g)
    fh = W.complex_normal(int(np.prod(N)), g).reshape(N)
    if prec == "f32":
        f = f.astype(np.complex64).astype(np.complex128)
        fh = fh.astype(np.complex64).astype(np.complex128)
    ea, eb, _, _ = _run(H, oracle_mod, N, x, f, fh, m, prec, method, sigma=sigma)
    print("%s N=%s M=%d m=%d %s: adjoint %.3e forward %.3e" % (method, N, M, m, prec, ea, eb))
    assert ea <= tol and eb <= tol


@pytest.mark.parametrize("tiles", [(8, 8, 512), (12, 20, 512), (32, 8, 512)])
def test_box_edges(H, oracle_mod, tiles):
    """Box edges other than the default, including boxes that do not divide
    the grid (uneven boxes) and a single box along a dim."""
    N = (20, 24, 16)
    M = 5000
    g = W.rng(88)
    x = W.uniform_points(M, 3, g)
    f = W.complex_normal(M, g)
    fh = W.complex_normal(int(np.prod(N)), g).reshape(N)
    ea, eb, _, _ = _run(H, oracle_mod, N, x, f, fh, 6, "f64", "boxes", tiles=tiles)
    print("boxes %s: adjoint %.3e forward %.3e" % (tiles, ea, eb))
    assert ea <= 1e-10 and eb <= 1e-10


@pytest.mark.parametrize("method", METHODS)
def test_methods_clustered(H, oracle_mod, method):
    """All points in a few cells (heavy boxes and runs) and on cell and
    domain edges."""
    N = (32, 32, 32)
    g = W.rng(91)
    M = 6000
    x = (np.floor(g.random((M, 3)) * 3) / 64.0 - 0.5 + 1.0 / 64.0).astype(np.float64)
    x[:200] = -0.5
    x[200:400] = 0.5 - 2.0 ** -30
    f = W.complex_normal(M, g)
    fh = W.complex_normal(int(np.prod(N)), g).reshape(N)
    ea, eb, _, _ = _run(H, oracle_mod, N, x, f, fh, 8, "f64", method)
    print("%s clustered: adjoint %.3e forward %.3e" % (method, ea, eb))
    assert ea <= 1e-12 and eb <= 1e-12


@pytest.mark.parametrize("prec,m,tol", [("f64", 8, 1e-12), ("f32", 4, 1e-5)])
def test_box_backward(H, oracle_mod, prec, m, tol):
    N = (16, 12, 20)
    M = 900
    g = W.rng(95)
    x = W.uniform_points(M, 3, g)
    f = W.complex_normal(M, g)
    gbar = W.complex_normal(int(np.prod(N)), g).reshape(N)
    cd = torch.complex128 if prec == "f64" else torch.complex64
    if prec == "f32":
        f = f.astype(np.complex64).astype(np.complex128)
        gbar = gbar.astype(np.complex64).astype(np.complex128)
    plan = H.Plan(N, M, m=m, precision=prec, with_grad=True, method="boxes")
    plan.set_points(torch.from_numpy(x).cuda())
    gf, gx = plan.adjoint_backward(torch.from_numpy(f).cuda().to(cd), torch.from_numpy(gbar).cuda().to(cd))
    rf, rx = oracle_mod.ndft_adjoint_grad(N, x, f, gbar)
    ef = oracle_mod.rel_l2(gf.cpu().numpy().astype(np.complex128), rf)
    ex = np.linalg.norm(gx.cpu().numpy().astype(np.float64) - rx) / np.linalg.norm(rx)
    print("boxes backward %s: grad_f %.3e grad_x %.3e" % (prec, ef, ex))
    assert ef <= tol and ex <= tol


def test_box_batch(H, oracle_mod):
    """A batch of transforms of different sizes under the box method, each
    against the oracle; repeated calls reuse the self-resetting queues."""
    Ns = [(16, 16, 16), (24, 32, 16), (8, 8, 8), (40, 24, 24)]
    Ms = [3000, 5000, 1, 800]
    g = W.rng(97)
    xs = [W.uniform_points(M, 3, g) for M in Ms]
    fs = [W.complex_normal(M, g) for M in Ms]
    plan = H.Plan(Ns, Ms, m=6, precision="f64", method="boxes")
    assert plan.method == "boxes"
    plan.set_points(torch.from_numpy(np.concatenate(xs)).cuda())
    ft = torch.from_numpy(np.concatenate(fs)).cuda()
    for rep in range(2):
        out = plan.adjoint(ft).cpu().numpy()
        for b, (N, x, f) in enumerate(zip(Ns, xs, fs)):
            _, fo = plan.offsets(b)
            a = out[fo:fo + int(np.prod(N))].reshape(N)
            e = oracle_mod.rel_l2(a, oracle_mod.ndft_adjoint(N, x, f))
            assert e <= 1e-10, (rep, b, e)


def test_methods_agree(H, oracle_mod):
    """The two methods give the same transform to rounding."""
    N = (32, 32, 32)
    M = 30000
    g = W.rng(99)
    x = W.uniform_points(M, 3, g)
    f = W.complex_normal(M, g)
    fh = W.complex_normal(int(np.prod(N)), g).reshape(N)
    _, _, a1, b1 = _run(H, oracle_mod, N, x, f, fh, 8, "f64", "lines")
    _, _, a2, b2 = _run(H, oracle_mod, N, x, f, fh, 8, "f64", "boxes")
    assert oracle_mod.rel_l2(a2, a1) <= 1e-14 and oracle_mod.rel_l2(b2, b1) <= 1e-14


@pytest.mark.parametrize("prec,m,tol", [("f64", 6, 1e-10), ("f32", 4, 1e-5)])
def test_mixed_batch(H, oracle_mod, prec, m, tol):
    """A batch whose dense transforms take the line sweeps and whose sparse
    ones take boxes (the default per-transform choice), each against the
    oracle, eager and graph-replayed."""
    Ns = [(16, 16, 16), (32, 32, 32), (24, 24, 24), (16, 16, 16)]
    Ms = [20000, 200, 9000, 3]        # densities 0.6, 0.0008, 0.08, 0.0001 points per cell
    g = W.rng(1600 + m)
    xs = [W.uniform_points(M, 3, g) for M in Ms]
    fs = [W.complex_normal(M, g) for M in Ms]
    if prec == "f32":
        fs = [f.astype(np.complex64).astype(np.complex128) for f in fs]
    cd = torch.complex128 if prec == "f64" else torch.complex64
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = H.Plan(Ns, Ms, m=m, precision=prec)
        assert plan.method == "mixed"
        plan.set_points(torch.from_numpy(np.concatenate(xs)).cuda())
        ft = torch.from_numpy(np.concatenate(fs)).cuda().to(cd)
        eager = plan.adjoint(ft).clone()
        out = torch.empty_like(eager)
        plan.capture(ft, out)
        for _ in range(2):
            out.zero_()
            plan.replay()
            torch.cuda.synchronize()
            err = (out - eager).abs().max().item() / eager.abs().max().item()
            assert err <= 1e-5, err
    torch.cuda.synchronize()
    eager = eager.cpu().numpy().astype(np.complex128)
    for b, (N, x, f) in enumerate(zip(Ns, xs, fs)):
        _, fo = plan.offsets(b)
        a = eager[fo:fo + int(np.prod(N))].reshape(N)
        e = oracle_mod.rel_l2(a, oracle_mod.ndft_adjoint(N, x, f))
        assert e <= tol, (b, e)
