"""The ring sweeps for 2m = 8 (the Spreading step of Algorithm 2 and the
Interpolating step of Algorithm 5, Section 3): tiles of 8 x 8 lines, slabs of
whole 8-plane phases, one wavefront per block of 8 lines sweeping its points
through the slab while the planes pass through an LDS ring.  Checked against
the direct FP64 oracle (Eqs. (5) and (6)) and against the staged sweeps, on
slabs that divide the grid and ragged ones, grids as small as the window
(n = 2m), clustered point sets (heavy tiles cut into line ranges), batches
and gradient plans; grids whose n0 is no multiple of 2m fall back to the
staged sweeps."""
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


def _adjoint(H, N, x, f, prec, tiles, with_grad=False, fh=None):
    cd = torch.complex128 if prec == "f64" else torch.complex64
    plan = H.Plan(N, x.shape[0], m=4, precision=prec, method="lines", tiles=tiles, with_grad=with_grad)
    plan.set_points(torch.from_numpy(x).cuda())
    a = plan.adjoint(torch.from_numpy(f).cuda().to(cd)).cpu().numpy().astype(np.complex128)
    if fh is None:
        return a
    b = plan.forward(torch.from_numpy(fh).cuda().to(cd)).cpu().numpy().astype(np.complex128)
    return a, b


def _data(seed, N, M, prec, clustered=False):
    g = W.rng(seed)
    if clustered:
        x = W.clustered_points(M // 2, 4, M // 8, 0.02, 3, g)
    else:
        x = W.uniform_points(M, 3, g)
    f = W.complex_normal(x.shape[0], g)
    if prec == "f32":
        f = f.astype(np.complex64).astype(np.complex128)
    return x, f


# N, M, Zs: slabs dividing n0 = 2 N0 or not, one slab, the window-sized grid
CASES = [
    ((16, 16, 16), 4096, 8),
    ((16, 16, 16), 4096, 24),
    ((12, 20, 16), 5000, 16),
    ((6, 10, 12), 2000, 8),
    ((4, 4, 4), 300, 8),
    ((16, 16, 16), 1, 32),
    ((32, 32, 32), 30000, 32),
]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("N,M,Zs", CASES)
def test_ring_against_oracle(H, oracle_mod, N, M, Zs, prec):
    x, f = _data(900 + M + Zs, N, M, prec)
    fh = W.complex_normal(int(np.prod(N)), W.rng(M + Zs)).reshape(N)
    if prec == "f32":
        fh = fh.astype(np.complex64).astype(np.complex128)
    a, b = _adjoint(H, N, x, f, prec, (8, Zs, 512), fh=fh)
    err = oracle_mod.rel_l2(a, oracle_mod.ndft_adjoint(N, x, f))
    errb = oracle_mod.rel_l2(b, oracle_mod.ndft_forward(N, x, fh))
    print("ring N=%s M=%d Zs=%d %s: adjoint rel-l2 %.3e forward %.3e" % (N, M, Zs, prec, err, errb))
    assert err <= 1e-5 and errb <= 1e-5


@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 2e-6)])
def test_ring_matches_staged(H, prec, tol):
    """Same points and values through the ring sweep (Zs = 16) and the staged
    sweep (Zs = 12): equal up to the order of the additions."""
    N, M = (20, 16, 24), 20000
    x, f = _data(77, N, M, prec)
    fh = W.complex_normal(int(np.prod(N)), W.rng(78)).reshape(N)
    ring, ringb = _adjoint(H, N, x, f, prec, (8, 16, 512), fh=fh)
    staged, stagedb = _adjoint(H, N, x, f, prec, (8, 12, 512), fh=fh)
    d = np.linalg.norm(ring - staged) / np.linalg.norm(staged)
    db = np.linalg.norm(ringb - stagedb) / np.linalg.norm(stagedb)
    print("ring vs staged %s: adjoint %.3e forward %.3e" % (prec, d, db))
    assert d <= tol and db <= tol


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_ring_clustered(H, oracle_mod, prec):
    """Half the points in four tight clusters: the heaviest (tile, slab)
    pairs are cut into ranges of blocks, so items start at blocks > 0."""
    N = (16, 16, 16)
    x, f = _data(31, N, 8000, prec, clustered=True)
    fh = W.complex_normal(int(np.prod(N)), W.rng(32)).reshape(N)
    if prec == "f32":
        fh = fh.astype(np.complex64).astype(np.complex128)
    a, b = _adjoint(H, N, x, f, prec, (8, 16, 512), fh=fh)
    err = oracle_mod.rel_l2(a, oracle_mod.ndft_adjoint(N, x, f))
    errb = oracle_mod.rel_l2(b, oracle_mod.ndft_forward(N, x, fh))
    print("ring clustered %s: adjoint %.3e forward %.3e" % (prec, err, errb))
    assert err <= 1e-5 and errb <= 1e-5


def test_ring_edges_of_the_torus(H, oracle_mod):
    """Points on the cell boundaries and at both ends of [-1/2, 1/2)."""
    N = (8, 8, 8)
    g = W.rng(5)
    grid = np.arange(-8, 8) / 16.0
    x = np.stack(np.meshgrid(grid[::3], grid[::5], grid[::2], indexing="ij"), -1).reshape(-1, 3)
    x = np.concatenate([x, np.array([[-0.5, -0.5, -0.5], [0.5 - 1e-13, 0.5 - 1e-13, -0.5]])])
    f = W.complex_normal(x.shape[0], g)
    fh = W.complex_normal(int(np.prod(N)), g).reshape(N)
    a, b = _adjoint(H, N, x, f, "f64", (8, 8, 512), fh=fh)
    err = oracle_mod.rel_l2(a, oracle_mod.ndft_adjoint(N, x, f))
    errb = oracle_mod.rel_l2(b, oracle_mod.ndft_forward(N, x, fh))
    assert err <= 1e-5 and errb <= 1e-5


def test_ring_batch_and_grad_plan(H, oracle_mod):
    """A batch of three transforms (later transforms start past sorted
    position 0) and a gradient plan (longer records)."""
    Ns = [(16, 16, 16), (12, 8, 20), (8, 8, 8)]
    Ms = [3000, 1500, 200]
    g = W.rng(61)
    xs = [W.uniform_points(M, 3, g) for M in Ms]
    fs = [W.complex_normal(M, g) for M in Ms]
    plan = H.Plan(Ns, Ms, m=4, precision="f64", method="lines", tiles=(8, 16, 512))
    plan.set_points(torch.from_numpy(np.concatenate(xs)).cuda())
    out = plan.adjoint(torch.from_numpy(np.concatenate(fs)).cuda()).cpu().numpy()
    for b in range(3):
        _, fo = plan.offsets(b)
        nb = int(np.prod(Ns[b]))
        err = oracle_mod.rel_l2(out[fo:fo + nb], oracle_mod.ndft_adjoint(Ns[b], xs[b], fs[b]).reshape(-1))
        print("ring batch b=%d: %.3e" % (b, err))
        assert err <= 1e-5
    fhs = [W.complex_normal(int(np.prod(Nb)), g) for Nb in Ns]
    back = plan.forward(torch.from_numpy(np.concatenate(fhs)).cuda()).cpu().numpy()
    for b in range(3):
        po, _ = plan.offsets(b)
        ref = oracle_mod.ndft_forward(Ns[b], xs[b], fhs[b].reshape(Ns[b]))
        assert oracle_mod.rel_l2(back[po:po + Ms[b]], ref) <= 1e-5
    a = _adjoint(H, Ns[0], xs[0], fs[0], "f64", (8, 16, 512), with_grad=True)
    assert oracle_mod.rel_l2(a, oracle_mod.ndft_adjoint(Ns[0], xs[0], fs[0])) <= 1e-5
