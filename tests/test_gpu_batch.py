"""Batching (many independent transforms with uneven M and N per launch) and
HIP-graph replay.

  * a mixed batch against the oracle, transform by transform;
  * the batch equals the same transforms run one plan at a time;
  * the graph-captured batch adjoint, replayed several times with other eager
    GPU work and synchronisations between replays, matches the eager result
    every time;
  * the 256-transform workload (M log-uniform in [1e3, 1e6], N in
    {32, 48, 64, 96}^3, complex64, m = 4) on sampled frequencies per transform.
"""
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


def _pack(elems, prec):
    cd = np.complex128 if prec == "f64" else np.complex64
    x = np.concatenate([e["x"] for e in elems])
    f = np.concatenate([e["f"] for e in elems]).astype(cd)
    return x, f


def _mixed(seed, sizes):
    g = W.rng(seed)
    out = []
    for (N, M) in sizes:
        out.append(dict(N=N, x=W.uniform_points(M, 3, g), f=W.complex_normal(M, g)))
    return out


SIZES = [((16, 16, 16), 900), ((24, 24, 24), 50), ((32, 16, 24), 3000), ((16, 16, 16), 1),
         ((12, 12, 12), 400), ((32, 32, 32), 5000)]


@pytest.mark.parametrize("prec,m,tol", [("f64", 8, 1e-12), ("f32", 4, 1e-5)])
def test_mixed_batch_against_oracle(H, oracle_mod, prec, m, tol):
    elems = _mixed(501, SIZES)
    x, f = _pack(elems, prec)
    plan = H.Plan([e["N"] for e in elems], [e["x"].shape[0] for e in elems], m=m, precision=prec)
    plan.set_points(torch.from_numpy(x).cuda())
    out = plan.adjoint(torch.from_numpy(f).cuda()).cpu().numpy().astype(np.complex128)
    fo = W.rng(502)
    fh_all = []
    for b, e in enumerate(elems):
        po, fo_off = plan.offsets(b)
        nb = int(np.prod(e["N"]))
        fu = f[po:po + e["x"].shape[0]].astype(np.complex128)
        ref = oracle_mod.ndft_adjoint(e["N"], e["x"], fu).reshape(-1)
        err = oracle_mod.rel_l2(out[fo_off:fo_off + nb], ref)
        print("batch %s b=%d N=%s M=%d rel-l2 %.3e" % (prec, b, e["N"], e["x"].shape[0], err))
        assert err <= tol
        fh_all.append(W.complex_normal(nb, fo))
    # forward of the whole batch
    cd = np.complex128 if prec == "f64" else np.complex64
    fh = np.concatenate(fh_all).astype(cd)
    back = plan.forward(torch.from_numpy(fh).cuda()).cpu().numpy().astype(np.complex128)
    for b, e in enumerate(elems):
        po, fo_off = plan.offsets(b)
        nb = int(np.prod(e["N"]))
        ref = oracle_mod.ndft_forward(e["N"], e["x"], fh[fo_off:fo_off + nb].astype(np.complex128).reshape(e["N"]))
        err = oracle_mod.rel_l2(back[po:po + e["x"].shape[0]], ref)
        assert err <= tol


def test_batch_equals_single_plans(H):
    elems = _mixed(503, SIZES)
    x, f = _pack(elems, "f64")
    plan = H.Plan([e["N"] for e in elems], [e["x"].shape[0] for e in elems], m=6, precision="f64")
    plan.set_points(torch.from_numpy(x).cuda())
    out = plan.adjoint(torch.from_numpy(f).cuda()).cpu().numpy()
    for b, e in enumerate(elems):
        po, fo = plan.offsets(b)
        single = H.Plan(e["N"], e["x"].shape[0], m=6, precision="f64")
        single.set_points(torch.from_numpy(e["x"]).cuda())
        s = single.adjoint(torch.from_numpy(f[po:po + e["x"].shape[0]]).cuda()).cpu().numpy().reshape(-1)
        nb = s.size
        assert np.linalg.norm(out[fo:fo + nb] - s) <= 1e-13 * np.linalg.norm(s)


def test_graph_replay_matches_eager(H):
    elems = _mixed(504, SIZES)
    x, f = _pack(elems, "f32")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = H.Plan([e["N"] for e in elems], [e["x"].shape[0] for e in elems], m=4, precision="f32")
        plan.set_points(torch.from_numpy(x).cuda())
        ft = torch.from_numpy(f).cuda()
        eager = plan.adjoint(ft).clone()
        out = torch.empty_like(eager)
        plan.capture(ft, out)
        other = torch.randn(1 << 20, device="cuda")
        for rep in range(4):
            out.zero_()
            plan.replay()
            torch.cuda.synchronize()
            err = (out - eager).abs().max().item() / eager.abs().max().item()
            print("replay %d max rel diff %.3e" % (rep, err))
            assert err <= 1e-5
            # eager work and another plan's eager call between replays
            other = other * 1.0001 + 1.0
            plan.adjoint(ft)
            torch.cuda.synchronize()
    torch.cuda.synchronize()


def test_c4_batch_sampled(H, oracle_mod):
    """The 256-transform workload: every transform against the oracle on 64
    sampled frequencies, each within 1e-5 (relative l2 over its sample)."""
    elems = W.c4(256)
    x, f = _pack(elems, "f32")
    plan = H.Plan([e["N"] for e in elems], [e["x"].shape[0] for e in elems], m=4, precision="f32")
    plan.set_points(torch.from_numpy(x).cuda())
    out = plan.adjoint(torch.from_numpy(f).cuda()).cpu().numpy().astype(np.complex128)
    g = W.rng(505)
    errs = []
    for b in range(256):
        e = elems[b]
        po, fo = plan.offsets(b)
        nb = int(np.prod(e["N"]))
        kidx = W.sample_indices(nb, 64, g)
        fu = f[po:po + e["x"].shape[0]].astype(np.complex128)
        ref = oracle_mod.ndft_adjoint(e["N"], e["x"], fu, kidx=kidx)
        errs.append(oracle_mod.rel_l2(out[fo:fo + nb][kidx], ref))
    errs = np.array(errs)
    print("C4 256 transforms x 64 k: median %.3e worst %.3e (b=%d)" % (np.median(errs), errs.max(), errs.argmax()))
    assert errs.max() <= 1e-5


def test_graph_dropped_by_set_points(H, oracle_mod):
    """A captured batch graph holds the work list and workspace of the moment
    it was recorded: set_points (and any re-tiling) drops it, replay then
    reports ESTATE, and a new capture matches the eager result again."""
    elems = _mixed(507, SIZES)
    x, f = _pack(elems, "f32")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = H.Plan([e["N"] for e in elems], [e["x"].shape[0] for e in elems], m=4, precision="f32")
        plan.set_points(torch.from_numpy(x).cuda())
        ft = torch.from_numpy(f).cuda()
        out = torch.empty(plan.Ftot, dtype=torch.complex64, device="cuda")
        plan.capture(ft, out)
        plan.replay()
        # new points: half of the coordinates mirrored
        x2 = x.copy()
        x2[:, 0] = -x2[:, 0] - 1e-9
        x2 = W.wrap_unit(x2)
        plan.set_points(torch.from_numpy(x2).cuda())
        with pytest.raises(H.HpnfftError) as ei:
            plan.replay()
        assert ei.value.code == H.ESTATE
        eager = plan.adjoint(ft).clone()
        plan.capture(ft, out)
        out.zero_()
        plan.replay()
        torch.cuda.synchronize()
        err = (out - eager).abs().max().item() / eager.abs().max().item()
        assert err <= 1e-5
        # the replayed result is the transform of the new points
        po, fo = plan.offsets(5)
        e = elems[5]
        nb = int(np.prod(e["N"]))
        kidx = W.sample_indices(nb, 64, W.rng(508))
        ref = oracle_mod.ndft_adjoint(e["N"], x2[po:po + e["x"].shape[0]],
                                      f[po:po + e["x"].shape[0]].astype(np.complex128), kidx=kidx)
        got = out.cpu().numpy().astype(np.complex128)[fo:fo + nb][kidx]
        assert oracle_mod.rel_l2(got, ref) <= 1e-5
        # re-tiling drops it too
        plan.set_tiles(8, 8, 512)
        plan.set_points(torch.from_numpy(x2).cuda())
        with pytest.raises(H.HpnfftError) as ei:
            plan.replay()
        assert ei.value.code == H.ESTATE
    torch.cuda.synchronize()


def test_autotune_cache(H, oracle_mod, tmp_path, monkeypatch):
    """With HPNFFT_TUNE_CACHE set, the first autotune writes its choice to the
    cache file and a second plan of the same shape takes it from there (no
    candidate timing); the cached tiling reproduces the oracle result."""
    path = tmp_path / "tune.json"
    monkeypatch.setenv("HPNFFT_TUNE_CACHE", str(path))
    g = W.rng(509)
    N = (24, 24, 24)
    M = 30000
    x = W.uniform_points(M, 3, g)
    f = W.complex_normal(M, g).astype(np.complex64)
    import time
    plan = H.Plan(N, M, m=4, precision="f32")
    plan.set_points(torch.from_numpy(x).cuda())
    t0 = time.perf_counter()
    tiles = plan.autotune()
    t_first = time.perf_counter() - t0
    txt = path.read_text()
    assert '"hpnfft_tune_cache": 3' in txt and "[%d, %d, %d]" % tiles in txt
    plan2 = H.Plan(N, M, m=4, precision="f32")
    plan2.set_points(torch.from_numpy(x).cuda())
    t0 = time.perf_counter()
    tiles2 = plan2.autotune()
    t_second = time.perf_counter() - t0
    print("autotune %.3f s, cached %.3f s, tiles %s" % (t_first, t_second, tiles))
    assert tiles2 == tiles and plan2.tiles == tiles
    assert t_second < t_first
    out = plan2.adjoint(torch.from_numpy(f).cuda()).cpu().numpy().astype(np.complex128)
    kidx = W.sample_indices(24 ** 3, 256, g)
    ref = oracle_mod.ndft_adjoint(N, x, f.astype(np.complex128), kidx=kidx)
    assert oracle_mod.rel_l2(out.reshape(-1)[kidx], ref) <= 1e-5


def test_autotuner_keeps_results(H, oracle_mod):
    """The tiling autotuner times candidate tilings on the plan's own points
    and keeps the fastest; results before and after agree with the oracle."""
    g = W.rng(506)
    N = (24, 24, 24)
    x = W.uniform_points(20000, 3, g)
    f = W.complex_normal(20000, g).astype(np.complex64)
    plan = H.Plan(N, 20000, m=4, precision="f32")
    plan.set_points(torch.from_numpy(x).cuda())
    before = plan.adjoint(torch.from_numpy(f).cuda()).cpu().numpy()
    tiles = plan.autotune()
    assert tiles == plan.tiles and tiles[0] >= 4 and tiles[2] % 64 == 0
    after = plan.adjoint(torch.from_numpy(f).cuda()).cpu().numpy()
    kidx = W.sample_indices(24 ** 3, 64, g)
    ref = oracle_mod.ndft_adjoint(N, x, f.astype(np.complex128), kidx=kidx)
    for out in (before, after):
        assert oracle_mod.rel_l2(out.reshape(-1)[kidx].astype(np.complex128), ref) <= 1e-5


def test_phase_profiling_mask(H):
    """Timing a subset of phases records events for those phases only, and
    the transforms' results do not depend on what is timed."""
    g = W.rng(77)
    N = (16, 12, 24)
    M = 3000
    x = torch.from_numpy(W.uniform_points(M, 3, g)).cuda()
    f = torch.from_numpy(W.complex_normal(M, g).astype(np.complex64)).cuda()
    fh = torch.from_numpy(W.complex_normal(int(np.prod(N)), g).reshape(N).astype(np.complex64)).cuda()
    plan = H.Plan(N, M, m=4, precision="f32")
    plan.set_points(x)
    ref_a = plan.adjoint(f).clone()
    ref_f = plan.forward(fh).clone()
    plan.profile(True, phases=["spread", "interp"])
    for _ in range(3):
        a = plan.adjoint(f)
        b = plan.forward(fh)
    ph = plan.profile_read()
    plan.profile(False)
    assert set(ph) == {"spread", "interp"}
    assert ph["spread"][1] == 3 and ph["interp"][1] == 3 and ph["spread"][0] > 0
    # the sums are atomic, so their order (and the last bits) may vary
    assert (a - ref_a).abs().max() <= 1e-5 * ref_a.abs().max()
    assert (b - ref_f).abs().max() <= 1e-5 * ref_f.abs().max()
    plan.profile(True)
    plan.adjoint(f)
    assert {"gather", "spread", "fft_a0", "fft_a1", "fft_a2"} <= set(plan.profile_read())
    plan.profile(False)
    with pytest.raises(ValueError):
        plan.profile(True, phases=["no_such_phase"])


@pytest.mark.parametrize("M", [1, 37, 20000])
def test_repeated_calls_reuse_work_queues(H, M):
    """The sweeps' work-queue counters reset themselves at the end of every
    launch: many adjoint / forward calls in a row (few points, so fewer work
    items than workgroup slots, and many) keep giving the first call's
    results (up to the order of the atomic sums)."""
    g = W.rng(78 + M)
    N = (16, 16, 16)
    x = torch.from_numpy(W.uniform_points(M, 3, g)).cuda()
    f = torch.from_numpy(W.complex_normal(M, g).astype(np.complex64)).cuda()
    fh = torch.from_numpy(W.complex_normal(16 ** 3, g).reshape(N).astype(np.complex64)).cuda()
    plan = H.Plan(N, M, m=4, precision="f32")
    plan.set_points(x)
    a0 = plan.adjoint(f).clone()
    b0 = plan.forward(fh).clone()
    for _ in range(10):
        a = plan.adjoint(f)
        b = plan.forward(fh)
    torch.cuda.synchronize()
    assert (a - a0).abs().max() <= 1e-5 * a0.abs().max()
    assert (b - b0).abs().max() <= 1e-5 * b0.abs().max()
    plan.set_points(x)  # re-binning keeps them valid too
    a = plan.adjoint(f)
    assert (a - a0).abs().max() <= 1e-5 * a0.abs().max()


@pytest.mark.parametrize("prec,m,tol", [("f64", 8, 1e-12), ("f32", 4, 1e-5)])
def test_autotune_keeps_the_points(H, prec, m, tol):
    """After autotuning, the plan still holds its own points: an adjoint
    without a new set_points equals the one before.  The grid (n = 48 x 36 x
    64) makes the stored points' offset in the workspace depend on the tile
    edge, so a copy read from a candidate's layout would be wrong."""
    g = W.rng(79)
    N = (24, 18, 32)
    M = 6000
    x = torch.from_numpy(W.uniform_points(M, 3, g)).cuda()
    cd = torch.complex128 if prec == "f64" else torch.complex64
    f = torch.from_numpy(W.complex_normal(M, g)).cuda().to(cd)
    plan = H.Plan(N, M, m=m, precision=prec)
    plan.set_points(x)
    ref = plan.adjoint(f).clone()
    plan.autotune()
    got = plan.adjoint(f)
    err = ((got - ref).abs().norm() / ref.abs().norm()).item()
    print("autotune %s m=%d tiles=%s: rel change %.3e" % (prec, m, plan.tiles, err))
    assert err <= tol
