#!/usr/bin/env python
"""Benchmark of the NFFT hot path on one MI355X.

Workload: bandwidth N = 64^3 (grid n = 128^3, sigma = 2), M = 2^20 points
i.i.d. uniform in [-1/2, 1/2)^3, complex values with re, im ~ N(0, 1).
One step = the whole path once: set_points (bin, sort, window tables),
adjoint (Eq. (5): spread, FFT, roll-off/crop) and forward (Eq. (6):
roll-off/pad, inverse FFT, interpolate).

Headline: the float32 path at m = 4 (relative l2 error <= 1e-5 against the
FP64 oracle).  Reported beside it: the float64 path at m = 8 (<= 1e-12).
value = M / (seconds per step).

Prints one JSON line on stdout.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "NFFT points/s at rel-err 1e-5 FP32 vs FP64 plain (1e-12); spread HBM GB/s"
PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}
N = (64, 64, 64)
M = 1 << 20


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def phase_work(prec: str, m: int, n: int, Nb: int, Mp: int):
    """Algorithmic work per launch of each phase: (kind, amount).
    alu phases count 2 FMA = 4 flops per window tap ((2m)^3 taps per point);
    hbm phases count bytes each launch must read plus write once."""
    r = 8 if prec == "f64" else 4
    C = 2 * r
    n3, N3 = n ** 3, Nb ** 3
    taps = Mp * (2 * m) ** 3
    return {
        "spread": ("alu", taps * 4.0),
        "interp": ("alu", taps * 4.0),
        "fft_a0": ("hbm", (n3 + n * n * Nb) * C),
        "fft_a1": ("hbm", (n * n * Nb + n * Nb * Nb) * C),
        "fft_a2": ("hbm", (n * Nb * Nb + N3) * C),
        "fft_f0": ("hbm", (N3 + n * Nb * Nb) * C),
        "fft_f1": ("hbm", (n * Nb * Nb + n * n * Nb) * C),
        "fft_f2": ("hbm", (n * n * Nb + n3) * C),
        "gather": ("hbm", Mp * (4 + 2 * C)),
        "scatter": ("hbm", Mp * (4 + 2 * C)),
    }


def spread_bytes(prec: str, m: int, n: int, Mp: int, d: int = 3) -> float:
    """Spread algorithmic HBM bytes of the method itself: per point its d
    coordinates and its complex value read (M (d + 2) s), the grid written
    once (n^d 2 s).  Implementation-specific tables (the per-point window
    records) are not counted."""
    r = 8 if prec == "f64" else 4
    return Mp * (d + 2) * r + n ** d * 2 * r


def hbm_copy_gbs(torch, H, nbytes: int = 1 << 30, reps: int = 10) -> float:
    """Achievable HBM rate: the library's streaming copy kernel over nbytes
    (read + write counted), best of reps launches timed with HIP events."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    best = 1e30
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        H.device_copy(b, a)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / best / 1e9


def src_hash() -> str:
    """Hash of every kernel and plan source (a change to any of them, the
    tiling included, invalidates the counter summary)."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2001_01583_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            with open(os.path.join(d, f), "rb") as fh:
                h.update(f.encode())
                h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, prec: str, m: int):
    """Bytes per launch from the committed rocprofv3 counter summary, if it was
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_c2.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("src_hash") != src_hash():
        return None
    return d.get("kernels", {}).get("%s_%s_m%d" % (kernel, prec, m))


COPY_BYTES = 1 << 30


def copy_calibration(torch):
    """A plain device copy of known size (1 GiB read + 1 GiB written) for
    calibrating the FETCH_SIZE / WRITE_SIZE counters."""
    a = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    torch.mul(a, 1.0, out=b)  # an elementwise kernel: 1 GiB read, 1 GiB written
    torch.cuda.synchronize()
    del a, b


def summarize_counters(fetch_dir: str, write_dir: str, out_json: str, command: str):
    """Per-kernel average FETCH_SIZE and WRITE_SIZE (KiB per dispatch) from two
    rocprofv3 --pmc runs, each scaled by the copy kernel's measured/known ratio."""
    import csv
    import glob

    def load(d, counter):
        rows = []
        for fn in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(fn) as fh:
                rows += [r for r in csv.DictReader(fh) if r.get("Counter_Name") == counter]
        agg = {}
        for r in rows:
            name = r["Kernel_Name"]
            agg.setdefault(name, []).append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in agg.items()}

    fetch = load(fetch_dir, "FETCH_SIZE")
    write = load(write_dir, "WRITE_SIZE")

    def copy_kib(d):
        # the calibration kernel: torch.mul(a, 1.0, out=b) over 1 GiB
        cands = [(k, v) for k, v in d.items() if "MulFunctor" in k]
        return max(cands, key=lambda kv: kv[1]) if cands else (None, None)

    ck, cf = copy_kib(fetch)
    wk, cw = copy_kib(write)
    known_kib = COPY_BYTES / 1024.0
    f_scale = known_kib / cf if cf else None
    w_scale = known_kib / cw if cw else None
    kern = {}
    import re
    for full in set(fetch) | set(write):
        # the sweep kernels of the default line: the ring sweeps (2m = 8,
        # m = 4), the line interpolation and the staged sweeps (whose second
        # template argument is 2m)
        mt = re.match(r"(?:void )?hpnfft::k_(spread|interp)(_ring|_lines)?<(float|double)(?:, (\d+))?", full)
        if not mt:
            continue
        m = 4 if mt.group(2) == "_ring" else int(mt.group(4)) // 2
        prec = "f32" if mt.group(3) == "float" else "f64"
        fb = fetch.get(full, 0.0) * 1024.0 * (f_scale or 1.0)
        wb = write.get(full, 0.0) * 1024.0 * (w_scale or 1.0)
        kern["%s_%s_m%d" % (mt.group(1), prec, m)] = round(fb + wb)
    out = {"src_hash": src_hash(), "command": command, "copy_kernel_fetch": ck, "copy_kernel_write": wk,
           "fetch_scale": f_scale, "write_scale": w_scale, "kernels": kern,
           "raw_kib": {"fetch": fetch, "write": write}}
    with open(out_json, "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
    print(json.dumps({k: v for k, v in out.items() if k != "raw_kib"}, indent=1))


def run_path(H, torch, W, data, prec: str, m: int, steps: int, warmup: int, method: str = "auto"):
    dev = torch.device("cuda", 0)
    cd = torch.complex128 if prec == "f64" else torch.complex64
    plan = H.Plan(N, M, m=m, precision=prec, device=dev, method=method)
    x = torch.from_numpy(data["x"]).to(dev)
    f = torch.from_numpy(data["f"]).to(dev).to(cd)
    fh_in = torch.from_numpy(data["fhat"]).to(dev).to(cd)
    fh_out = torch.empty(N, dtype=cd, device=dev)
    f_out = torch.empty(M, dtype=cd, device=dev)

    def step():
        plan.set_points(x)
        plan.adjoint(f, out=fh_out)
        plan.forward(fh_in, out=f_out)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # phase table: every phase timed, outside the timed region (an event
    # between two kernels delays the second by a few microseconds)
    plan.profile(True)
    for _ in range(max(2, min(steps, 5))):
        step()
    phases = plan.profile_read()
    work = phase_work(prec, m, 2 * N[0], N[0], M)
    dom = max((k for k in phases if k in work), key=lambda k: phases[k][0])
    # timed region: only the dominant kernel carries events (its launch
    # durations for the roofline)
    plan.profile(True, phases=[dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dom_timed = plan.profile_read()[dom]
    plan.profile(False)
    ms_step = (t1 - t0) * 1e3 / steps
    return dict(plan=plan, ms_per_step=ms_step, phases=phases, dom=dom, dom_timed=dom_timed,
                fhat=fh_out.cpu().numpy(), fout=f_out.cpu().numpy(), tiles=plan.tiles, method=plan.method)


def summarize(res, prec, m, copy_gbs=None):
    n = 2 * N[0]
    work = phase_work(prec, m, n, N[0], M)
    table = {}
    for name, (ms, cnt) in res["phases"].items():
        per = ms / max(cnt, 1)
        row = {"ms_per_launch": round(per, 5), "launches": cnt}
        if name in work:
            kind, amount = work[name]
            if kind == "alu":
                row["tflops"] = round(amount / (per * 1e-3) / 1e12, 3)
            else:
                gbs = amount / (per * 1e-3) / 1e9
                row["gbs"] = round(gbs, 1)
                row["hbm_frac"] = round(gbs / PEAK_HBM_GBS, 4)
                if copy_gbs:
                    row["hbm_frac_of_copy"] = round(gbs / copy_gbs, 4)
        table[name] = row
    dom = res["dom"]
    kind, amount = work[dom]
    ms, cnt = res["dom_timed"]  # HIP events over the timed region
    per_s = ms / cnt * 1e-3
    if kind == "alu":
        ach, peak, unit = amount / per_s / 1e12, PEAK_TFLOPS[prec], "TFLOP/s"
    else:
        ach, peak, unit = amount / per_s / 1e9, PEAK_HBM_GBS, "GB/s"
    traffic = measured_traffic(dom, prec, m)
    roof = {"bound": kind, "kernel": dom, "achieved": round(ach, 3), "peak": peak, "unit": unit,
            "frac": round(ach / peak, 4), "traffic": traffic}
    if kind == "alu":
        # the library is built without packed FP32 instructions: one FMA per
        # lane per cycle, 78.6 TFLOP/s in either precision
        roof["peak_note"] = ("vector %s peak; without packed FP32 the reachable rate is 78.6 TFLOP/s"
                             % prec)
        roof["frac_of_unpacked"] = round(ach / 78.6, 4)
    sp_ms, sp_cnt = res["phases"].get("spread", (0.0, 0))
    spread_gbs = spread_bytes(prec, m, n, M) / (sp_ms / max(sp_cnt, 1) * 1e-3) / 1e9 if sp_cnt else None
    return table, roof, spread_gbs


def cpu_baseline(data, gpu):
    """The FP64 oracle (direct Eq. (5) and Eq. (6)) on a bounded sample of the
    same workload, timed on the host cores; the same samples give the GPU
    results' relative l2 errors."""
    import numpy as np

    import oracle
    import workloads as W
    oracle.build()
    g = W.rng(99)
    x, f, fhat = data["x"], data["f"], data["fhat"]
    nall = N[0] * N[1] * N[2]
    # calibrate on enough outputs to occupy every host thread, then size the
    # sample to ~12 s (adjoint) + ~6 s (forward)
    kc = W.sample_indices(nall, 128, g)
    t0 = time.perf_counter()
    oracle.ndft_adjoint(N, x, f, kidx=kc)
    t_k = (time.perf_counter() - t0) / 128
    nk = int(max(128, min(32768, 12.0 / max(t_k, 1e-7))))
    kidx = W.sample_indices(nall, nk, g)
    jc = W.sample_indices(M, 512, g)
    t0 = time.perf_counter()
    oracle.ndft_forward(N, x, fhat, jidx=jc)
    t_j = (time.perf_counter() - t0) / 512
    nj = int(max(512, min(262144, 6.0 / max(t_j, 1e-7))))
    jidx = W.sample_indices(M, nj, g)

    errs = {}
    t0 = time.perf_counter()
    ref_a = oracle.ndft_adjoint(N, x, f, kidx=kidx)
    ta = time.perf_counter() - t0
    t0 = time.perf_counter()
    ref_f = oracle.ndft_forward(N, x, fhat, jidx=jidx)
    tf = time.perf_counter() - t0
    # the float32 runs received the same draws rounded: their oracle values
    # on the same (full) sample, outside the timed baseline
    fa = f.astype(np.complex64).astype(np.complex128)
    fb = fhat.astype(np.complex64).astype(np.complex128)
    ref32 = None
    for key, res in gpu.items():
        prec = key.split("_")[0]
        if prec == "f32":
            if ref32 is None:
                ref32 = (oracle.ndft_adjoint(N, x, fa, kidx=kidx), oracle.ndft_forward(N, x, fb, jidx=jidx))
            ra, rf = ref32
        else:
            ra, rf = ref_a, ref_f
        ea = oracle.rel_l2(res["fhat"].reshape(-1)[kidx].astype(np.complex128), ra)
        ef = oracle.rel_l2(res["fout"][jidx].astype(np.complex128), rf)
        errs[key] = {"adjoint": float("%.3e" % ea), "forward": float("%.3e" % ef), "k": int(nk), "j": int(nj)}
    t_adj_full = ta * nall / nk
    t_fwd_full = tf * M / nj
    cores = oracle.threads()
    base = {"value": round(M / (t_adj_full + t_fwd_full), 1), "unit": "points/s", "cores": cores,
            "kind": "oracle",
            "sample": "FP64 direct NDFT: %d sampled frequencies of the adjoint (Eq. 5, %.1f s) and %d "
                      "sampled points of the forward (Eq. 6, %.1f s) over all %d points; full-transform "
                      "time extrapolated linearly (cost is exactly proportional to outputs)"
                      % (nk, ta, nj, tf, M)}
    return base, errs


# ---------------------------------------------------------------------------
# Secondary workloads (--workload c3 | c4 | c5): one JSON line each, same keys.
def _time(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def bench_c3(H, torch, W, args, summary=False):
    """Precision workload: N = 128^3, M = 2^23 (half uniform, half in 64
    Gaussian clusters), m = 4; step = set_points + adjoint.  float32 against
    the float64 GPU path over all of I_N, and both against the oracle on
    sampled frequencies."""
    import numpy as np

    import oracle
    data = W.c3()
    N, x_np, f_np = data["N"], data["x"], data["f"]
    Mp = x_np.shape[0]
    dev = torch.device("cuda", 0)
    x = torch.from_numpy(x_np).to(dev)
    res = {}
    for prec in ("f32", "f64"):
        cd = torch.complex64 if prec == "f32" else torch.complex128
        plan = H.Plan(N, Mp, m=4, precision=prec, device=dev, method=args.method)
        f = torch.from_numpy(f_np).to(dev).to(cd)
        out = torch.empty(N, dtype=cd, device=dev)

        def step():
            plan.set_points(x)
            plan.adjoint(f, out=out)
        t = _time(torch, step, args.steps, args.warmup)
        plan.profile(True)
        step()
        torch.cuda.synchronize()
        ph = {k: v[0] / max(v[1], 1) for k, v in plan.profile_read().items()}
        plan.profile(False)
        res[prec] = dict(ms=t * 1e3, out=out.cpu().numpy().astype(np.complex128), phases=ph, tiles=plan.tiles)
        del plan
        torch.cuda.empty_cache()
    g = W.rng(98)
    kidx = W.sample_indices(int(np.prod(N)), 64, g)
    ref = oracle.ndft_adjoint(N, x_np, f_np.astype(np.complex64).astype(np.complex128), kidx=kidx)
    ref64 = oracle.ndft_adjoint(N, x_np, f_np, kidx=kidx)
    e32 = oracle.rel_l2(res["f32"]["out"].reshape(-1)[kidx], ref)
    e64 = oracle.rel_l2(res["f64"]["out"].reshape(-1)[kidx], ref64)
    e32_64 = oracle.rel_l2(res["f32"]["out"].reshape(-1), res["f64"]["out"].reshape(-1))
    r32 = res["f32"]
    if summary:
        return {"workload": "N=128^3, M=2^23 (half in 64 Gaussian clusters), m=4; step = set_points + adjoint",
                "f32_ms_per_step": round(r32["ms"], 4), "f64_ms_per_step": round(res["f64"]["ms"], 4),
                "f32_points_per_s": round(Mp / (r32["ms"] * 1e-3), 1),
                "fp32_speedup_over_fp64_equal_m": round(res["f64"]["ms"] / r32["ms"], 3),
                "rel_l2_f32_vs_f64_gpu_all_IN": float("%.3e" % e32_64),
                "rel_l2_vs_oracle_sampled": {"f32": float("%.3e" % e32), "f64": float("%.3e" % e64), "k": 64},
                "phases_f32_ms": {k: round(v, 4) for k, v in r32["phases"].items()},
                "phases_f64_ms": {k: round(v, 4) for k, v in res["f64"]["phases"].items()}}
    return {
        "metric": METRIC, "value": round(Mp / (r32["ms"] * 1e-3), 1), "unit": "points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(r32["ms"], 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "precision: NFFT N=128^3 (n=256^3), M=2^23 (half uniform, half in 64 Gaussian "
                               "clusters, std 0.02), complex64, Kaiser-Bessel m=4; step = set_points + adjoint",
                   "N": list(N), "M": Mp, "m": 4, "tiles": list(r32["tiles"])},
        "fp64_m4_ms_per_step": round(res["f64"]["ms"], 4),
        "fp32_speedup_over_fp64": round(res["f64"]["ms"] / r32["ms"], 3),
        "rel_l2_f32_vs_f64_gpu_all_IN": float("%.3e" % e32_64),
        "rel_l2_vs_oracle_sampled": {"f32": float("%.3e" % e32), "f64": float("%.3e" % e64), "k": 64},
        "phases_f32_ms": {k: round(v, 4) for k, v in r32["phases"].items()},
    }


def bench_c4(H, torch, W, args, summary=False):
    """Batching workload: 256 independent adjoints (M log-uniform in
    [1e3, 1e6], N in {32, 48, 64, 96}^3), float32, m = 4, one launch per
    phase; the adjoint captured in a HIP graph and replayed."""
    import numpy as np
    elems = W.c4(256)
    dev = torch.device("cuda", 0)
    x = torch.from_numpy(np.concatenate([e["x"] for e in elems])).to(dev)
    f = torch.from_numpy(np.concatenate([e["f"] for e in elems]).astype(np.complex64)).to(dev)
    Ms = [e["x"].shape[0] for e in elems]
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        plan = H.Plan([e["N"] for e in elems], Ms, m=4, precision="f32", device=dev, method=args.method)
        plan.set_points(x)
        t_tune = time.perf_counter()
        plan.autotune()  # bin sizes (tile, slab, threads) chosen on these points
        t_tune = time.perf_counter() - t_tune
        # the choice is in the tuning cache now: a second tuning of the same
        # batch shape reads it instead of timing the candidates
        t_cached = time.perf_counter()
        plan.autotune()
        t_cached = time.perf_counter() - t_cached
        t_sp = _time(torch, lambda: plan.set_points(x), max(2, args.steps // 4), 1)
        out = plan.adjoint(f)
        t_eager = _time(torch, lambda: plan.adjoint(f, out=out), args.steps, args.warmup)
        plan.profile(True)
        plan.adjoint(f, out=out)
        torch.cuda.synchronize()
        phases = {k: round(v[0] / max(v[1], 1), 4) for k, v in plan.profile_read().items()}
        plan.profile(False)
        gout = torch.empty_like(out)
        plan.capture(f, gout)
        t_graph = _time(torch, plan.replay, args.steps, args.warmup)
        diff = (gout - out).abs().max().item() / max(out.abs().max().item(), 1e-30)
    Mt = int(sum(Ms))
    if summary:
        return {"workload": "256 adjoints, M log-uniform in [1e3, 1e6], N in {32,48,64,96}^3, f32, m=4; "
                            "step = one graph-replayed batched adjoint",
                "ms_per_step": round(t_graph * 1e3, 4), "points_per_s": round(Mt / t_graph, 1),
                "M_total": Mt, "eager_ms_per_step": round(t_eager * 1e3, 4),
                "set_points_ms": round(t_sp * 1e3, 4), "tiles": list(plan.tiles),
                "autotune_s": round(t_tune, 2), "autotune_cached_s": round(t_cached, 3),
                "graph_vs_eager_max_rel_diff": float("%.3e" % diff), "phases_ms": phases}
    return {
        "metric": METRIC, "value": round(Mt / t_graph, 1), "unit": "points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(t_graph * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batching: 256 adjoint NFFTs, M log-uniform in [1e3, 1e6], N in {32,48,64,96}^3, "
                               "complex64, m=4, autotuned tiling; step = one graph-replayed batched adjoint (points already set)",
                   "B": 256, "M_total": Mt, "tiles": list(plan.tiles)},
        "eager_ms_per_step": round(t_eager * 1e3, 4), "set_points_ms": round(t_sp * 1e3, 4),
        "autotune_s": round(t_tune, 2), "autotune_cached_s": round(t_cached, 3),
        "graph_vs_eager_max_rel_diff": float("%.3e" % diff), "phases_ms": phases,
    }


def bench_c5(H, torch, W, args, summary=False):
    """Differentiation workload: reciprocal Ewald energy and forces of a
    fluorite lattice of 24^3 cells (165,888 ions, displacements std 0.01 r0),
    N = 128^3; step = set_points + adjoint (S) + energy/gbar + backward."""
    import numpy as np
    from paper_2001_01583_amd import ewald as E
    r_np, q_np, L_box = W.fluorite(24, 0.01, seed=5)
    dev = torch.device("cuda", 0)
    r = torch.from_numpy(r_np).to(dev)
    q = torch.from_numpy(q_np).to(dev)
    lo, hi = E.alpha_window(L_box, 128)
    alpha = 0.5 * (lo + hi)
    out = {}
    for prec, m in (("f64", 8), ("f32", 4)):
        ew = E.Ewald(r.shape[0], L_box, alpha, N=(128, 128, 128), m=m, precision=prec, device=dev,
                     method=args.method)
        t_tune = time.perf_counter()
        tiles = ew.autotune(r)  # once per lattice: tiling timed on these ions, gradient included
        t_tune = time.perf_counter() - t_tune
        t = _time(torch, lambda: ew.reciprocal(r, q, forces=True), args.steps, args.warmup)
        ew.plan.profile(True)
        U, F = ew.reciprocal(r, q, forces=True)
        torch.cuda.synchronize()
        ph = {k: round(v[0] / max(v[1], 1), 4) for k, v in ew.plan.profile_read().items()}
        ew.plan.profile(False)
        out[prec] = dict(ms=t * 1e3, U=float(U), F=F.cpu().numpy(), phases=ph, tiles=list(tiles),
                         tune_s=round(t_tune, 2))
        del ew
        torch.cuda.empty_cache()
    fdiff = np.abs(out["f32"]["F"] - out["f64"]["F"]).max() / np.abs(out["f64"]["F"]).max()
    nion = int(r.shape[0])
    if summary:
        return {"workload": "Ewald reciprocal energy + forces, fluorite 24^3 cells (165,888 ions), N=128^3; "
                            "step = set_points + adjoint + Eq. (12) + backward",
                "f64_m8_ms_per_step": round(out["f64"]["ms"], 4), "f32_m4_ms_per_step": round(out["f32"]["ms"], 4),
                "f64_ions_per_s": round(nion / (out["f64"]["ms"] * 1e-3), 1),
                "tiles_f64": out["f64"]["tiles"], "tiles_f32": out["f32"]["tiles"],
                "autotune_s": {"f64": out["f64"]["tune_s"], "f32": out["f32"]["tune_s"]},
                "forces_f32_vs_f64_max_rel": float("%.3e" % fdiff),
                "phases_f64_ms": out["f64"]["phases"], "phases_f32_ms": out["f32"]["phases"]}
    return {
        "metric": METRIC, "value": round(nion / (out["f64"]["ms"] * 1e-3), 1), "unit": "ions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(out["f64"]["ms"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "Ewald reciprocal energy + forces, fluorite 24^3 cells (165,888 ions, "
                               "displacement std 0.01 r0), N=128^3, float64 m=8 (float32 m=4 beside); step = "
                               "set_points + adjoint + Eq. (12) energy + backward (forces); autotuned tilings",
                   "ions": nion, "N": [128, 128, 128], "alpha": round(alpha, 6), "L_box": round(L_box, 6),
                   "tiles_f64": out["f64"]["tiles"], "tiles_f32": out["f32"]["tiles"]},
        "autotune_s": {"f64": out["f64"]["tune_s"], "f32": out["f32"]["tune_s"]},
        "fp32_m4_ms_per_step": round(out["f32"]["ms"], 4),
        "energy_f64": out["f64"]["U"], "energy_f32": out["f32"]["U"],
        "forces_f32_vs_f64_max_rel": float("%.3e" % fdiff), "phases_f64_ms": out["f64"]["phases"],
    }


def bench_c5sweep(H, torch, W, args, summary=False):
    """The differentiation workload over its lattice and grid sizes: fluorite
    L^3 cells (L = 4, 8, 12, 16, 24: 768 to 165,888 ions, displacements std
    0.01 r0) on N^3 grids (N = 64, 128, 256), float64 m=8 and float32 m=4,
    default tilings; step = set_points + adjoint + Eq. (12) energy + backward
    (forces)."""
    import numpy as np
    from paper_2001_01583_amd import ewald as E
    dev = torch.device("cuda", 0)
    steps = max(3, min(args.steps, 10))
    rows = []
    for cells in (4, 8, 12, 16, 24):
        r_np, q_np, L_box = W.fluorite(cells, 0.01, seed=5)
        r = torch.from_numpy(r_np).to(dev)
        q = torch.from_numpy(q_np).to(dev)
        for Nn in (64, 128, 256):
            lo, hi = E.alpha_window(L_box, Nn)
            alpha = 0.5 * (lo + hi)
            row = {"cells": cells, "ions": int(r.shape[0]), "N": Nn, "alpha": round(alpha, 6)}
            forces = {}
            for prec, m in (("f64", 8), ("f32", 4)):
                ew = E.Ewald(r.shape[0], L_box, alpha, N=(Nn, Nn, Nn), m=m, precision=prec, device=dev,
                             method=args.method)
                t = _time(torch, lambda: ew.reciprocal(r, q, forces=True), steps, 1)
                U, F = ew.reciprocal(r, q, forces=True)
                torch.cuda.synchronize()
                row["%s_m%d_ms" % (prec, m)] = round(t * 1e3, 4)
                row["%s_energy" % prec] = float(U)
                row["%s_method" % prec] = ew.plan.method
                forces[prec] = F.cpu().numpy()
                del ew
                torch.cuda.empty_cache()
            row["energy_f32_vs_f64_rel"] = float("%.3e" % abs((row["f32_energy"] - row["f64_energy"]) /
                                                              row["f64_energy"]))
            row["forces_f32_vs_f64_max_rel"] = float("%.3e" % (np.abs(forces["f32"] - forces["f64"]).max() /
                                                              np.abs(forces["f64"]).max()))
            log("c5 sweep %d^3 cells N=%d: f64 %.3f ms, f32 %.3f ms" % (cells, Nn, row["f64_m8_ms"],
                                                                        row["f32_m4_ms"]))
            rows.append(row)
    if summary:
        return {"workload": "Ewald reciprocal energy + forces over L = 4..24 cells and N = 64..256", "rows": rows}
    last = [rw for rw in rows if rw["cells"] == 24 and rw["N"] == 128][0]
    return {
        "metric": METRIC, "value": round(last["ions"] / (last["f64_m8_ms"] * 1e-3), 1), "unit": "ions/s",
        "n_gpus": 1, "steps": steps, "warmup": 1, "ms_per_step": last["f64_m8_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "Ewald reciprocal energy + forces, fluorite L^3 cells (L = 4, 8, 12, 16, 24, "
                               "displacement std 0.01 r0) on N^3 grids (N = 64, 128, 256), float64 m=8 and "
                               "float32 m=4, default tilings; value: L = 24, N = 128, float64"},
        "rows": rows,
    }


def bench_enuf(H, torch, W, args, summary=False):
    """Full Ewald (HP-ENUF) step on fluorite lattices of the paper's timing
    sweep, 12 * c^3 ions for c = 32, 45, 56, 64 (393,216 .. 3,145,728 ions):
    set_points + adjoint (S) + Eq. (12) energy + backward (reciprocal
    forces) + cell-list real-space energy and forces (Eq. (11)).  float64,
    m = 8, alpha = 1 / r0, cut-off and bandwidth for 1e-12 in both sums.
    Lattice at zero displacement, so the Madelung constant (Eq. (10)) checks
    every size against the value Section 5 prints (2.5194)."""
    from paper_2001_01583_amd import ewald as E
    dev = torch.device("cuda", 0)
    rows = []
    cells_list = [int(c) for c in args.enuf_cells.split(",")]
    for c in cells_list:
        r_np, q_np, L_box = W.fluorite(c, 0.0)
        alpha = 1.0
        rcut, Nb = E.parameters(L_box, alpha, 1e-12)
        r = torch.from_numpy(r_np).to(dev)
        q = torch.from_numpy(q_np).to(dev)
        nion = int(r.shape[0])
        ew = E.Ewald(nion, L_box, alpha, N=(Nb, Nb, Nb), m=8, precision="f64", rcut=rcut, device=dev,
                     method=args.method,
                     real_method="cells")

        def step():
            Uk, Fk = ew.reciprocal(r, q, forces=True)
            Ur, Fr = ew.real_space(r, q, forces=True)
            return Uk, Fk, Ur, Fr

        steps = max(2, min(args.steps, 5))
        t = _time(torch, step, steps, 1)
        t_real = _time(torch, lambda: ew.real_space(r, q, forces=True), steps, 1)
        Uk, Fk, Ur, Fr = step()
        torch.cuda.synchronize()
        U = float(Uk) + float(Ur)
        mad = E.madelung_constant(U, nion)
        F = (Fk + Fr).abs().max().item()
        rows.append({"cells": c, "ions": nion, "L_box": round(L_box, 4), "N": Nb, "n": 2 * Nb,
                     "rcut": round(rcut, 4), "ms_per_step": round(t * 1e3, 3),
                     "real_space_ms": round(t_real * 1e3, 3), "ions_per_s": round(nion / t, 1),
                     "madelung": round(mad, 10), "max_abs_force": float("%.3e" % F)})
        log("enuf %d^3 cells (%d ions, N=%d): %.2f ms/step (real space %.2f ms), Madelung %.9f, max|F| %.2e"
            % (c, nion, Nb, t * 1e3, t_real * 1e3, mad, F))
        del ew, r, q
        torch.cuda.empty_cache()
    if summary:
        return {"workload": "HP-ENUF step (Ewald: reciprocal by NFFT + cell-list real space, energy and forces), "
                            "fluorite lattices, float64 m=8, 1e-12", "rows": rows}
    last = rows[-1]
    return {
        "metric": METRIC, "value": last["ions_per_s"], "unit": "ions/s", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": last["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "HP-ENUF ion sweep: fluorite c^3 cells (12 c^3 ions) for c in %s; step = reciprocal "
                               "(set_points + adjoint + Eq. (12) + backward) + real space (cell lists, Eq. (11)), "
                               "energy and forces, float64 m=8, alpha=1/r0, 1e-12" % cells_list},
        "rows": rows,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the precision, batching and Ewald summaries of the default line")
    ap.add_argument("--copy-calib", action="store_true",
                    help="run a 1 GiB device copy first (counter calibration for rocprofv3 --pmc runs)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/traffic_c2.json from two rocprofv3 --pmc output folders")
    ap.add_argument("--counters-command", default="", help="command line recorded with the summary")
    ap.add_argument("--method", default="auto", choices=["auto", "lines", "boxes"],
                    help="sweep method of the spread and interpolation (default: the library's choice)")
    ap.add_argument("--enuf-cells", default="32,45,56,64",
                    help="lattice sizes (cells per edge) of the enuf workload")
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "c5", "c5sweep", "enuf"],
                    help="c2 (default): N=64^3, M=2^20, set_points+adjoint+forward; c3: precision N=128^3, "
                         "M=2^23; c4: 256-transform batch; c5: Ewald forces, 165,888 ions; c5sweep: Ewald "
                         "forces over L = 4..24 cells and N = 64..256; enuf: full Ewald ion sweep")
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(args.summarize_counters[0], args.summarize_counters[1],
                           os.path.join(ROOT, "profiles", "traffic_c2.json"), args.counters_command)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU's share only: this build has no multi-GPU path "
              "(the paper's subcell decomposition across GPUs is described, not run); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np  # noqa: F401
    import torch

    import workloads as W
    from paper_2001_01583_amd import hpnfft as H

    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    if not os.environ.get("HPNFFT_TUNE_CACHE"):
        # the autotuner's cache for this run (a fresh file: every choice is
        # timed once, then read back by later tunings of the same shape)
        import tempfile
        os.environ["HPNFFT_TUNE_CACHE"] = os.path.join(tempfile.mkdtemp(prefix="hpnfft_"), "tune.json")
    if args.workload != "c2":
        fn = {"c3": bench_c3, "c4": bench_c4, "c5": bench_c5, "c5sweep": bench_c5sweep,
              "enuf": bench_enuf}[args.workload]
        print(json.dumps(fn(H, torch, W, args)), flush=True)
        return
    data = W.c2()
    log("workload ready: N=%s M=%d" % (N, M))
    if args.copy_calib:
        copy_calibration(torch)
    copy_gbs = hbm_copy_gbs(torch, H)
    log("streaming copy: %.1f GB/s" % copy_gbs)
    gpu = {}
    gpu["f32_m4"] = run_path(H, torch, W, data, "f32", 4, args.steps, args.warmup, args.method)
    log("f32 m=4: %.3f ms/step" % gpu["f32_m4"]["ms_per_step"])
    if not args.no_fp64:
        gpu["f64_m4"] = run_path(H, torch, W, data, "f64", 4, max(3, args.steps // 2), args.warmup, args.method)
        log("f64 m=4: %.3f ms/step" % gpu["f64_m4"]["ms_per_step"])
        gpu["f64_m8"] = run_path(H, torch, W, data, "f64", 8, max(3, args.steps // 2), args.warmup, args.method)
        log("f64 m=8: %.3f ms/step" % gpu["f64_m8"]["ms_per_step"])

    main_res = gpu["f32_m4"]
    table, roof, spread_gbs = summarize(main_res, "f32", 4, copy_gbs)
    out = {
        "metric": METRIC,
        "value": round(M / (main_res["ms_per_step"] * 1e-3), 1),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "NFFT N=64^3 (n=128^3, sigma=2), M=2^20 uniform points, complex64, "
                               "Kaiser-Bessel m=4; step = set_points + adjoint (Eq. 5) + forward (Eq. 6)",
                   "N": list(N), "M": M, "m": 4, "sigma": 2.0, "tiles": list(main_res["tiles"]),
                   "method": main_res["method"]},
        "roofline": roof,
        "hbm_copy_gbs": round(copy_gbs, 1),
        "spread_gbs_algorithmic": None if spread_gbs is None else round(spread_gbs, 1),
        "spread_hbm_frac": None if spread_gbs is None else round(spread_gbs / PEAK_HBM_GBS, 4),
        "spread_hbm_frac_of_copy": None if spread_gbs is None else round(spread_gbs / copy_gbs, 4),
        "spread_bytes_note": "M (d+2) s + n^3 2 s per launch (points and values in, grid out once)",
        "phases": table,
    }
    if "f64_m8" in gpu:
        for key in ("f64_m8", "f64_m4"):
            r64 = gpu[key]
            mm = int(key[-1])
            t64, roof64, sp64 = summarize(r64, "f64", mm, copy_gbs)
            out["fp64_m%d" % mm] = {"value": round(M / (r64["ms_per_step"] * 1e-3), 1), "unit": "points/s",
                                    "ms_per_step": round(r64["ms_per_step"], 4), "dtype": "f64", "m": mm,
                                    "tiles": list(r64["tiles"]), "method": r64["method"], "roofline": roof64,
                                    "spread_gbs_algorithmic": None if sp64 is None else round(sp64, 1),
                                    "phases": t64}
        # E1 speed-up at equal M, N and m; the m = 8 ratio is the 1e-12 path's
        out["fp32_speedup_over_fp64_equal_m"] = round(gpu["f64_m4"]["ms_per_step"] / main_res["ms_per_step"], 3)
        out["f32_m4_over_f64_m8"] = round(gpu["f64_m8"]["ms_per_step"] / main_res["ms_per_step"], 3)
        a32 = main_res["fhat"].reshape(-1).astype(np.complex128)
        o32 = main_res["fout"].astype(np.complex128)
        out["rel_l2_f32_vs_f64m8_gpu_all"] = {
            "adjoint_all_IN": float("%.3e" % rel(a32, gpu["f64_m8"]["fhat"].reshape(-1))),
            "forward_all_points": float("%.3e" % rel(o32, gpu["f64_m8"]["fout"]))}
    if not args.no_secondary:
        for name, fn in (("c3", bench_c3), ("c4", bench_c4), ("c5", bench_c5)):
            t0 = time.perf_counter()
            out[name] = fn(H, torch, W, args, summary=True)
            log("%s: %.1f s" % (name, time.perf_counter() - t0))
    if not args.no_cpu_baseline:
        base, errs = cpu_baseline(data, gpu)
        out["cpu_baseline"] = base
        out["rel_l2_sampled"] = errs
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


def rel(a, b) -> float:
    """Eq. (9) relative l2 of a against b (host arrays)."""
    import numpy as np
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


if __name__ == "__main__":
    main()
