"""Python binding of libhpnfft (ctypes).  Argument marshalling only.

Every transform step runs in the HIP library; PyTorch provides device memory
(the plan's workspace and the output tensors) and the current HIP stream.
There is no CPU fallback: without the built library or without a GPU the
calls raise.
"""
from __future__ import annotations

import ctypes
import math
import os
import re
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhpnfft.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "hpnfft.h")

OK, EINVAL, EDOMAIN, ENOMEM, EHIP, ESTATE, ESIZE = 0, -1, -2, -3, -4, -5, -6
KAISER_BESSEL, GAUSSIAN, BSPLINE, SINC_POWER = 0, 1, 2, 3
METHOD_AUTO, METHOD_LINES, METHOD_BOXES, METHOD_MIXED = 0, 1, 2, 3
METHODS = {"auto": METHOD_AUTO, "lines": METHOD_LINES, "boxes": METHOD_BOXES}
WINDOWS = {"kaiser_bessel": KAISER_BESSEL, "kb": KAISER_BESSEL, "gaussian": GAUSSIAN,
           "bspline": BSPLINE, "sinc_power": SINC_POWER}
F64, F32 = 0, 1
WITH_GRADIENT = 1
DETERMINISTIC = 2

_lib = None


class HpnfftError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = _load().hpnfft_strerror(code).decode() if _lib is not None else str(code)
        super().__init__("%s: %s (status %d)" % (where, msg, code))


def _load():
    """Load libhpnfft.so (must be built beforehand with paper_2001_01583_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libhpnfft.so is not built (run paper_2001_01583_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i64p = ctypes.POINTER(ctypes.c_int64)
    ip = ctypes.POINTER(ctypes.c_int)
    sig = {
        "hpnfft_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "hpnfft_plan_create": (ctypes.c_int, [ctypes.POINTER(P), ctypes.c_int, i64p, ctypes.c_int64,
                                              ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                              ctypes.c_uint]),
        "hpnfft_batch_create": (ctypes.c_int, [ctypes.POINTER(P), ctypes.c_int, i64p, i64p, ctypes.c_double,
                                               ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint]),
        "hpnfft_plan_destroy": (ctypes.c_int, [P]),
        "hpnfft_set_stream": (ctypes.c_int, [P, P]),
        "hpnfft_set_tiles": (ctypes.c_int, [P, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
        "hpnfft_set_method": (ctypes.c_int, [P, ctypes.c_int]),
        "hpnfft_get_method": (ctypes.c_int, [P, ip]),
        "hpnfft_get_tiles": (ctypes.c_int, [P, ip, ip, ip]),
        "hpnfft_workspace_size": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_size_t)]),
        "hpnfft_set_workspace": (ctypes.c_int, [P, P, ctypes.c_size_t]),
        "hpnfft_set_points": (ctypes.c_int, [P, P]),
        "hpnfft_set_points_f32": (ctypes.c_int, [P, P]),
        "hpnfft_batch_set_points": (ctypes.c_int, [P, P]),
        "hpnfft_adjoint": (ctypes.c_int, [P, P, P]),
        "hpnfft_forward": (ctypes.c_int, [P, P, P]),
        "hpnfft_batch_adjoint": (ctypes.c_int, [P, P, P]),
        "hpnfft_batch_forward": (ctypes.c_int, [P, P, P]),
        "hpnfft_adjoint_backward": (ctypes.c_int, [P, P, P, P, P]),
        "hpnfft_ewald_recip": (ctypes.c_int, [P, P, ctypes.c_double, ctypes.c_double, P, P]),
        "hpnfft_autotune": (ctypes.c_int, [P, P, P, ip, ip, ip]),
        "hpnfft_ewald_real": (ctypes.c_int, [P, P, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_double, P, P, P, P]),
        "hpnfft_ewald_real_cells_workspace": (ctypes.c_int, [ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                                             ctypes.POINTER(ctypes.c_size_t)]),
        "hpnfft_ewald_real_cells": (ctypes.c_int, [P, P, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                                   ctypes.c_double, P, P, P, ctypes.c_size_t, P]),
        "hpnfft_ewald_real_static": (ctypes.c_int, [P, P, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                                    ctypes.c_double, P, P, P]),
        "hpnfft_ewald_real_static_max_ions": (ctypes.c_int64, []),
        "hpnfft_plan_info": (ctypes.c_int, [P, i64p, i64p]),
        "hpnfft_check_points": (ctypes.c_int, [P, ctypes.c_int64, ctypes.c_int, i64p]),
        "hpnfft_copy": (ctypes.c_int, [P, P, ctypes.c_size_t, P]),
        "hpnfft_batch_capture": (ctypes.c_int, [P, P, P]),
        "hpnfft_batch_launch": (ctypes.c_int, [P]),
        "hpnfft_batch_offsets": (ctypes.c_int, [P, ctypes.c_int, i64p, i64p]),
        "hpnfft_profile": (ctypes.c_int, [P, ctypes.c_int]),
        "hpnfft_profile_phases": (ctypes.c_int, [P, ctypes.c_uint]),
        "hpnfft_profile_read": (ctypes.c_int, [P, P, P]),
        "hpnfft_phase_name": (ctypes.c_char_p, [ctypes.c_int]),
        "hpnfft_window_eval": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int64,
                                              P, P, P]),
        "hpnfft_window_rolloff": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int64,
                                                 ctypes.c_int64, P]),
        "hpnfft_window_error_bound": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                                     ctypes.POINTER(ctypes.c_double)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def declared_symbols() -> list:
    """Names of the functions include/hpnfft.h declares."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(hpnfft_\w+)\s*\(", txt)))


def _check(rc: int, where: str):
    if rc != OK:
        raise HpnfftError(rc, where)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_ptr(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _require_gpu(device):
    if not torch.cuda.is_available():
        raise RuntimeError("hpnfft needs a ROCm GPU; no CPU fallback exists")
    dev = torch.device(device)
    if dev.type != "cuda":
        raise ValueError("hpnfft runs on a ROCm GPU device, got %s" % dev)
    if dev.index is None:
        dev = torch.device("cuda", torch.cuda.current_device())
    return dev


class Plan:
    """NFFT plan for B >= 1 transforms (B = 1: a single transform).

    N: (N0, N1, N2) or a list of B such triples; M: int or list of B ints.
    precision: "f64" (complex128 values) or "f32" (complex64 values).
    """

    def __init__(self, N, M, sigma: float = 2.0, m: int = 8, precision: str = "f64",
                 with_grad: bool = False, device="cuda", tiles: Optional[Sequence[int]] = None,
                 window: str = "kaiser_bessel", method: str = "auto", deterministic: bool = False):
        lib = _load()
        self.device = _require_gpu(device)
        if isinstance(M, int):
            Ns, Ms = [tuple(int(v) for v in N)], [int(M)]
            self.batched = False
        else:
            Ns, Ms = [tuple(int(v) for v in n) for n in N], [int(v) for v in M]
            self.batched = True
        self.N, self.M = Ns, Ms
        self.B = len(Ms)
        self.d = len(Ns[0])
        if not 1 <= self.d <= 3 or any(len(n) != self.d for n in Ns) or (self.batched and self.d != 3):
            raise ValueError("N must give 1, 2 or 3 sizes per transform (batches: 3)")
        self.m, self.sigma = int(m), float(sigma)
        self.window = window
        win = _window_code(window)
        self.precision = precision
        self.prec_code = {"f64": F64, "f32": F32}[precision]
        self.cdtype = torch.complex128 if precision == "f64" else torch.complex64
        self.rdtype = torch.float64 if precision == "f64" else torch.float32
        self.with_grad = with_grad
        self._h = ctypes.c_void_p()
        Narr = (ctypes.c_int64 * (self.d * self.B))(*[v for n in Ns for v in n])
        Marr = (ctypes.c_int64 * self.B)(*Ms)
        flags = (WITH_GRADIENT if with_grad else 0) | (DETERMINISTIC if deterministic else 0)
        with torch.cuda.device(self.device):
            if self.batched:
                rc = lib.hpnfft_batch_create(ctypes.byref(self._h), self.B, Narr, Marr, self.sigma, self.m,
                                             win, self.prec_code, flags)
            else:
                rc = lib.hpnfft_plan_create(ctypes.byref(self._h), self.d, Narr, Ms[0], self.sigma, self.m,
                                            win, self.prec_code, flags)
        _check(rc, "plan_create")
        if method != "auto":
            _check(lib.hpnfft_set_method(self._h, METHODS[method]), "set_method")
        self.Mtot = sum(Ms)
        self.Ftot = sum(math.prod(n) for n in Ns)
        if tiles is not None:
            _check(lib.hpnfft_set_tiles(self._h, *[int(v) for v in tiles]), "set_tiles")
        self._alloc_workspace()
        self.have_points = False
        # incremented by every set_points: autograd's backward re-sets its
        # forward's points when another call has replaced them since
        self.points_generation = 0

    # -- internals ---------------------------------------------------------
    def _alloc_workspace(self):
        lib = _load()
        sz = ctypes.c_size_t()
        _check(lib.hpnfft_workspace_size(self._h, ctypes.byref(sz)), "workspace_size")
        self.ws_bytes = int(sz.value)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        self._ws_ptr = base + off
        self._sync_stream()
        _check(lib.hpnfft_set_workspace(self._h, ctypes.c_void_p(self._ws_ptr), self.ws_bytes),
               "set_workspace")

    def _sync_stream(self):
        _check(_load().hpnfft_set_stream(self._h, _stream_ptr(self.device)), "set_stream")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.hpnfft_plan_destroy(h)
            self._h = None

    def _vals(self, t: torch.Tensor, n: int, name: str) -> torch.Tensor:
        if t.device != self.device or t.dtype != self.cdtype:
            raise TypeError("%s must be %s on %s" % (name, self.cdtype, self.device))
        if t.numel() != n:
            raise ValueError("%s must have %d elements" % (name, n))
        return t.contiguous()

    # -- API ---------------------------------------------------------------
    @property
    def method(self) -> str:
        """Sweep method in use: "lines", "boxes" or "mixed" (a batch using both)."""
        v = ctypes.c_int()
        _check(_load().hpnfft_get_method(self._h, ctypes.byref(v)), "get_method")
        return {METHOD_LINES: "lines", METHOD_BOXES: "boxes", METHOD_MIXED: "mixed"}[v.value]

    @property
    def tiles(self):
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(_load().hpnfft_get_tiles(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), "get_tiles")
        return a.value, b.value, c.value

    def set_tiles(self, tile: int, slab: int, threads: int):
        lib = _load()
        _check(lib.hpnfft_set_tiles(self._h, int(tile), int(slab), int(threads)), "set_tiles")
        self._alloc_workspace()
        self.have_points = False

    def set_points(self, x: torch.Tensor):
        """x: (sum M, d) float64 (or float32) on the plan's device, in [-1/2, 1/2)."""
        if x.device != self.device or x.shape != (self.Mtot, self.d):
            raise ValueError("x must be (%d, %d) on %s" % (self.Mtot, self.d, self.device))
        lib = _load()
        self._sync_stream()
        x = x.contiguous()
        self._points_copy = x
        self.points_generation += 1
        if x.dtype == torch.float64:
            fn = lib.hpnfft_batch_set_points if self.batched else lib.hpnfft_set_points
            rc = fn(self._h, _ptr(x))
        elif x.dtype == torch.float32 and not self.batched:
            rc = lib.hpnfft_set_points_f32(self._h, _ptr(x))
        else:
            raise TypeError("x must be float64 (or float32 for a single transform)")
        self.have_points = rc == OK
        _check(rc, "set_points")

    def adjoint(self, f: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Eq. (5): fhat(k) = sum_j f_j exp(-2 pi i k.x_j).  Returns (N0,N1,N2)
        (single transform) or the packed (sum prod N_b,) vector (batch)."""
        f = self._vals(f, self.Mtot, "f")
        if out is None:
            shape = tuple(self.N[0]) if not self.batched else (self.Ftot,)
            out = torch.empty(shape, dtype=self.cdtype, device=self.device)
        self._sync_stream()
        _check(_load().hpnfft_adjoint(self._h, _ptr(f), _ptr(out)), "adjoint")
        return out

    def forward(self, fhat: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Eq. (6): f_j = sum_k fhat(k) exp(+2 pi i k.x_j)."""
        fhat = self._vals(fhat, self.Ftot, "fhat")
        if out is None:
            out = torch.empty(self.Mtot, dtype=self.cdtype, device=self.device)
        self._sync_stream()
        _check(_load().hpnfft_forward(self._h, _ptr(fhat), _ptr(out)), "forward")
        return out

    def adjoint_backward(self, f: torch.Tensor, grad_fhat: torch.Tensor, need_f: bool = True,
                         need_x: bool = True):
        """(grad_f, grad_x) of a real loss through Eq. (5); see hpnfft.h."""
        if not self.with_grad:
            raise RuntimeError("plan was created without with_grad=True")
        f = self._vals(f, self.Mtot, "f")
        g = self._vals(grad_fhat, self.Ftot, "grad_fhat")
        gf = torch.empty(self.Mtot, dtype=self.cdtype, device=self.device) if need_f else None
        gx = torch.empty((self.Mtot, self.d), dtype=self.rdtype, device=self.device) if need_x else None
        self._sync_stream()
        _check(_load().hpnfft_adjoint_backward(self._h, _ptr(f), _ptr(g), _ptr(gf), _ptr(gx)),
               "adjoint_backward")
        return gf, gx

    def ewald_recip(self, S: torch.Tensor, L: float, alpha: float, want_gbar: bool = True):
        """Eq. (12) reciprocal sum (without self term) from S = A q; returns a
        0-d float64 device tensor and, optionally, dE/dRe S + i dE/dIm S."""
        S = self._vals(S, self.Ftot, "S")
        energy = torch.empty((), dtype=torch.float64, device=self.device)
        gbar = torch.empty_like(S) if want_gbar else None
        self._sync_stream()
        _check(_load().hpnfft_ewald_recip(self._h, _ptr(S), float(L), float(alpha), _ptr(energy), _ptr(gbar)),
               "ewald_recip")
        return energy, gbar

    def autotune(self, max_workspace_bytes: Optional[int] = None):
        """Time candidate tilings on the current points; keep the fastest."""
        if not self.have_points:
            raise RuntimeError("set_points first")
        lib = _load()
        # grow the workspace to fit every candidate (sizes depend on tiling)
        need = self.ws_bytes
        keep = self.tiles
        # the candidate set of hpnfft_autotune (line method: tile, slab,
        # threads; box method: box edges)
        if self.method == "boxes":
            grid = [(T, Zs, 512) for T in (8, 12, 16, 20, 24, 32) for Zs in (8, 12, 16, 20, 24, 32)]
        else:
            grid = [(T, Zs, th) for T in (4, 6, 8, 12, 16) for Zs in (8, 16, 24, 32) for th in (512, 1024)]
        for T, Zs, th in grid:
            if lib.hpnfft_set_tiles(self._h, T, Zs, th) == OK:
                sz = ctypes.c_size_t()
                lib.hpnfft_workspace_size(self._h, ctypes.byref(sz))
                need = max(need, int(sz.value))
        if max_workspace_bytes is not None:
            need = min(need, int(max_workspace_bytes))
        _check(lib.hpnfft_set_tiles(self._h, *keep), "set_tiles")
        x_keep = self._points_copy
        self.ws = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self._ws_ptr = base + ((-base) % 256)
        self.ws_bytes = need
        self._sync_stream()
        _check(lib.hpnfft_set_workspace(self._h, ctypes.c_void_p(self._ws_ptr), need), "set_workspace")
        self.set_points(x_keep)
        # nonzero values: the spread skips the grid atomics of cells that sum
        # to zero, so zeros would time every candidate without its flush
        f = torch.ones(self.Mtot, dtype=self.cdtype, device=self.device)
        fh = torch.ones(self.Ftot, dtype=self.cdtype, device=self.device)
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib.hpnfft_autotune(self._h, _ptr(f), _ptr(fh), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
               "autotune")
        return a.value, b.value, c.value

    # live timing ------------------------------------------------------------
    NPHASES = 14

    def profile(self, enable: bool = True, phases=None):
        """Record HIP events around every kernel group on the plan's stream
        (or, with phases = a list of phase names, around those only)."""
        self._sync_stream()
        if phases is None:
            _check(_load().hpnfft_profile(self._h, 1 if enable else 0), "profile")
            return
        lib = _load()
        names = {lib.hpnfft_phase_name(i).decode(): i for i in range(self.NPHASES)}
        mask = 0
        for ph in phases:
            if ph not in names:
                raise ValueError("unknown phase %r" % ph)
            mask |= 1 << names[ph]
        _check(lib.hpnfft_profile_phases(self._h, ctypes.c_uint(mask if enable else 0)), "profile_phases")

    def profile_read(self) -> dict:
        """{phase: (total_ms, launches)} for the calls since the last read."""
        import numpy as np
        ms = np.zeros(self.NPHASES, dtype=np.float64)
        cnt = np.zeros(self.NPHASES, dtype=np.int64)
        _check(_load().hpnfft_profile_read(self._h, ms.ctypes.data_as(ctypes.c_void_p),
                                           cnt.ctypes.data_as(ctypes.c_void_p)), "profile_read")
        lib = _load()
        return {lib.hpnfft_phase_name(i).decode(): (float(ms[i]), int(cnt[i]))
                for i in range(self.NPHASES) if cnt[i]}

    # batch graph
    def capture(self, f: torch.Tensor, fhat_out: torch.Tensor):
        """Record the (batch) adjoint into a HIP graph on the current stream."""
        f = self._vals(f, self.Mtot, "f")
        self._graph_bufs = (f, fhat_out)
        self._sync_stream()
        _check(_load().hpnfft_batch_capture(self._h, _ptr(f), _ptr(fhat_out)), "batch_capture")

    def replay(self):
        self._sync_stream()
        _check(_load().hpnfft_batch_launch(self._h), "batch_launch")

    def offsets(self, b: int):
        po, fo = ctypes.c_int64(), ctypes.c_int64()
        _check(_load().hpnfft_batch_offsets(self._h, int(b), ctypes.byref(po), ctypes.byref(fo)), "offsets")
        return po.value, fo.value

    def info(self):
        n = (ctypes.c_int64 * 3)()
        M = ctypes.c_int64()
        _check(_load().hpnfft_plan_info(self._h, n, ctypes.byref(M)), "plan_info")
        return tuple(n)[:self.d], M.value


class NFFTAdjoint(torch.autograd.Function):
    """fhat = A(x) f (Eq. (5)) with gradients with respect to x and f."""

    @staticmethod
    def forward(ctx, x, f, plan: Plan):
        plan.set_points(x.detach())
        fhat = plan.adjoint(f.detach())
        ctx.save_for_backward(x.detach(), f.detach())
        ctx.plan = plan
        ctx.generation = plan.points_generation
        return fhat

    @staticmethod
    def backward(ctx, grad_fhat):
        x, f = ctx.saved_tensors
        plan = ctx.plan
        # the plan may hold other points by now (another transform or
        # set_points on the same plan ran after this forward): restore ours
        if plan.points_generation != ctx.generation:
            plan.set_points(x)
            ctx.generation = plan.points_generation
        need_x, need_f = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        gf, gx = plan.adjoint_backward(f, grad_fhat.contiguous(), need_f=need_f, need_x=need_x)
        if gx is not None and gx.dtype != torch.float64:
            gx = gx.to(torch.float64)
        return gx, gf, None


def nfft_adjoint(x: torch.Tensor, f: torch.Tensor, plan: Plan) -> torch.Tensor:
    """Differentiable Eq. (5) transform on the given plan."""
    return NFFTAdjoint.apply(x, f, plan)


def check_points(x) -> int:
    """Host-side domain check of an (M, d) float64 array: -1 if every
    coordinate lies in [-1/2, 1/2), else the index of the first point that
    does not (no GPU needed)."""
    import numpy as np
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if x.ndim != 2:
        raise ValueError("x must be (M, d)")
    bad = ctypes.c_int64()
    rc = _load().hpnfft_check_points(x.ctypes.data_as(ctypes.c_void_p), x.shape[0], x.shape[1],
                                     ctypes.byref(bad))
    if rc not in (OK, EDOMAIN):
        _check(rc, "check_points")
    return int(bad.value)


def device_copy(dst: torch.Tensor, src: torch.Tensor):
    """dst <- src with the library's streaming copy kernel (same byte size,
    contiguous, 16-byte aligned), on the current stream."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes or not (dst.is_contiguous() and src.is_contiguous()):
        raise ValueError("dst and src must be contiguous with the same byte size")
    _check(_load().hpnfft_copy(_ptr(dst), _ptr(src), nbytes, _stream_ptr(src.device)), "copy")


def _window_code(window) -> int:
    if isinstance(window, int):
        return window
    if window not in WINDOWS:
        raise ValueError("window must be one of %s" % sorted(WINDOWS))
    return WINDOWS[window]


def window_eval(m: int, sigma: float, t, window="kaiser_bessel"):
    """Host-only helper: a normalised window of the family and its derivative."""
    import numpy as np
    t = np.ascontiguousarray(np.asarray(t, dtype=np.float64))
    phi = np.empty_like(t)
    dphi = np.empty_like(t)
    _check(_load().hpnfft_window_eval(_window_code(window), int(m), float(sigma), t.size,
                                      t.ctypes.data_as(ctypes.c_void_p),
                                      phi.ctypes.data_as(ctypes.c_void_p), dphi.ctypes.data_as(ctypes.c_void_p)),
           "window_eval")
    return phi, dphi


def window_rolloff(m: int, sigma: float, n: int, N: int, window="kaiser_bessel"):
    """Host-only helper: roll-off factors 1/D(k) for k = -N/2 .. N/2-1."""
    import numpy as np
    out = np.empty(N, dtype=np.float64)
    _check(_load().hpnfft_window_rolloff(_window_code(window), int(m), float(sigma), int(n), int(N),
                                         out.ctypes.data_as(ctypes.c_void_p)), "window_rolloff")
    return out


def window_error_bound(m: int, sigma: float, window="kaiser_bessel") -> float:
    """Host-only helper: the library's a-priori one-dimensional error bound E
    (|approximate - exact| <= E ||input||_1 per output)."""
    out = ctypes.c_double()
    _check(_load().hpnfft_window_error_bound(_window_code(window), int(m), float(sigma), ctypes.byref(out)),
           "window_error_bound")
    return out.value
