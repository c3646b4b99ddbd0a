"""FP64 CPU oracle for the NDFT (test infrastructure only).

Plain direct evaluation of the paper's Eq. (5) (the NDFT), Eq. (6) (its
transpose), the analytic gradient of Eq. (5), the Ewald energy of
Eqs. (10)-(12) and the Eq. (9) error metric.  The arithmetic lives in
``ndft.c`` (plain C, IEEE double, OpenMP over outputs, compensated sums); this
module only builds and calls it.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ndft.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_f64p = ctypes.POINTER(ctypes.c_double)


def build(force: bool = False) -> str:
    """Compile ndft.c into liboracle.so with gcc (no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            lib.oracle_ndft_adjoint.argtypes = [ctypes.c_int, _i64p, ctypes.c_int64, _f64p, _f64p,
                                                ctypes.c_int64, _i64p, _f64p]
            lib.oracle_ndft_forward.argtypes = lib.oracle_ndft_adjoint.argtypes
            lib.oracle_ndft_adjoint_grad.argtypes = [ctypes.c_int, _i64p, ctypes.c_int64, _f64p, _f64p,
                                                     _f64p, ctypes.c_int64, _i64p, _f64p, _f64p]
            for fn in (lib.oracle_ndft_adjoint, lib.oracle_ndft_forward, lib.oracle_ndft_adjoint_grad):
                fn.restype = ctypes.c_int
            lib.oracle_ewald_real.argtypes = [ctypes.c_int64, _f64p, _f64p, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_int, _f64p]
            lib.oracle_ewald_real.restype = ctypes.c_double
            lib.oracle_ewald_recip.argtypes = [ctypes.c_int64, _f64p, _f64p, ctypes.c_double,
                                               ctypes.c_double, ctypes.c_int]
            lib.oracle_ewald_recip.restype = ctypes.c_double
            lib.oracle_ewald_recip_forces.argtypes = [ctypes.c_int64, _f64p, _f64p, ctypes.c_double,
                                                      ctypes.c_double, ctypes.c_int, _f64p, _f64p]
            lib.oracle_ewald_recip_forces.restype = ctypes.c_int
            lib.oracle_ewald_recip_sel.argtypes = [ctypes.c_int64, _f64p, _f64p, ctypes.c_double,
                                                   ctypes.c_double, ctypes.c_int, ctypes.c_int64, _i64p,
                                                   _f64p, _f64p]
            lib.oracle_ewald_recip_sel.restype = ctypes.c_double
            lib.oracle_rel_l2.argtypes = [ctypes.c_int64, _f64p, _f64p]
            lib.oracle_rel_l2.restype = ctypes.c_double
            lib.oracle_threads.argtypes = []
            lib.oracle_threads.restype = ctypes.c_int
            _lib = lib
    return _lib


def _p(a, t=_f64p):
    return a.ctypes.data_as(t)


def _cplx(a) -> np.ndarray:
    """complex array -> contiguous interleaved float64 view source."""
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


def _prep(N, x):
    N = np.ascontiguousarray(np.asarray(N, dtype=np.int64))
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    d = N.size
    if x.ndim != 2 or x.shape[1] != d:
        raise ValueError("x must be M x d")
    return N, x, d


def ndft_adjoint(N, x, f, kidx=None) -> np.ndarray:
    """Eq. (5): fhat(k) = sum_j f_j exp(-2 pi i k.x_j) for k in I_N.

    Returns the full C-order array of shape N (frequency k_t at index
    k_t + N_t/2) when ``kidx`` is None, else the values at the given linear
    indices of that array.
    """
    N, x, d = _prep(N, x)
    f = _cplx(f).reshape(-1)
    M = x.shape[0]
    if f.size != M:
        raise ValueError("f must have M entries")
    lib = _load()
    if kidx is None:
        nk = int(np.prod(N))
        out = np.empty(nk, dtype=np.complex128)
        rc = lib.oracle_ndft_adjoint(d, _p(N, _i64p), M, _p(x), _p(f.view(np.float64)), nk, None,
                                     _p(out.view(np.float64)))
        if rc:
            raise RuntimeError("oracle_ndft_adjoint failed")
        return out.reshape(tuple(N))
    kidx = np.ascontiguousarray(np.asarray(kidx, dtype=np.int64))
    out = np.empty(kidx.size, dtype=np.complex128)
    rc = lib.oracle_ndft_adjoint(d, _p(N, _i64p), M, _p(x), _p(f.view(np.float64)), kidx.size,
                                 _p(kidx, _i64p), _p(out.view(np.float64)))
    if rc:
        raise RuntimeError("oracle_ndft_adjoint failed")
    return out


def ndft_forward(N, x, fhat, jidx=None) -> np.ndarray:
    """Eq. (6): f(x_j) = sum_{k in I_N} fhat(k) exp(+2 pi i k.x_j)."""
    N, x, d = _prep(N, x)
    fh = _cplx(fhat).reshape(-1)
    if fh.size != int(np.prod(N)):
        raise ValueError("fhat must have #I_N entries")
    M = x.shape[0]
    lib = _load()
    if jidx is None:
        out = np.empty(M, dtype=np.complex128)
        rc = lib.oracle_ndft_forward(d, _p(N, _i64p), M, _p(x), _p(fh.view(np.float64)), M, None,
                                     _p(out.view(np.float64)))
    else:
        jidx = np.ascontiguousarray(np.asarray(jidx, dtype=np.int64))
        out = np.empty(jidx.size, dtype=np.complex128)
        rc = lib.oracle_ndft_forward(d, _p(N, _i64p), M, _p(x), _p(fh.view(np.float64)), jidx.size,
                                     _p(jidx, _i64p), _p(out.view(np.float64)))
    if rc:
        raise RuntimeError("oracle_ndft_forward failed")
    return out


def ndft_adjoint_grad(N, x, f, gbar, jidx=None):
    """Analytic gradient of a real loss through Eq. (5).

    ``gbar`` = dL/dRe fhat + i dL/dIm fhat over all of I_N.  Returns
    (grad_f, grad_x) with grad_f in the same (dL/dRe + i dL/dIm) convention.
    """
    N, x, d = _prep(N, x)
    f = _cplx(f).reshape(-1)
    g = _cplx(gbar).reshape(-1)
    M = x.shape[0]
    lib = _load()
    if jidx is None:
        nj, jp = M, None
    else:
        jidx = np.ascontiguousarray(np.asarray(jidx, dtype=np.int64))
        nj, jp = jidx.size, _p(jidx, _i64p)
    gf = np.empty(nj, dtype=np.complex128)
    gx = np.empty((nj, d), dtype=np.float64)
    rc = lib.oracle_ndft_adjoint_grad(d, _p(N, _i64p), M, _p(x), _p(f.view(np.float64)),
                                      _p(g.view(np.float64)), nj, jp, _p(gf.view(np.float64)), _p(gx))
    if rc:
        raise RuntimeError("oracle_ndft_adjoint_grad failed")
    return gf, gx


def ewald_real(r, q, L, alpha, nshell, forces=False):
    """Eq. (11) real-space Ewald energy (and forces) over |n_t| <= nshell images."""
    r = np.ascontiguousarray(np.asarray(r, dtype=np.float64))
    q = np.ascontiguousarray(np.asarray(q, dtype=np.float64))
    lib = _load()
    F = np.empty_like(r) if forces else None
    e = lib.oracle_ewald_real(q.size, _p(r), _p(q), float(L), float(alpha), int(nshell),
                              _p(F) if forces else None)
    return (e, F) if forces else e


def ewald_recip(r, q, L, alpha, kmax):
    """Eq. (12) reciprocal-space Ewald energy over the cube |n_t| <= kmax."""
    r = np.ascontiguousarray(np.asarray(r, dtype=np.float64))
    q = np.ascontiguousarray(np.asarray(q, dtype=np.float64))
    return _load().oracle_ewald_recip(q.size, _p(r), _p(q), float(L), float(alpha), int(kmax))


def ewald_recip_forces(r, q, L, alpha, kmax):
    """Forces -dU/dr of Eq. (12), structure factors summed directly."""
    r = np.ascontiguousarray(np.asarray(r, dtype=np.float64))
    q = np.ascontiguousarray(np.asarray(q, dtype=np.float64))
    side = 2 * int(kmax) + 1
    S = np.empty(2 * side ** 3, dtype=np.float64)
    F = np.empty_like(r)
    _load().oracle_ewald_recip_forces(q.size, _p(r), _p(q), float(L), float(alpha), int(kmax),
                                      _p(S), _p(F))
    return F


def ewald_recip_selected(r, q, L, alpha, kmax, sel):
    """Eq. (12) energy (self term included) and the forces of the ions listed
    in ``sel`` only.  Returns (U, F[len(sel), 3], S) with S the structure
    factors over the cube |n_t| <= kmax (complex, n_0 slowest)."""
    r = np.ascontiguousarray(np.asarray(r, dtype=np.float64))
    q = np.ascontiguousarray(np.asarray(q, dtype=np.float64))
    sel = np.ascontiguousarray(np.asarray(sel, dtype=np.int64))
    side = 2 * int(kmax) + 1
    S = np.empty(2 * side ** 3, dtype=np.float64)
    F = np.empty((sel.size, 3), dtype=np.float64)
    U = _load().oracle_ewald_recip_sel(q.size, _p(r), _p(q), float(L), float(alpha), int(kmax), sel.size,
                                       _p(sel, _i64p), _p(S), _p(F))
    return U, F, S.view(np.complex128)


def threads() -> int:
    """Host threads the oracle's parallel loops use."""
    return int(_load().oracle_threads())


def rel_l2(a, s) -> float:
    """Eq. (9): ||a - s||_2 / ||s||_2 over complex vectors."""
    a = _cplx(a).reshape(-1)
    s = _cplx(s).reshape(-1)
    if a.size != s.size:
        raise ValueError("size mismatch")
    return float(_load().oracle_rel_l2(a.size, _p(a.view(np.float64)), _p(s.view(np.float64))))


def madelung_from_energy(U, n_ions, ions_per_molecule=3, z_plus=2, z_minus=1):
    """Eq. (10) with the sign fixed so that an attractive lattice gives a
    positive constant: -U * m / (N * Z+ * |Z-|)."""
    return -U * ions_per_molecule / (n_ions * z_plus * z_minus)
