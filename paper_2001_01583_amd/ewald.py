"""Ewald electrostatics with the NFFT structure factor (Section 5 of the paper).

  Eq. (11)  U^R = 1/2 sum'_n sum_{i,j} q_i q_j erfc(alpha |r_ij + n L|) / |r_ij + n L|
  Eq. (12)  U^K = 1/(2 pi L) sum_{k != 0} exp(-pi^2 |k|^2 / (alpha L)^2) / |k|^2 |S(k)|^2
                  - alpha / sqrt(pi) sum_i q_i^2,
            S(k) = sum_i q_i exp(-2 pi i k.r_i / L)  =  Eq. (5) with f = q, x = r / L
  Eq. (10)  Madelung = -U m / (N Z+ |Z-|)   (m ions per formula unit)

The structure factor is the library's adjoint transform; the reciprocal
energy and its derivative dU/dRe S + i dU/dIm S are a library kernel (float64
reduction); forces come from the adjoint's backward,
F_i = -(1/L) d U / d x_i.  The k sum runs over the NFFT frequency box I_N
without k = 0.  The real-space part is a library kernel too: a cell-list
pair sum when the box holds at least three cut-off lengths, else a direct
minimum-image pair sum.
"""
from __future__ import annotations

import ctypes
import math
from typing import Optional, Sequence

import torch

from . import hpnfft as H


def alpha_window(L_box: float, N: int, eps: float = 1e-12):
    """Range of the Ewald parameter for which both sums reach `eps`:
    real space within L/2 needs alpha >= 2 sqrt(ln(1/eps)) / L, the
    reciprocal cube |k| <= N/2 needs alpha <= pi N / (2 L sqrt(ln(1/eps)))."""
    ell = math.log(1.0 / eps)
    return 2.0 * math.sqrt(ell) / L_box, math.pi * N / (2.0 * L_box * math.sqrt(ell))


def _smooth(v: int) -> bool:
    for p in (2, 3, 5, 7):
        while v % p == 0:
            v //= p
    return v == 1


def parameters(L_box: float, alpha: float, eps: float = 1e-12, sigma: float = 2.0):
    """Cut-off and bandwidth that bring both Ewald sums to `eps` at a given
    alpha (the inverse of alpha_window): rcut = sqrt(ln(1/eps)) / alpha, and
    the smallest even N >= 2 alpha L sqrt(ln(1/eps)) / pi whose grid
    sigma N factors into 2, 3, 5, 7."""
    ell = math.sqrt(math.log(1.0 / eps))
    rcut = ell / alpha
    N = int(math.ceil(2.0 * alpha * L_box * ell / math.pi))
    N += N % 2
    while not (_smooth(int(round(sigma * N))) and abs(sigma * N - round(sigma * N)) < 1e-9
               and int(round(sigma * N)) % 2 == 0):
        N += 2
    return rcut, N


def madelung_constant(U: float, n_ions: int, ions_per_formula: int = 3, z_plus: int = 2,
                      z_minus: int = 1) -> float:
    """Eq. (10) with the sign that makes an attractive lattice positive."""
    return -U * ions_per_formula / (n_ions * z_plus * z_minus)


class Ewald:
    """Reciprocal (NFFT) plus real-space Ewald energy and forces of M charges
    in a cubic box of side L (positions anywhere; wrapped periodically)."""

    def __init__(self, M: int, L_box: float, alpha: float, N: Sequence[int] = (64, 64, 64), m: int = 8,
                 precision: str = "f64", rcut: Optional[float] = None, device="cuda", real_method: str = "auto",
                 method: str = "auto"):
        self.M, self.L, self.alpha = int(M), float(L_box), float(alpha)
        self.rcut = float(rcut) if rcut is not None else 0.5 * self.L
        self.plan = H.Plan(tuple(N), self.M, m=m, precision=precision, with_grad=True, device=device,
                           method=method)
        self.device = self.plan.device
        if real_method not in ("auto", "cells", "direct"):
            raise ValueError("real_method must be auto, cells or direct")
        can_cells = self.L >= 3.0 * self.rcut
        if real_method == "cells" and not can_cells:
            raise ValueError("cell lists need L >= 3 rcut")
        self.real_method = ("cells" if can_cells else "direct") if real_method == "auto" else real_method
        if self.real_method == "cells":
            sz = ctypes.c_size_t()
            H._check(H._load().hpnfft_ewald_real_cells_workspace(self.M, self.L, self.rcut, ctypes.byref(sz)),
                     "ewald_real_cells_workspace")
            self._cells_bytes = int(sz.value)
            self._cells_ws = torch.empty(self._cells_bytes + 256, dtype=torch.uint8, device=self.device)
            self._cells_ptr = self._cells_ws.data_ptr() + ((-self._cells_ws.data_ptr()) % 256)
        else:
            self._scratch = torch.empty((self.M + 255) // 256 + 8, dtype=torch.float64, device=self.device)

    def autotune(self, r: torch.Tensor):
        """Pick the plan's tiling on these positions (once per lattice; the
        timing covers the adjoint and the gradient used for forces)."""
        self.plan.set_points(self._unit(r.to(torch.float64)))
        return self.plan.autotune()

    def _unit(self, r: torch.Tensor) -> torch.Tensor:
        x = r / self.L
        x = x - torch.floor(x + 0.5)
        # rounding can leave exactly +1/2; map it to -1/2 (same periodic point)
        return torch.where(x >= 0.5, x - 1.0, x).contiguous()

    def reciprocal(self, r: torch.Tensor, q: torch.Tensor, forces: bool = True):
        """(U^K including the self term, F^K) via the NFFT (Eq. (12))."""
        plan = self.plan
        plan.set_points(self._unit(r.to(torch.float64)))
        qc = q.to(plan.cdtype).contiguous()
        S = plan.adjoint(qc)
        e, gbar = plan.ewald_recip(S, self.L, self.alpha, want_gbar=forces)
        self_term = self.alpha / math.sqrt(math.pi) * torch.sum(q.to(torch.float64) ** 2)
        U = e - self_term
        F = None
        if forces:
            _, gx = plan.adjoint_backward(qc, gbar.reshape(-1), need_f=False, need_x=True)
            F = -gx.to(torch.float64) / self.L
        return U, F

    def real_space(self, r: torch.Tensor, q: torch.Tensor, forces: bool = True):
        """(U^R, F^R) of Eq. (11): cell-list pairs within rcut, or direct
        minimum-image pairs (library kernels)."""
        r = r.to(torch.float64).contiguous()
        q = q.to(torch.float64).contiguous()
        energy = torch.empty((), dtype=torch.float64, device=self.device)
        F = torch.empty((self.M, 3), dtype=torch.float64, device=self.device) if forces else None
        stream = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
        if self.real_method == "cells":
            rc = H._load().hpnfft_ewald_real_cells(H._ptr(r), H._ptr(q), self.M, self.L, self.alpha, self.rcut,
                                                   H._ptr(energy), H._ptr(F), ctypes.c_void_p(self._cells_ptr),
                                                   self._cells_bytes, stream)
            H._check(rc, "ewald_real_cells")
        else:
            rc = H._load().hpnfft_ewald_real(H._ptr(r), H._ptr(q), self.M, self.L, self.alpha, self.rcut,
                                             H._ptr(energy), H._ptr(F), H._ptr(self._scratch), stream)
            H._check(rc, "ewald_real")
        return energy, F

    def energy_forces(self, r: torch.Tensor, q: torch.Tensor, forces: bool = True):
        Uk, Fk = self.reciprocal(r, q, forces)
        Ur, Fr = self.real_space(r, q, forces)
        return Uk + Ur, (Fk + Fr) if forces else None


def reciprocal_energy_autograd(r: torch.Tensor, q: torch.Tensor, ew: Ewald) -> torch.Tensor:
    """U^K written with the differentiable transform (NFFTAdjoint) so that
    torch.autograd gives the forces; the energy reduction itself is the
    library's float64 kernel wrapped as a custom function."""
    x = ew._unit(r.to(torch.float64))
    qc = q.to(ew.plan.cdtype)
    S = H.nfft_adjoint(x, qc, ew.plan)
    return _RecipEnergy.apply(S, ew) - ew.alpha / math.sqrt(math.pi) * torch.sum(q.to(torch.float64) ** 2)


class _RecipEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, S, ew: Ewald):
        e, gbar = ew.plan.ewald_recip(S.contiguous(), ew.L, ew.alpha, want_gbar=True)
        ctx.save_for_backward(gbar)
        return e

    @staticmethod
    def backward(ctx, ge):
        (gbar,) = ctx.saved_tensors
        return gbar * ge.to(gbar.real.dtype), None
