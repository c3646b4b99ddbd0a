"""Real-space Ewald sum of Eq. (11) with cell lists (Section 5's HP-ENUF
runs reach 12 * 64^3 ions, beyond a direct O(M^2) pair sum).

  * against the direct Ewald oracle (all pairs over the 27 nearest images)
    on a displaced fluorite lattice, energy and every force;
  * against the library's direct minimum-image kernel on random charges at
    random (partly out-of-box) positions: the same truncated sum;
  * bitwise reproducible (one writer per force, fixed-order energy sum);
  * argument checks (L >= 3 rcut, workspace size).
"""
import ctypes

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


def _cells(H, r, q, L, alpha, rcut):
    dev = torch.device("cuda", 0)
    M = r.shape[0]
    lib = H._load()
    sz = ctypes.c_size_t()
    assert lib.hpnfft_ewald_real_cells_workspace(M, L, rcut, ctypes.byref(sz)) == H.OK
    ws = torch.empty(sz.value + 256, dtype=torch.uint8, device=dev)
    ptr = ws.data_ptr() + ((-ws.data_ptr()) % 256)
    rt = torch.from_numpy(np.ascontiguousarray(r)).to(dev)
    qt = torch.from_numpy(np.ascontiguousarray(q)).to(dev)
    e = torch.empty((), dtype=torch.float64, device=dev)
    F = torch.empty((M, 3), dtype=torch.float64, device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    rc = lib.hpnfft_ewald_real_cells(H._ptr(rt), H._ptr(qt), M, L, alpha, rcut, H._ptr(e), H._ptr(F),
                                     ctypes.c_void_p(ptr), sz.value, stream)
    assert rc == H.OK, H.HpnfftError(rc, "ewald_real_cells")
    return e.item(), F.cpu().numpy()


def _direct(H, r, q, L, alpha, rcut):
    dev = torch.device("cuda", 0)
    M = r.shape[0]
    rt = torch.from_numpy(np.ascontiguousarray(r)).to(dev)
    qt = torch.from_numpy(np.ascontiguousarray(q)).to(dev)
    e = torch.empty((), dtype=torch.float64, device=dev)
    F = torch.empty((M, 3), dtype=torch.float64, device=dev)
    part = torch.empty((M + 255) // 256, dtype=torch.float64, device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    rc = H._load().hpnfft_ewald_real(H._ptr(rt), H._ptr(qt), M, L, alpha, rcut, H._ptr(e), H._ptr(F),
                                     H._ptr(part), stream)
    assert rc == H.OK
    return e.item(), F.cpu().numpy()


def test_cells_against_direct_oracle(H, oracle_mod):
    r, q, L = W.fluorite(8, displacement_std=0.01, seed=81)
    alpha = 1.2
    rcut = L / 3.0           # erfc(alpha rcut) ~ 1e-25: the truncation is below rounding
    U, F = _cells(H, r, q, L, alpha, rcut)
    Uo, Fo = oracle_mod.ewald_real(r, q, L, alpha, 1, forces=True)
    eu = abs(U - Uo) / abs(Uo)
    ef = np.max(np.abs(F - Fo)) / np.max(np.abs(Fo))
    print("cells vs oracle (6144 ions): energy %.3e forces %.3e" % (eu, ef))
    assert eu <= 1e-12 and ef <= 1e-11


@pytest.mark.parametrize("M,L,rcut", [(5000, 20.0, 6.0), (20000, 31.0, 4.5), (777, 13.0, 4.3)])
def test_cells_equal_direct_kernel(H, M, L, rcut):
    g = W.rng(900 + M)
    r = (g.random((M, 3)) * 1.4 - 0.2) * L        # some ions outside [0, L)
    q = g.standard_normal(M)
    alpha = 1.0
    U, F = _cells(H, r, q, L, alpha, rcut)
    Ud, Fd = _direct(H, r, q, L, alpha, rcut)
    eu = abs(U - Ud) / abs(Ud)
    ef = np.max(np.abs(F - Fd)) / np.max(np.abs(Fd))
    print("cells vs direct kernel M=%d L=%g rcut=%g: energy %.3e forces %.3e" % (M, L, rcut, eu, ef))
    assert eu <= 1e-12 and ef <= 1e-12


def test_cells_bitwise_reproducible(H):
    r, q, L = W.fluorite(6, displacement_std=0.05, seed=66)
    a = _cells(H, r, q, L, 1.3, 4.0)
    b = _cells(H, r, q, L, 1.3, 4.0)
    assert a[0] == b[0] and np.array_equal(a[1], b[1])


def test_cells_argument_checks(H):
    lib = H._load()
    sz = ctypes.c_size_t()
    assert lib.hpnfft_ewald_real_cells_workspace(100, 10.0, 4.0, ctypes.byref(sz)) == H.EINVAL  # L < 3 rcut
    assert lib.hpnfft_ewald_real_cells_workspace(100, 12.0, 4.0, ctypes.byref(sz)) == H.OK
    buf = torch.zeros(1024, dtype=torch.float64, device="cuda")
    rc = lib.hpnfft_ewald_real_cells(H._ptr(buf), H._ptr(buf), 100, 12.0, 1.0, 4.0, H._ptr(buf), None,
                                     ctypes.c_void_p(buf.data_ptr()), 16, None)
    assert rc == H.ENOMEM   # refused before any launch
