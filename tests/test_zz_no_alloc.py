"""The allocation-free variant of the real-space Ewald sum (Eq. (11)).

hpnfft_ewald_real_static keeps its block partial sums in the library's
static device array instead of a caller buffer.  Called through the C-ABI
twice in a row, the second time with fewer ions, it must give the same
energy and forces as hpnfft_ewald_real with a caller-provided scratch
buffer (same kernels, same summation order: bit for bit), and it must
refuse ion counts beyond its fixed capacity before launching anything.
"""
import ctypes
import math

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


def _both(H, cells, seed):
    r, q, L = W.fluorite(cells, displacement_std=0.05, seed=seed)
    M = r.shape[0]
    alpha, rcut = 1.5, 0.5 * L
    dev = torch.device("cuda", 0)
    rt = torch.from_numpy(np.mod(r, L)).to(dev).contiguous()
    qt = torch.from_numpy(q).to(dev).contiguous()
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    lib = H._load()

    e_ref = torch.empty((), dtype=torch.float64, device=dev)
    f_ref = torch.empty((M, 3), dtype=torch.float64, device=dev)
    part = torch.empty(math.ceil(M / 256), dtype=torch.float64, device=dev)
    rc = lib.hpnfft_ewald_real(H._ptr(rt), H._ptr(qt), M, L, alpha, rcut, H._ptr(e_ref), H._ptr(f_ref),
                               H._ptr(part), stream)
    assert rc == H.OK, H.HpnfftError(rc, "ewald_real")

    e_st = torch.full((), float("nan"), dtype=torch.float64, device=dev)
    f_st = torch.full((M, 3), float("nan"), dtype=torch.float64, device=dev)
    rc = lib.hpnfft_ewald_real_static(H._ptr(rt), H._ptr(qt), M, L, alpha, rcut, H._ptr(e_st), H._ptr(f_st),
                                      stream)
    assert rc == H.OK, H.HpnfftError(rc, "ewald_real_static")
    torch.cuda.synchronize()
    return M, e_ref.item(), f_ref.cpu(), e_st.item(), f_st.cpu()


def test_static_variant_matches_scratch_variant_twice(H):
    results = []
    for cells, seed in ((3, 11), (2, 12)):     # second call: fewer ions
        M, e_ref, f_ref, e_st, f_st = _both(H, cells, seed)
        print("ewald_real_static: cells=%d M=%d energy %.15e (scratch variant %.15e)" % (cells, M, e_st, e_ref),
              flush=True)
        assert math.isfinite(e_ref) and e_ref != 0.0
        assert e_st == e_ref
        assert torch.equal(f_st, f_ref)
        results.append(M)
    assert results[1] < results[0]


def test_static_variant_rejects_oversize(H):
    lib = H._load()
    cap = lib.hpnfft_ewald_real_static_max_ions()
    assert cap == 65536 * 256
    dev = torch.device("cuda", 0)
    buf = torch.zeros(8, dtype=torch.float64, device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    # refused on the host before any launch: the small buffers are never read
    rc = lib.hpnfft_ewald_real_static(H._ptr(buf), H._ptr(buf), cap + 1, 10.0, 1.0, 2.0, H._ptr(buf), None,
                                      stream)
    assert rc == H.ESIZE
    assert b"scratch" in lib.hpnfft_strerror(rc)
