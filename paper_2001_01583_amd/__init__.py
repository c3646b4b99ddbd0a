"""hpnfft: nonequispaced FFT (the NFFT evaluation of the NDFT, Eq. (5) of
Yang & Wang, arXiv 2001.01583, and its transpose Eq. (6)) on AMD MI355X.

The compute path is the HIP library libhpnfft.so (C-ABI in include/hpnfft.h);
this package only binds it.  Build it with ``paper_2001_01583_amd.build.build()``.
"""
from .hpnfft import (HpnfftError, NFFTAdjoint, Plan, declared_symbols, nfft_adjoint,  # noqa: F401
                     window_eval, window_rolloff)

__all__ = ["Plan", "NFFTAdjoint", "nfft_adjoint", "HpnfftError", "declared_symbols",
           "window_eval", "window_rolloff"]
