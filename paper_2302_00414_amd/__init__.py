"""MI355X (gfx950) weighted adjoint NFFT: the reconstruction step of the
direct inverse NFFT by density compensation (Kircheis & Potts, arXiv
2302.00414, eq. (3.7) / Algorithm 3.7), fhat ~ D^* F^* B^* W f, and the
forward NFFT A ~ B F D (Algorithm 2.1).

The compute path is the HIP library ``libnfft_mi355x.so`` behind the C ABI of
``include/nfft.h``; :mod:`paper_2302_00414_amd.nfft` is a thin PyTorch/ctypes
binding with the same entry-point names. Importing this package does not
load the library; creating a plan does, and fails loudly if it is missing.
"""
__all__ = ["nfft", "workloads", "build"]
