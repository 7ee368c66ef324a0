"""MI355X-native NUFFT pair of PyNUFFT (arXiv 1710.03197): A = V F S and
A^H = S^H F^H V^H on gfx950, behind the C ABI of include/nufft_mi355x.h.

Submodules:
  data      seeded synthetic trajectories, phantoms and coil maps (numpy)
  plan      Plan: ctypes binding of the C ABI over torch device tensors
  autograd  NufftFunction: torch.autograd.Function with hand-written backward
  solvers   conjugate gradient on the normal equations (Section 2.2)
  build     hipcc build of libnufft_mi355x.so
"""

__all__ = ["Plan", "NufftError", "nufft", "data"]


def __getattr__(name):
    # lazy: importing the package (e.g. for `data`) does not load the GPU library
    if name == "Plan":
        from .plan import Plan
        return Plan
    if name == "NufftError":
        from ._lib import NufftError
        return NufftError
    if name == "nufft":
        from .autograd import nufft
        return nufft
    raise AttributeError(name)
