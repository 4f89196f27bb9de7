"""libtdse: gfx950 (MI355X) batched 1D-TDSE microscopic solver of the
multiscale high-harmonic-generation model of arXiv 2507.04115.

Submodules:
  binding   ctypes binding of the C-ABI (include/libtdse.h)
  autograd  torch.autograd.Function over the forward and adjoint kernels
  build     hipcc build of libtdse.so
"""
__all__ = ["binding", "autograd", "build"]
