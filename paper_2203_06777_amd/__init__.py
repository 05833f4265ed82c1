"""MI355X-native domain-wall fermion operator library (HIP kernels behind a C ABI).

Submodules:
  dwf       ctypes binding of libdwf.so (entry points under the C names) and a Context helper
  autograd  torch.autograd Functions: the linear operator D_DW and the action phi^dag (D^dag D)^-1 phi
  build     compiles libdwf.so for gfx950 with hipcc
"""

__all__ = ["dwf", "autograd", "build"]
