"""MI355X (gfx950) particle-particle ladder of the Cholesky-vector CC vector
function (arXiv 2310.04559, eqs. cholesky and vfunction).

Submodules:
  native  -- ctypes binding of libccladder.so (the C ABI in include/ccladder.h)
  ladder  -- torch.autograd.Function over the forward and adjoint entry points
  inputs  -- seeded synthetic workloads
  build   -- hipcc build of the library
Importing the package loads nothing native; ``native.load()`` does, and fails
loudly when the library is not built.
"""
__all__ = ["native", "ladder", "inputs", "build"]
