"""MI355X (gfx950) implementation of the hot path of geodesic-shooting
PDE-constrained LDDMM with inexact Gauss-Newton-Krylov optimisation
(M. Hernandez, arXiv 1807.04638): EPDiff shooting with semi-Lagrangian
transport, the adjoint / incremental adjoint Jacobi sweeps, the Gauss-Newton
Hessian-vector product, CG in V and the Gauss-Newton loop.

The compute lives in the HIP library ``liblddmm.so`` (C ABI in include/lddmm.h);
``lddmm.Registration`` is its ctypes binding.
"""

from .lddmm import Batch, LddmmError, Registration, load_library  # noqa: F401
