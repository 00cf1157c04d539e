"""FP64 CPU oracle for geodesic-shooting PDE-constrained LDDMM (EPDiff constraint,
semi-Lagrangian state transport, adjoint / incremental adjoint Jacobi sweeps,
Gauss-Newton-Krylov optimisation), and in ``oracle.pde_lddmm`` the comparison
method of the paper's Section 2.3 (PDE-LDDMM with stationary or non-stationary
velocities: transport state, continuity-equation adjoint, Gauss-Newton-Krylov).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or load
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library and imports nothing from ``paper_1807_04638_amd``.
"""

from .lddmm_oracle import *  # noqa: F401,F403
from . import pde_lddmm  # noqa: F401
