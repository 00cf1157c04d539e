"""Seeded synthetic inputs shared by the GPU path's tests/benchmarks and the CPU oracle.

This package holds no arithmetic of the registration method itself: it only draws
template phantoms, band-limited random velocity fields and noise with NumPy's
``default_rng``.  Targets (template warped by shooting) are formed by the caller
with whichever implementation it is exercising.
"""

from .phantoms import (  # noqa: F401
    WorkloadSpec,
    WORKLOADS,
    phantom,
    random_velocity,
    noise,
    random_field,
)
