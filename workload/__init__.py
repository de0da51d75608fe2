"""Seeded synthetic SAR workloads for Online FISTA.

This package only *draws inputs*: the pixel grid, the platform trajectory, the
stepped-frequency grid, a sparse complex reflectivity scene, unit-variance
complex noise draws and per-pulse phase errors.  It holds none of the method's
arithmetic (no forward operator, no Gram, no FISTA step), so the FP64 oracle
and the GPU library can both consume its arrays without sharing any of the
computation they are compared on.
"""

from .scenes import (
    CONFIGS,
    Workload,
    WorkloadSpec,
    library_kwargs,
    make_workload,
    spec,
)

__all__ = ["CONFIGS", "Workload", "WorkloadSpec", "library_kwargs", "make_workload", "spec"]
