"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle.

This package builds the *inputs* of the divergence-distance hot path and
nothing else: domain geometry (unit-disk sample points, square grid domains
with rectangular obstacles), their triangulations and interior adjacency,
seeded target/source/arrival choices, and the discrete Poisson-kernel matrix
each workload hands to ``load_kernel``.

It holds no divergence, logarithm, path or minimum-search arithmetic.  The
Poisson kernel of the unit-disk workload is the closed form that defines that
workload; the Poisson kernel of a grid domain is the discrete harmonic measure
of the grid graph under the textbook five-point stencil.  The oracle derives
the same matrix independently from the cotangent FEM of the triangulation and a
CPU test checks the two against each other, so the shared input is pinned too.
"""

from .seeds import rng, SEED_STREAMS
from .disk import DiskInstance, disk_instance
from .grid import GridDomain, grid_domain, harmonic_measure_5pt
from .configs import CONFIGS, build_config

__all__ = [
    "rng", "SEED_STREAMS", "DiskInstance", "disk_instance", "GridDomain",
    "grid_domain", "harmonic_measure_5pt", "CONFIGS", "build_config",
]
