"""The five workloads, by what they are and their sizes.

disk4096      unit disk, closed-form kernel, B=256 boundary angles, N=4096 points r<=0.95
grid257       257x257 grid, 3 rectangles with sides U[0.05,0.2]; dense FP32 and CSR at
              tau=1e-6
grid1025      1025x1025 grid, 20 rectangles with sides U[0.025,0.075]; 64 targets per launch
serving4      serving over 129/257/513/1025 grids with 2/5/10/20 rectangles
grid1025_csr  the 1025x1025 domain truncated at tau=1e-5 row-relative; 256 targets
"""

from .disk import disk_instance
from .grid import grid_domain

CONFIGS = {
    "disk4096": dict(kind="disk", N=4096, B=256, r_max=0.95, seed_id=0, targets=1),
    "grid257": dict(kind="grid", G=257, obstacles=3, sides=(0.05, 0.2), seed_id=1, targets=1,
               tau=1e-6),
    "grid1025": dict(kind="grid", G=1025, obstacles=20, sides=(0.025, 0.075), seed_id=2, targets=64),
    "serving4": dict(kind="serving", seed_id=3,
               domains=[(129, 2, (0.05, 0.2)), (257, 5, (0.05, 0.2)),
                        (513, 10, (0.05, 0.2)), (1025, 20, (0.025, 0.075))],
               qps=200.0, max_steps=4000, max_batch=64),
    "grid1025_csr": dict(kind="grid", G=1025, obstacles=20, sides=(0.025, 0.075), seed_id=2, targets=256,
               tau=1e-5),
}


def build_config(name, **override):
    """Geometry object of a disk/grid workload (the kernel matrix is built lazily)."""
    c = dict(CONFIGS[name])
    c.update(override)
    if c["kind"] == "disk":
        return disk_instance(N=c["N"], B=c["B"], r_max=c["r_max"], seed_id=c["seed_id"])
    if c["kind"] == "grid":
        return grid_domain(c["G"], c["obstacles"], c["sides"], seed_id=c["seed_id"])
    raise ValueError(f"{name} is not a single-domain workload")
