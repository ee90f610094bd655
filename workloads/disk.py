"""Unit-disk workload: closed-form Poisson kernel sampled at B boundary angles.

Points are uniform by area in the disk of radius ``r_max``; boundary samples
sit at angles 2*pi*b/B.  Row x of the kernel matrix is the disk Poisson kernel
(Section III, eq. 15) evaluated at the B boundary samples and scaled to sum 1
(the sampled harmonic measure), kept in FP64.  The path graph is the Delaunay
triangulation of the sample points.
"""

from dataclasses import dataclass

import numpy as np
from scipy.spatial import Delaunay

from .seeds import rng


@dataclass
class DiskInstance:
    z: np.ndarray          # complex128 [N] sample points
    theta: np.ndarray      # float64 [B] boundary angles
    P: np.ndarray          # float64 [N, B] row-normalised Poisson kernel
    adj_ptr: np.ndarray    # int64 [N+1] Delaunay adjacency (CSR, sorted)
    adj_idx: np.ndarray    # int32 [nnz]
    triangles: np.ndarray  # int64 [F, 3]

    def interior_mesh(self):
        """(faces [F, 3], xy [N, 2]) of the Delaunay triangulation of the points."""
        return self.triangles, np.column_stack([self.z.real, self.z.imag])

    @property
    def N(self):
        return self.P.shape[0]

    @property
    def B(self):
        return self.P.shape[1]


def edges_to_csr(n, edges):
    """Symmetric CSR (sorted neighbour lists) from an undirected edge list."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    e = np.concatenate([e, e[:, ::-1]])
    e = np.unique(e, axis=0)                      # sorted by (row, col)
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(ptr, e[:, 0] + 1, 1)
    ptr = np.cumsum(ptr)
    return ptr, e[:, 1].astype(np.int32)


def disk_instance(N=4096, B=256, r_max=0.95, seed_id=0) -> DiskInstance:
    g = rng(seed_id, "geometry")
    u = g.random(N)
    v = g.random(N)
    z = r_max * np.sqrt(u) * np.exp(2j * np.pi * v)
    theta = 2.0 * np.pi * np.arange(B) / B
    s = np.exp(1j * theta)
    raw = (1.0 - np.abs(z) ** 2)[:, None] / np.abs(z[:, None] - s[None, :]) ** 2
    P = raw / raw.sum(axis=1, keepdims=True)
    tri = Delaunay(np.column_stack([z.real, z.imag])).simplices.astype(np.int64)
    edges = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    ptr, idx = edges_to_csr(N, edges)
    return DiskInstance(z=z, theta=theta, P=P, adj_ptr=ptr, adj_idx=idx, triangles=tri)
