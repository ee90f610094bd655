"""Square grid domains with rectangular obstacles.

Geometry: the unit square on a G x G vertex grid (spacing h = 1/(G-1)); every
cell is split on its (i,j)-(i+1,j+1) diagonal into two right triangles.  Each
obstacle is an axis-aligned rectangle with corners snapped to grid vertices;
the cells it covers and the vertices strictly inside it are removed, and the
vertices on its border join the outer-square vertices as boundary vertices.
Rectangles keep at least ``gap`` cells from each other and from the outer
square, so every interior vertex keeps all six incident triangles and the
interior stays connected.

Vertex order: global id g = j*G + i; interior rows and boundary columns are
listed in increasing g.

Kernel matrix: the discrete harmonic measure of the interior under the
five-point stencil (4 u_v - sum of the four axis neighbours = 0, boundary
neighbours carrying the indicator of one boundary vertex), solved in FP64 by
sparse LU, one right-hand side per boundary vertex.
"""

import os
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .disk import edges_to_csr
from .seeds import rng


@dataclass
class GridDomain:
    G: int
    rects: list                   # [(i0, j0, i1, j1)] obstacle corners (vertex indices)
    interior: np.ndarray          # int64 [N] global ids of interior vertices
    boundary: np.ndarray          # int64 [K] global ids of boundary vertices
    triangles: np.ndarray         # int64 [F, 3] global ids, counter-clockwise
    adj_ptr: np.ndarray           # int64 [N+1] interior-only triangulation edges
    adj_idx: np.ndarray           # int32
    seed_id: int = 0
    _P: np.ndarray = field(default=None, repr=False)

    @property
    def N(self):
        return len(self.interior)

    @property
    def K(self):
        return len(self.boundary)

    @property
    def h(self):
        return 1.0 / (self.G - 1)

    def xy(self):
        """Coordinates of all G*G grid vertices (removed ones included)."""
        g = np.arange(self.G * self.G)
        return np.column_stack([(g % self.G) * self.h, (g // self.G) * self.h])

    def interior_mesh(self):
        """(faces [F, 3] interior-local ids, xy [N, 2]): the triangles whose three
        vertices are interior, and the interior vertex coordinates."""
        loc = -np.ones(self.G * self.G, dtype=np.int64)
        loc[self.interior] = np.arange(self.N)
        f = loc[self.triangles]
        return f[(f >= 0).all(axis=1)], self.xy()[self.interior]

    def node_type(self):
        """uint8 [G*G]: 0 removed (inside an obstacle), 1 interior, 2 boundary."""
        t = np.zeros(self.G * self.G, dtype=np.uint8)
        t[self.interior] = 1
        t[self.boundary] = 2
        return t

    def poisson_kernel(self, dtype=np.float64, workers=None, progress=None):
        if self._P is None or self._P.dtype != dtype:
            self._P = harmonic_measure_5pt(self, dtype=dtype, workers=workers, progress=progress)
        return self._P


def _sample_rects(G, n_obstacles, side_range, seed_id, gap):
    g = rng(seed_id, "geometry")
    h = 1.0 / (G - 1)
    rects = []
    tries = 0
    while len(rects) < n_obstacles:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not place obstacles")
        w = max(2, int(round(g.uniform(*side_range) / h)))
        ht = max(2, int(round(g.uniform(*side_range) / h)))
        hi_i = (G - 1) - gap - w
        hi_j = (G - 1) - gap - ht
        if hi_i < gap or hi_j < gap:
            continue
        i0 = int(g.integers(gap, hi_i + 1))
        j0 = int(g.integers(gap, hi_j + 1))
        r = (i0, j0, i0 + w, j0 + ht)
        ok = True
        for q in rects:
            # separated by at least `gap` cells along some axis
            if not (r[0] >= q[2] + gap or q[0] >= r[2] + gap or
                    r[1] >= q[3] + gap or q[1] >= r[3] + gap):
                ok = False
                break
        if ok:
            rects.append(r)
    return rects


def grid_domain(G, n_obstacles, side_range=(0.05, 0.2), seed_id=0, gap=2) -> GridDomain:
    rects = _sample_rects(G, n_obstacles, side_range, seed_id, gap)
    I, J = np.meshgrid(np.arange(G), np.arange(G), indexing="xy")  # I[j,i] = i
    removed = np.zeros((G, G), dtype=bool)       # indexed [j, i]
    bnd = np.zeros((G, G), dtype=bool)
    bnd[0, :] = bnd[-1, :] = bnd[:, 0] = bnd[:, -1] = True
    cell_removed = np.zeros((G - 1, G - 1), dtype=bool)
    for (i0, j0, i1, j1) in rects:
        removed[j0 + 1:j1, i0 + 1:i1] = True
        bnd[j0:j1 + 1, i0:i1 + 1] = True
        cell_removed[j0:j1, i0:i1] = True
    bnd &= ~removed
    inter = ~removed & ~bnd
    gid = (J * G + I)
    interior = np.sort(gid[inter].ravel()).astype(np.int64)
    boundary = np.sort(gid[bnd].ravel()).astype(np.int64)

    cj, ci = np.nonzero(~cell_removed)
    g00 = cj * G + ci
    g10 = g00 + 1
    g11 = g00 + G + 1
    g01 = g00 + G
    triangles = np.concatenate([np.column_stack([g00, g10, g11]),
                                np.column_stack([g00, g11, g01])]).astype(np.int64)

    # interior-only adjacency = triangulation edges between interior vertices
    loc = -np.ones(G * G, dtype=np.int64)
    loc[interior] = np.arange(len(interior))
    ii = interior % G
    jj = interior // G
    edges = []
    for di, dj in ((1, 0), (0, 1), (1, 1)):
        ni, nj = ii + di, jj + dj
        ok = (ni < G) & (nj < G)
        nb = np.where(ok, nj * G + ni, 0)
        ok &= loc[nb] >= 0
        edges.append(np.column_stack([loc[interior[ok]], loc[nb[ok]]]))
    ptr, idx = edges_to_csr(len(interior), np.concatenate(edges))

    dom = GridDomain(G=G, rects=rects, interior=interior, boundary=boundary,
                     triangles=triangles, adj_ptr=ptr, adj_idx=idx, seed_id=seed_id)
    _check_connected(dom)
    return dom


def _check_connected(dom):
    n = dom.N
    seen = np.zeros(n, dtype=bool)
    seen[0] = True
    frontier = np.array([0])
    while len(frontier):
        nb = np.concatenate([dom.adj_idx[dom.adj_ptr[v]:dom.adj_ptr[v + 1]] for v in frontier])
        nb = np.unique(nb)
        nb = nb[~seen[nb]]
        seen[nb] = True
        frontier = nb
    if not seen.all():
        raise RuntimeError("interior of the grid domain is not connected")


def _five_point_system(dom):
    """Sparse A (interior x interior) and R (interior x boundary) of the stencil."""
    G = dom.G
    n, k = dom.N, dom.K
    iloc = -np.ones(G * G, dtype=np.int64)
    iloc[dom.interior] = np.arange(n)
    bloc = -np.ones(G * G, dtype=np.int64)
    bloc[dom.boundary] = np.arange(k)
    rows_a, cols_a, vals_a = [np.arange(n)], [np.arange(n)], [np.full(n, 4.0)]
    rows_r, cols_r = [], []
    for off in (1, -1, G, -G):
        nb = dom.interior + off          # axis neighbours always exist for interior vertices
        a = iloc[nb] >= 0
        rows_a.append(np.nonzero(a)[0]); cols_a.append(iloc[nb[a]]); vals_a.append(np.full(a.sum(), -1.0))
        b = bloc[nb] >= 0
        rows_r.append(np.nonzero(b)[0]); cols_r.append(bloc[nb[b]])
    A = sp.csc_matrix((np.concatenate(vals_a), (np.concatenate(rows_a), np.concatenate(cols_a))),
                      shape=(n, n))
    rr, cc = np.concatenate(rows_r), np.concatenate(cols_r)
    R = sp.csc_matrix((np.ones(len(rr)), (rr, cc)), shape=(n, k))
    return A, R


_WORK = {}


def _solve_chunk(args):
    lo, hi = args
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)
    lu, R, out_name, shape, dtype = _WORK["lu"], _WORK["R"], _WORK["name"], _WORK["shape"], _WORK["dtype"]
    if lu is None:
        lu = _WORK["lu"] = spla.splu(_WORK["A"])
    X = lu.solve(R[:, lo:hi].toarray())
    np.maximum(X, 0.0, out=X)   # the exact solution is >= 0; clear round-off below zero
    out = np.memmap(out_name, dtype=dtype, mode="r+", shape=shape)
    out[:, lo:hi] = X.astype(dtype)
    out.flush()
    del out
    return hi - lo


def gpu_initialised():
    """True when this process may hold a GPU context: torch's device runtime is
    initialised, or the HIP library has been loaded.  Forking such a process
    is unsafe."""
    import sys
    torch = sys.modules.get("torch")
    if torch is not None and torch.cuda.is_initialized():
        return True
    lib = sys.modules.get("paper_1708_02845_amd._lib")
    return bool(lib is not None and getattr(lib, "_lib", None) is not None)


def harmonic_measure_5pt(dom, dtype=np.float64, workers=None, chunk=128, progress=None,
                         out_path=None):
    """Dense [N, K] matrix: row v = harmonic measure of interior vertex v.

    With several workers the columns are solved in forked processes into a
    shared memory-mapped file, which is returned mapped (no final copy); a
    process that already holds a GPU context does not fork and solves in
    process instead.  ``out_path``: write the matrix to this raw file (row-major,
    kept after return) and return it mapped.  ``progress(done_columns, K)`` is
    called as chunks finish.
    """
    A, R = _five_point_system(dom)
    n, k = dom.N, dom.K
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    if workers > 1 and gpu_initialised():
        workers = 1
    work = [(lo, min(k, lo + chunk)) for lo in range(0, k, chunk)]
    if workers <= 1 or len(work) <= 1 or n * k < 2_000_000:
        lu = spla.splu(A)
        P = (np.empty((n, k), dtype=dtype) if out_path is None else
             np.memmap(out_path, dtype=dtype, mode="w+", shape=(n, k)))
        for lo, hi in work:
            X = lu.solve(R[:, lo:hi].toarray())
            np.maximum(X, 0.0, out=X)
            P[:, lo:hi] = X
            if progress:
                progress(hi, k)
        return P
    import multiprocessing as mp
    import tempfile
    if out_path is None:
        d = "/dev/shm" if os.path.isdir("/dev/shm") else None
        fd, name = tempfile.mkstemp(prefix="hm5pt_", dir=d)
        os.close(fd)
    else:
        name = out_path
    assert not gpu_initialised()
    try:
        out = np.memmap(name, dtype=dtype, mode="w+", shape=(n, k))
        del out
        _WORK.update(A=A, R=R, lu=None, name=name, shape=(n, k), dtype=dtype)
        done = 0
        with mp.get_context("fork").Pool(workers) as pool:
            for m in pool.imap_unordered(_solve_chunk, work):
                done += m
                if progress:
                    progress(done, k)
        P = np.memmap(name, dtype=dtype, mode="r+", shape=(n, k))
    finally:
        _WORK.clear()
        if out_path is None:
            os.unlink(name)      # the mapping stays valid until P is released
    return P
