"""Discrete Laplacians of a planar triangle mesh (Section IV).

* ``cotan_laplacian``: L^c_ij = (cot alpha_ij + cot beta_ij)/2 for each mesh
  edge ij, alpha/beta the angles opposite the edge in its (one or two)
  triangles; L^c_ii = -sum_j L^c_ij (Section IV, cotangent formula).
* ``area_laplacian``: L = A^{-1} L^c with a_i one third of the area of the
  triangles incident on vertex i (Section IV).
* ``normalized_laplacian``: L^n = Z^{-1} L^c, Z = diag(L^c) (Section IV).
* ``block_split``: the (I, B) blocks of eq. (18).

Parity pinned by: the textbook five-point stencil on right-triangle grids,
symmetry and zero row sums, and exact reproduction of linear functions
(tests/test_oracle_fem.py).
"""

import numpy as np
import scipy.sparse as sp


def _cot_at_corners(xy, tris):
    """cot of the interior angle at each corner of each triangle, [F, 3]."""
    out = np.empty(tris.shape, dtype=np.float64)
    for c in range(3):
        a = xy[tris[:, c]]
        b = xy[tris[:, (c + 1) % 3]]
        d = xy[tris[:, (c + 2) % 3]]
        u = b - a
        v = d - a
        dot = u[:, 0] * v[:, 0] + u[:, 1] * v[:, 1]
        cross = np.abs(u[:, 0] * v[:, 1] - u[:, 1] * v[:, 0])
        out[:, c] = dot / cross
    return out


def cotan_laplacian(xy, tris, n=None):
    """Symmetric sparse L^c (n x n) from vertex coordinates and triangles."""
    xy = np.asarray(xy, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    if n is None:
        n = xy.shape[0]
    cot = _cot_at_corners(xy, tris)
    rows, cols, vals = [], [], []
    for c in range(3):
        # the edge opposite corner c joins corners c+1 and c+2
        i = tris[:, (c + 1) % 3]
        j = tris[:, (c + 2) % 3]
        w = 0.5 * cot[:, c]
        rows += [i, j]
        cols += [j, i]
        vals += [w, w]
    off = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                        shape=(n, n)).tocsr()
    off.sum_duplicates()
    diag = -np.asarray(off.sum(axis=1)).ravel()
    return (off + sp.diags(diag)).tocsr()


def vertex_areas(xy, tris, n=None):
    """a_i = one third of the total area of the triangles incident on i."""
    xy = np.asarray(xy, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    if n is None:
        n = xy.shape[0]
    p0, p1, p2 = xy[tris[:, 0]], xy[tris[:, 1]], xy[tris[:, 2]]
    area = 0.5 * np.abs((p1[:, 0] - p0[:, 0]) * (p2[:, 1] - p0[:, 1])
                        - (p1[:, 1] - p0[:, 1]) * (p2[:, 0] - p0[:, 0]))
    a = np.zeros(n)
    for c in range(3):
        np.add.at(a, tris[:, c], area / 3.0)
    return a


def area_laplacian(xy, tris, n=None):
    """L = A^{-1} L^c (non-symmetric)."""
    Lc = cotan_laplacian(xy, tris, n)
    a = vertex_areas(xy, tris, Lc.shape[0])
    inv = np.where(a > 0, 1.0 / np.where(a > 0, a, 1.0), 0.0)
    return (sp.diags(inv) @ Lc).tocsr()


def normalized_laplacian(xy, tris, n=None):
    """L^n = Z^{-1} L^c with Z = diag(L^c): unit diagonal."""
    Lc = cotan_laplacian(xy, tris, n)
    z = Lc.diagonal()
    inv = np.where(z != 0, 1.0 / np.where(z != 0, z, 1.0), 0.0)
    return (sp.diags(inv) @ Lc).tocsr()


def block_split(L, interior, boundary):
    """(L_II, L_IB) of the block structure of eq. (18)."""
    L = sp.csr_matrix(L)
    LI = L[interior]
    return LI[:, interior].tocsc(), LI[:, boundary].tocsc()
