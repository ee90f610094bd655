"""Pins for the oracle's Laplacians and Poisson kernel (Section IV, eqs. 18, 32-33)."""

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.spatial import Delaunay

from conftest import frac, read_golden
from oracle import fem, poisson
from workloads import grid_domain


def disk_mesh(n_interior=300, n_boundary=64, seed=0):
    """Delaunay mesh of random points in the unit disk plus points on its circle."""
    g = np.random.default_rng(seed)
    r = 0.9 * np.sqrt(g.random(n_interior))
    a = 2 * np.pi * g.random(n_interior)
    th = 2 * np.pi * np.arange(n_boundary) / n_boundary
    z = np.concatenate([r * np.exp(1j * a), np.exp(1j * th)])
    xy = np.column_stack([z.real, z.imag])
    tris = Delaunay(xy).simplices.astype(np.int64)
    interior = np.arange(n_interior)
    boundary = np.arange(n_interior, n_interior + n_boundary)
    return xy, tris, interior, boundary


@pytest.fixture(scope="module")
def small_grid():
    return grid_domain(33, 2, (0.1, 0.3), seed_id=7)


def test_cotan_weights_on_right_triangle_grid_are_five_point(small_grid):
    # Textbook special case: on a right-triangle grid the cot weights are 1 on
    # axis edges shared by two triangles, 1/2 on axis edges with one triangle,
    # and 0 on the diagonals (cot of the right angle).
    g = small_grid
    L = fem.cotan_laplacian(g.xy(), g.triangles).tocoo()
    G = g.G
    off = L.row != L.col
    r, c, v = L.row[off], L.col[off], L.data[off]
    diff = np.abs(c - r)
    diag_edge = diff == G + 1
    assert np.all(np.abs(v[diag_edge]) < 1e-14)
    axis = ~diag_edge
    assert np.all(np.isin(np.round(v[axis], 12), [0.5, 1.0]))
    # every interior row is exactly the five-point stencil
    Ld = sp.csr_matrix(L)
    for x in g.interior[::37]:
        row = Ld.getrow(x)
        nz = {int(k): val for k, val in zip(row.indices, row.data) if abs(val) > 1e-14}
        assert nz == pytest.approx({x - 1: 1.0, x + 1: 1.0, x - G: 1.0, x + G: 1.0, x: -4.0})


def test_cotan_symmetric_zero_row_sums():
    xy, tris, _, _ = disk_mesh()
    L = fem.cotan_laplacian(xy, tris)
    assert abs(L - L.T).max() < 1e-13
    assert np.abs(np.asarray(L.sum(axis=1))).max() < 1e-12


def test_cotan_annihilates_linear_functions_at_interior_vertices():
    # Linear precision of the cotangent Laplacian on any planar triangulation.
    xy, tris, interior, _ = disk_mesh(seed=3)
    L = fem.cotan_laplacian(xy, tris)
    for f in (xy[:, 0], xy[:, 1], 2.0 * xy[:, 0] - 3.0 * xy[:, 1] + 0.5):
        assert np.abs((L @ f)[interior]).max() < 1e-11


@pytest.mark.parametrize("mesh", ["grid", "disk"])
def test_poisson_kernel_rows_are_probability_vectors(mesh, small_grid):
    if mesh == "grid":
        g = small_grid
        xy, tris, I, B = g.xy(), g.triangles, g.interior, g.boundary
    else:
        xy, tris, I, B = disk_mesh(seed=1)
    P = poisson.poisson_kernel(fem.cotan_laplacian(xy, tris), I, B)
    assert np.abs(P.sum(axis=1) - 1.0).max() < 1e-12     # unit-sum rows (eq. 13)
    assert P.min() > -1e-15                              # non-negative


@pytest.mark.parametrize("mesh", ["grid", "disk"])
def test_poisson_kernel_reproduces_linear_boundary_data(mesh, small_grid):
    # The harmonic extension of linear boundary data is that linear function,
    # because L^c annihilates linear functions at interior vertices.
    if mesh == "grid":
        g = small_grid
        xy, tris, I, B = g.xy(), g.triangles, g.interior, g.boundary
    else:
        xy, tris, I, B = disk_mesh(seed=2)
    P = poisson.poisson_kernel(fem.cotan_laplacian(xy, tris), I, B)
    for f in (xy[:, 0], xy[:, 1], 0.3 - xy[:, 0] + 4.0 * xy[:, 1]):
        assert np.abs(P @ f[B] - f[I]).max() < 1e-11


def test_poisson_kernel_same_from_all_three_laplacians(small_grid):
    g = small_grid
    xy, tris, I, B = g.xy(), g.triangles, g.interior, g.boundary
    Pc = poisson.poisson_kernel(fem.cotan_laplacian(xy, tris), I, B)
    Pa = poisson.poisson_kernel(fem.area_laplacian(xy, tris), I, B)
    Pn = poisson.poisson_kernel(fem.normalized_laplacian(xy, tris), I, B)
    assert np.abs(Pa - Pc).max() < 1e-13
    assert np.abs(Pn - Pc).max() < 1e-13


def test_poisson_kernel_row_and_column_solves_agree_with_dense(small_grid):
    g = small_grid
    xy, tris, I, B = g.xy(), g.triangles, g.interior, g.boundary
    Lc = fem.cotan_laplacian(xy, tris)
    P = poisson.poisson_kernel(Lc, I, B)
    rows = [0, 17, len(I) // 2, len(I) - 1]
    assert np.abs(poisson.poisson_kernel_rows(Lc, I, B, rows) - P[rows]).max() < 1e-14
    assert np.abs(poisson.poisson_kernel_dense(Lc, I, B) - P).max() < 1e-13


def test_poisson_kernel_hand_solved_two_vertex_grid():
    rows = {r[0]: r[1:] for r in read_golden("grid4x3_two_vertex.txt")}
    G = 4
    i, j = np.meshgrid(np.arange(G), np.arange(3), indexing="xy")
    xy = np.column_stack([i.ravel(), j.ravel()]).astype(float)
    tris = []
    for cj in range(2):
        for ci in range(3):
            g00 = cj * G + ci
            tris += [(g00, g00 + 1, g00 + G + 1), (g00, g00 + G + 1, g00 + G)]
    interior = np.array([5, 6])
    boundary = np.array([0, 1, 2, 3, 4, 7, 8, 9, 10, 11])
    P = poisson.poisson_kernel(fem.cotan_laplacian(xy, np.array(tris)), interior, boundary)
    expect = np.array([[frac(v) for v in rows["a"]], [frac(v) for v in rows["b"]]])
    assert np.abs(P - expect).max() < 1e-15


def test_workload_kernel_matches_fem_kernel(small_grid):
    # The workload's five-point harmonic measure equals the oracle's FEM kernel.
    g = small_grid
    P_fem = poisson.poisson_kernel(fem.cotan_laplacian(g.xy(), g.triangles), g.interior, g.boundary)
    assert np.abs(g.poisson_kernel() - P_fem).max() < 1e-13


def test_grid_outer_corners_are_the_only_zero_columns(small_grid):
    g = small_grid
    P = g.poisson_kernel()
    zero = np.nonzero(P.max(axis=0) == 0)[0]
    G = g.G
    assert set(g.boundary[zero].tolist()) == {0, G - 1, G * (G - 1), G * G - 1}


def test_poisson_kernel_of_square_matches_sine_series():
    # Closed form of the discrete problem on the plain (G x G) square: with
    # M = G - 1 and boundary vertex (m, 0) on the bottom edge, separation of
    # variables in the five-point equations gives
    #   u(i, j) = sum_k c_k sin(k pi i / M) sinh(mu_k (M - j)) / sinh(mu_k M),
    #   cosh mu_k = 2 - cos(k pi / M),  c_k = (2 / M) sin(k pi m / M),
    # the discrete sine series of the boundary indicator.  Pins the oracle's
    # stencil, boundary coupling and solve against an independent formula.
    G = 17
    M = G - 1
    g = grid_domain(G, 0, seed_id=0)
    P = poisson.poisson_kernel(fem.cotan_laplacian(g.xy(), g.triangles), g.interior, g.boundary)
    col = {int(b): c for c, b in enumerate(g.boundary)}
    ii = g.interior % G
    jj = g.interior // G
    k = np.arange(1, M)
    mu = np.arccosh(2.0 - np.cos(k * np.pi / M))
    for m in (1, 5, 8, 15):
        ck = (2.0 / M) * np.sin(k * np.pi * m / M)
        u = (ck[None, :] * np.sin(np.outer(ii, k) * np.pi / M) *
             np.sinh(np.outer(M - jj, mu)) / np.sinh(mu * M)[None, :]).sum(axis=1)
        assert np.abs(P[:, col[m]] - u).max() < 1e-13, m
