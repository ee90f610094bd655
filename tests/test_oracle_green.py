"""Pins for the oracle's discrete Dirichlet Green's function (Section IV,
eqs. 19-23), the comparison distance D."""

import numpy as np
import pytest

from oracle import fem, green
from workloads import grid_domain


@pytest.fixture(scope="module")
def obstacle_grid():
    g = grid_domain(33, 2, (0.1, 0.3), seed_id=7)
    return g, fem.cotan_laplacian(g.xy(), g.triangles, n=g.G * g.G)


def test_green_function_of_square_matches_eigen_expansion():
    # On the plain square the five-point Green's function has the textbook
    # expansion over the discrete sine eigenvectors (an independent formula:
    # no solve).  Interior vertex (i, j) of the G x G grid is position
    # (i - 1, j - 1) of the M x M interior grid, M = G - 2.
    G = 19
    M = G - 2
    g = grid_domain(G, 0, seed_id=0)
    Lc = fem.cotan_laplacian(g.xy(), g.triangles, n=G * G)
    loc = {int(v): n for n, v in enumerate(g.interior)}
    ii, jj = g.interior % G, g.interior // G
    for (pi, pj) in [(1, 1), (5, 9), (9, 9), (17, 3)]:
        p = loc[pj * G + pi]
        D = green.green_columns(Lc, g.interior, g.boundary, [p])[0]
        ref = green.grid_green_closed_form(M, pi - 1, pj - 1)[jj - 1, ii - 1]
        assert np.abs(D - ref).max() < 1e-13 * np.abs(ref).max(), (pi, pj)


def test_green_column_is_the_scaled_harmonic_potential(obstacle_grid):
    # eq. (22) against eq. (23): D_Jp = D_pp Q_Jp, with Q from its own solve on
    # J = I minus p (boundary values Q_p = 1, Q_B = 0)
    g, Lc = obstacle_grid
    for p in (0, 123, g.N // 2, g.N - 1):
        D = green.green_columns(Lc, g.interior, g.boundary, [p])[0]
        Q = green.harmonic_potential(Lc, g.interior, g.boundary, p)
        assert Q[p] == 1.0
        assert np.abs(D - D[p] * Q).max() < 1e-12 * D[p], p


def test_green_function_is_symmetric_positive_with_its_maximum_at_the_pole(obstacle_grid):
    g, Lc = obstacle_grid
    poles = [3, 200, 511, g.N - 7]
    D = green.green_columns(Lc, g.interior, g.boundary, poles)
    for a, p in enumerate(poles):
        assert (D[a] > 0).all()
        assert int(np.argmax(D[a])) == p
        for b, q in enumerate(poles):
            assert abs(D[a, q] - D[b, p]) <= 1e-13 * max(D[a, q], D[b, p])


def test_green_function_residual(obstacle_grid):
    # -L_II D_Ip = e_p, row by row
    g, Lc = obstacle_grid
    LII, _ = fem.block_split(Lc, g.interior, g.boundary)
    p = 321
    D = green.green_columns(Lc, g.interior, g.boundary, [p])[0]
    r = -(LII @ D)
    e = np.zeros(g.N)
    e[p] = 1.0
    assert np.abs(r - e).max() < 1e-12
