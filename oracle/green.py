"""Discrete Dirichlet Green's function (Section IV, "The Dirichlet Green's
function", eqs. 19-23) -- the comparison distance D of Tables I-II.

With the cotangent Laplacian L^c (positive off-diagonal weights, L_ii = -sum),
-L^c_II is symmetric positive definite.  The Green's function with pole at the
interior vertex p is the column

    D_Ip = (-L^c_II)^{-1} e_p,

harmonic at every interior vertex but p, zero on the boundary, positive, with
its maximum at p; the potential followed downhill towards p is -D (Section
II: the potential is the negative of the Green's function).  The sign is the
reading that makes D positive as in the continuous case; eq. (20) writes
D_II = L_II^{-1} with the Laplacian's sign left implicit.

Functions:

* ``green_columns``   D_Ip for a list of poles, one sparse LU of -L_II, one
                      solve per pole (the paper's pre-factorise-then-back-
                      substitute scheme);
* ``harmonic_potential``  Q_Jp of eq. (23) by its own solve on J = I \\ {p}:
                      the Laplace equation with Q_p = 1 and Q_B = 0;
* ``grid_green_closed_form``  the textbook eigen-expansion of the five-point
                      Green's function on a plain M x M interior grid.

Pinned by (tests/test_oracle_green.py): D_Jp = D_pp Q_Jp (eq. 22 against
eq. 23, two different solves), the closed form on the plain square, symmetry
D_pq = D_qp, and the discrete maximum principle (D > 0 inside, largest at p).
"""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import block_split


def green_columns(Lc, interior, boundary, poles):
    """FP64 [len(poles), m]: row i is D_Ip for p = poles[i] (interior-local ids)."""
    LII, _ = block_split(Lc, interior, boundary)
    lu = spla.splu((-LII).tocsc())
    m = LII.shape[0]
    poles = np.asarray(poles, dtype=np.int64)
    E = np.zeros((m, len(poles)))
    E[poles, np.arange(len(poles))] = 1.0
    return lu.solve(E).T


def harmonic_potential(Lc, interior, boundary, p):
    """Q on the interior vertices (interior-local ids): Q_p = 1, Q = 0 on the
    boundary, and L^c Q = 0 at every interior vertex but p (eq. 23)."""
    LII, _ = block_split(Lc, interior, boundary)
    LII = sp.csr_matrix(LII)
    m = LII.shape[0]
    J = np.setdiff1d(np.arange(m), [p])
    LJJ = LII[J][:, J].tocsc()
    LJp = LII[J][:, [p]].toarray().ravel()
    Q = np.empty(m)
    Q[p] = 1.0
    Q[J] = spla.spsolve(LJJ, -LJp)
    return Q


def grid_green_closed_form(M, i, j):
    """Five-point Green's function of the M x M interior grid of the plain
    square (boundary all around), pole at interior grid position (i, j)
    (0-based), as an [M, M] array indexed [row j', column i']:

        D(x, p) = sum_{k,l} phi_kl(x) phi_kl(p) / lambda_kl,
        phi_kl(a, b) = (2 / (M + 1)) sin(k pi (a+1) / (M+1)) sin(l pi (b+1) / (M+1)),
        lambda_kl = 4 - 2 cos(k pi / (M+1)) - 2 cos(l pi / (M+1)),

    the eigen-expansion of (-L)^{-1} for the discrete sine eigenvectors."""
    k = np.arange(1, M + 1)
    s = np.sin(np.outer(np.arange(1, M + 1), k) * np.pi / (M + 1))   # [position, mode]
    lam = 4.0 - 2.0 * np.cos(k * np.pi / (M + 1))[:, None] - 2.0 * np.cos(k * np.pi / (M + 1))[None, :]
    c = (2.0 / (M + 1)) ** 2
    # coefficient of mode (k, l): phi_kl(p) / lambda_kl, with k along i and l along j
    coef = c * np.outer(s[i], s[j]) / lam             # [k, l]
    return (s @ coef @ s.T).T                          # [i', j'] -> [j', i']
