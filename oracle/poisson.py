"""Discrete Poisson kernel (Section IV "The divergence distances", eqs. 32-33).

Every column b of P_IB is the discrete harmonic function on the interior whose
boundary values are the indicator of boundary vertex b:

    L_II P_IB + L_IB I = 0   =>   P_IB = -L_II^{-1} L_IB.

The full P of eq. (33) stacks the identity below P_IB for the boundary rows;
the path works on interior rows only, so these functions return P_IB.

Three independent evaluations:

* ``poisson_kernel``       column solves with a sparse LU of L_II (the paper's
                           pre-factorise-then-back-substitute scheme, Section IV).
* ``poisson_kernel_rows``  row solves: for symmetric L^c, row x of P_IB is
                           (L_II^{-1} e_x)^T (-L_IB).
* ``poisson_kernel_dense`` dense ``numpy.linalg.solve`` for tiny meshes.

Parity pinned by: unit row sums (eq. 13 and its discrete statement), P >= 0,
identical P from L, L^c and L^n (Section IV), exact reproduction of linear
boundary data, a hand-solved two-vertex grid (tests/golden), and agreement of
the three evaluations.
"""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import block_split


def poisson_kernel(L, interior, boundary, chunk=256):
    """Dense FP64 [m, k] = -L_II^{-1} L_IB by sparse LU and column solves."""
    LII, LIB = block_split(L, interior, boundary)
    lu = spla.splu(LII.tocsc())
    m, k = LIB.shape
    P = np.empty((m, k))
    for lo in range(0, k, chunk):
        hi = min(k, lo + chunk)
        P[:, lo:hi] = -lu.solve(LIB[:, lo:hi].toarray())
    return P


class RowSolver:
    """Rows of P_IB by row solves, with one sparse LU of L_II for many calls;
    requires the symmetric L^c.  Row x is (L_II^{-1} e_x)^T (-L_IB)."""

    def __init__(self, Lc, interior, boundary):
        LII, LIB = block_split(Lc, interior, boundary)
        self.m = LII.shape[0]
        self.lu = spla.splu(LII.tocsc())
        self.LIBt = sp.csr_matrix(LIB).T.tocsr()

    def rows(self, rows):
        rows = np.asarray(rows, dtype=np.int64)
        E = np.zeros((self.m, len(rows)))
        E[rows, np.arange(len(rows))] = 1.0
        Y = self.lu.solve(E)                          # columns of L_II^{-1}
        return -(self.LIBt @ Y).T                     # y^T L_IB with sign of eq. (33)


def poisson_kernel_rows(Lc, interior, boundary, rows):
    """Selected rows of P_IB by row solves; requires the symmetric L^c."""
    return RowSolver(Lc, interior, boundary).rows(rows)


def poisson_kernel_dense(L, interior, boundary):
    """Brute force with a dense solve (tiny meshes only)."""
    L = sp.csr_matrix(L).toarray()
    LII = L[np.ix_(interior, interior)]
    LIB = L[np.ix_(interior, boundary)]
    return -np.linalg.solve(LII, LIB)
