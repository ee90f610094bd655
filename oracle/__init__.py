"""FP64 CPU oracle for the divergence-distance path.

TEST INFRASTRUCTURE.  This package is a plain, slow, obviously correct
implementation of what the path computes, written from the paper (Chen,
Gotsman, Hormann, "Path Planning with Divergence-Based Distance Functions").
It is used only by ``tests/``, by ``__graft_entry__.smoke()`` and by the CPU
baseline leg of ``bench.py``; the product library never imports, links or
calls it, and it shares no code with the HIP path.

Contents (each function cites the passage it follows):

* ``fem``        cotangent Laplacian L^c, area-weighted L, normalised L^n and
                 the interior/boundary block split (Section IV, eq. 18).
* ``poisson``    discrete Poisson kernel P_IB = -L_II^{-1} L_IB (eqs. 32-33),
                 by column solves, by row solves and by a dense brute-force solve.
* ``divergence`` TV (eq. 34) and KL (eq. 35) distance fields, and the
                 truncated (sparsified) fields.
* ``path``       edge-based steepest-descent path and the spurious local-minimum
                 count (Section IV "Gradient-descent path generation", Section V
                 "Low resolution discretizations").
* ``disk``       unit-disk closed forms (Appendix eqs. A1, A6, A8, A10).
* ``green``      discrete Dirichlet Green's function D_Ip = (-L_II)^{-1} e_p
                 and the harmonic potential of eq. (23) (Section IV, eqs.
                 19-23): the comparison distance D.

Precision: FP64 throughout.  Inputs handed to the library in FP32 are upcast
to FP64 before the oracle sees them, so oracle and library read the same
numbers.
"""

from . import fem, poisson, divergence, path, disk, green

__all__ = ["fem", "poisson", "divergence", "path", "disk", "green"]
