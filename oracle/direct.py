"""Direct solves of ``A x = b`` (plain FP64).  Test infrastructure only.

Every solve of the method ends, within its tolerance, at the plain
definition ``x = A^{-1} b`` (Sec. 1 states the problem as ``A x = b``; the
Sec. 2.2 and Sec. 4.1 boxes stop on the residual of that system).  This
module computes that result by a sparse LU factorisation of the explicit
matrix, as one library step (scipy's SuperLU with its default fill-reducing
column ordering), so that GPU solutions at full size can be compared with
it element by element.  For ``A^T`` the same factors are used with the
transposed solve.

Pinned in ``tests/test_oracle_direct.py`` against dense ``numpy.linalg.solve``
on grids with n <= 4000 and by the residual it leaves.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from . import operators


class DirectSolver:
    """LU factors of the explicit matrix of ``op``; ``solve(b)`` returns
    ``A^{-1} b`` and ``solve(b, transpose=True)`` returns ``A^{-T} b``."""

    def __init__(self, op: operators.StencilOp):
        self.op = op
        self.lu = spla.splu(operators.to_csr(op).tocsc())

    def solve(self, b, transpose=False):
        b = np.asarray(b, dtype=np.float64)
        return self.lu.solve(b, trans="T" if transpose else "N")


def solve(op, b, transpose=False):
    """``A^{-1} b`` (or ``A^{-T} b``) for one right-hand side."""
    return DirectSolver(op).solve(b, transpose)


def solution_error(x, xstar):
    """Relative error ``||x - x*|| / ||x*||`` (Euclidean norms)."""
    x = np.asarray(x, dtype=np.float64)
    xstar = np.asarray(xstar, dtype=np.float64)
    return float(np.linalg.norm(x - xstar) / np.linalg.norm(xstar))
