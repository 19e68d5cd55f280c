"""Pins of the oracle's direct solve (x = A^{-1} b by sparse LU), which the
full-size GPU parity tests compare against: dense numpy.linalg.solve on grids
with n <= 4000 for every operator kind, A and A^T, and the residual it leaves
on a larger grid."""
import numpy as np
import pytest

import workloads as W
from oracle import direct as D, operators as O


def _ops():
    yield O.const_cd((63, 63), (40.0, 0.0))                 # the small 2-D workload
    yield O.const_cd((15, 13, 11), (50.0, 20.0, 10.0))      # 3-D, every axis convected
    yield O.div_k((41, 37), W.kfield((41, 37), 5), (60.0, 0.0))
    yield O.example1_operator(31)


@pytest.mark.parametrize("idx", range(4))
@pytest.mark.parametrize("transpose", [False, True])
def test_direct_matches_dense_solve(idx, transpose):
    op = list(_ops())[idx]
    assert op.n <= 4000
    A = O.to_csr(op).toarray()
    b = W.rhs(op.n, 11 + idx)
    xd = np.linalg.solve(A.T if transpose else A, b)
    x = D.solve(op, b, transpose=transpose)
    assert D.solution_error(x, xd) <= 1e-12


def test_direct_residual_on_a_larger_grid():
    op = O.const_cd((255, 255), (100.0, 0.0))
    b = W.rhs(op.n, 2)
    ds = D.DirectSolver(op)
    for tr in (False, True):
        x = ds.solve(b, transpose=tr)
        r = b - (O.apply_transpose(op, x) if tr else O.apply(op, x))
        assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(b)


def test_solution_error_definition():
    assert D.solution_error([1.0, 2.0], [1.0, 2.0]) == 0.0
    assert np.isclose(D.solution_error([3.0, 4.0], [0.0, 5.0]), np.sqrt(9 + 1) / 5)
