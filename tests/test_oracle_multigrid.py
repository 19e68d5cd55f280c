"""Pins of the oracle's multigrid preconditioner (positively shifted
Laplacian, Sec. 5 Example 5) against facts outside the recursive code: the
dense two-level formula M^{-1} = (I - E) A^{-1} on a 3 x 3 grid, convergence to
the direct solve with the textbook contraction, symmetry and linearity."""
import numpy as np
import scipy.sparse.linalg as spl

import workloads as W
from oracle import operators as O, multigrid as MG, transfer as T


def _dense(op):
    return O.to_csr(op).toarray()


def test_two_level_equals_dense_formula():
    """3 x 3 grid over a single coarse point: one V-cycle is
    (I - E) A^{-1} with E = S^nu (I - P A_c^{-1} R A) S^nu, S = I - omega D^{-1} A;
    two V-cycles are 2 M^{-1} - M^{-1} A M^{-1}."""
    op = O.const_cd((3, 3), (0.0, 0.0), sigma=50.0)
    ops = MG.levels(op)
    assert len(ops) == 2 and ops[1].dims == (1, 1)
    A = _dense(op)
    Ac = _dense(ops[1])
    n = op.n
    P = np.stack([T.prolongate(np.eye(1)[:, j], (1, 1)) for j in range(1)], axis=1)
    R = np.stack([T.restrict(np.eye(n)[:, j], (3, 3)) for j in range(n)], axis=1)
    S = np.eye(n) - (4.0 / 5.0) / op.coef["C"] * A
    for nu in (1, 2, 3):
        E = np.linalg.matrix_power(S, nu) @ (np.eye(n) - P @ np.linalg.solve(Ac, R @ A)) @ np.linalg.matrix_power(S, nu)
        Minv = (np.eye(n) - E) @ np.linalg.inv(A)
        got = np.stack([MG.mg_apply(ops, np.eye(n)[:, j], cycles=1, nu=nu) for j in range(n)], axis=1)
        np.testing.assert_allclose(got, Minv, rtol=1e-12, atol=1e-14 * np.abs(Minv).max())
        got2 = np.stack([MG.mg_apply(ops, np.eye(n)[:, j], cycles=2, nu=nu) for j in range(n)], axis=1)
        np.testing.assert_allclose(got2, 2 * Minv - Minv @ A @ Minv, rtol=1e-11, atol=1e-14 * np.abs(Minv).max())


def test_converges_to_direct_solve_with_textbook_contraction():
    for dims, sigma in (((63, 63), 400.0), ((15, 15, 15), 100.0)):
        op = O.const_cd(dims, (0.0,) * len(dims), sigma=sigma)
        ops = MG.levels(op)
        assert ops[-1].dims == (1,) * len(dims)
        v = W.rhs(op.n, 5)
        xs = spl.spsolve(O.to_csr(op).tocsc(), v)
        errs = [np.linalg.norm(MG.mg_apply(ops, v, cycles=c) - xs) for c in range(1, 13)]
        assert errs[-1] <= 1e-9 * np.linalg.norm(xs)
        # damped-Jacobi V(2,2) cycles contract the error by about 0.14 (2-D) / 0.17 (3-D)
        rates = [errs[i + 1] / errs[i] for i in range(6)]
        assert max(rates) <= 0.2


def test_symmetric_and_linear():
    op = O.const_cd((31, 31), (0.0, 0.0), sigma=900.0)
    ops = MG.levels(op)
    x, y = W.rhs(op.n, 6), W.rhs(op.n, 7)
    Mx, My = MG.mg_apply(ops, x), MG.mg_apply(ops, y)
    assert abs(x @ My - y @ Mx) <= 1e-12 * abs(x @ My)
    np.testing.assert_allclose(MG.mg_apply(ops, 2.0 * x - 3.0 * y), 2.0 * Mx - 3.0 * My, rtol=1e-11,
                               atol=1e-14 * np.abs(Mx).max())
