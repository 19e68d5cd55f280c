"""Geometric multigrid for a constant-coefficient operator, used as the
preconditioner of Sec. 5, Example 5: solutions with the positively shifted
Laplacian ``-Lap(u) + kappa^2 u`` precondition the Helmholtz operator
``-Lap(u) - kappa^2 u`` on both grids.  Test infrastructure only.

The paper does not describe its multigrid; the reading used here (the same on
the GPU) is a textbook V-cycle:

* levels: the operator's grid and its nested coarse grids (``n -> (n-1)/2``
  per axis, the same PDE rediscretised, ``operators.coarsen``) while every
  side is odd and at least 3;
* smoother: damped Jacobi with the constant diagonal ``d``,
  ``z <- z + omega (v - A z) / d``, ``omega = 4/5`` (2-D) or ``6/7`` (3-D),
  ``nu`` sweeps before and ``nu`` after the coarse correction; the first
  sweep from ``z = 0`` is ``z = omega v / d``;
* residual restricted by full weighting, correction prolongated bilinearly
  (trilinearly) and added (``transfer.py``);
* coarsest grid: 20 damped-Jacobi sweeps from zero (a single point for the
  2^L - 1 grids of the workloads, where they are exact to rounding);
* the preconditioner is ``cycles`` V-cycles from a zero initial guess,
  ``z_1 = V(v)``, ``z_{c+1} = z_c + V(v - A z_c)``: a fixed linear operator,
  so Krylov methods can use it as ``M^{-1}``.
"""
from __future__ import annotations

import numpy as np

from . import operators, transfer

COARSEST_SWEEPS = 20


def levels(op):
    """The operator and its rediscretised coarse operators."""
    assert op.kind == "const", "multigrid needs constant coefficients"
    ops = [op]
    while all(d % 2 == 1 and d >= 3 for d in ops[-1].dims):
        ops.append(operators.coarsen(ops[-1]))
    return ops


def _omega(op):
    return 4.0 / 5.0 if op.dim == 2 else 6.0 / 7.0


def _sweeps(op, v, z, count):
    d = op.coef["C"]
    w = _omega(op)
    for _ in range(count):
        if z is None:
            z = (w / d) * v
        else:
            z = z + (w / d) * (v - operators.apply(op, z))
    return z


def vcycle(ops, v, nu=2, level=0):
    """One V-cycle for ``A_level z = v`` from ``z = 0``."""
    op = ops[level]
    if level == len(ops) - 1:
        return _sweeps(op, v, None, COARSEST_SWEEPS)
    z = _sweeps(op, v, None, nu)
    r = v - operators.apply(op, z)
    zc = vcycle(ops, transfer.restrict(r, op.dims), nu, level + 1)
    z = z + transfer.prolongate(zc, ops[level + 1].dims)
    return _sweeps(op, v, z, nu)


def mg_apply(ops, v, cycles=2, nu=2):
    """``M^{-1} v``: ``cycles`` V-cycles from zero on the finest level."""
    v = np.asarray(v, dtype=np.float64)
    z = vcycle(ops, v, nu)
    for _ in range(cycles - 1):
        z = z + vcycle(ops, v - operators.apply(ops[0], z), nu)
    return z


__all__ = ["levels", "vcycle", "mg_apply", "COARSEST_SWEEPS"]
