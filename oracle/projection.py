"""Galerkin projection over approximate eigenvectors (plain FP64).
Test infrastructure only.

Follows the projection box of Sec. 2.2: with the current system
``A (x - x0) = r0`` and an orthonormal ``V`` (n x k) spanning the
approximate eigenvectors, form ``H = V^T A V`` and ``c = V^T r0``, solve
``H d = c``, and take ``x = x0 + V d`` and ``r = r0 - A V d``.

``H`` is formed once per operator and reused for every cycle and every
right-hand side (Sec. 4.1, Example 2: a second right-hand side "does not need
the coarse-grid work or forming of the projection matrix").
"""
from __future__ import annotations

import numpy as np

from . import operators


def projection_matrix(op, V, transpose=False):
    """``H = V^T A V`` (``A^T`` if ``transpose``)."""
    AV = operators.apply_transpose(op, V) if transpose else operators.apply(op, V)
    return V.T @ AV


def galerkin(op, V, H, x, r, transpose=False):
    """One Galerkin projection.  Returns ``(x_new, r_new, d)``.

    ``H d = c`` is solved by LU with partial pivoting (LAPACK gesv through
    ``numpy.linalg.solve``); ``r_new`` uses one operator application on
    ``V d`` (the box's ``r0 - A V d``)."""
    c = V.T @ r
    d = np.linalg.solve(H, c)
    xh = V @ d
    Axh = operators.apply_transpose(op, xh) if transpose else operators.apply(op, xh)
    return x + xh, r - Axh, d


def minres_projection(op, V, x, r):
    """MinRes variant mentioned after the Sec. 2.2 box: ``H = (AV)^T AV``,
    ``c = (AV)^T r0``.  Not used by the solvers (the paper uses Galerkin)."""
    AV = operators.apply(op, V)
    d = np.linalg.solve(AV.T @ AV, AV.T @ r)
    return x + V @ d, r - AV @ d, d
