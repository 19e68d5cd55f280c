"""Galerkin projection over approximate eigenvectors (plain FP64).
Test infrastructure only.

Follows the projection box of Sec. 2.2: with the current system
``A (x - x0) = r0`` and an orthonormal ``V`` (n x k) spanning the
approximate eigenvectors, form ``H = V^T A V`` and ``c = V^T r0``, solve
``H d = c``, and take ``x = x0 + V d`` and ``r = r0 - A V d``.

``H`` is formed once per operator and reused for every cycle and every
right-hand side (Sec. 4.1, Example 2: a second right-hand side "does not need
the coarse-grid work or forming of the projection matrix").  The MinRes
variant the paper notes after the box (not used in its experiments) is
:func:`minres_projection`.
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


def minres_matrix(op, V, transpose=False):
    """``W = A V`` (``A^T V`` if ``transpose``) and ``H = W^T W`` of the MinRes
    projection."""
    W = operators.apply_transpose(op, V) if transpose else operators.apply(op, V)
    return W, W.T @ W


def minres_projection(op, V, x, r, transpose=False, W=None, H=None):
    """The MinRes variant noted after the Sec. 2.2 box: the box's steps with
    ``H = (AV)^T AV`` and ``c = (AV)^T r0`` in place of ``V^T A V`` and
    ``V^T r0``; the update is the box's (``x0 + V d``, ``r0 - A V d``).
    ``W``, ``H`` from :func:`minres_matrix` (computed here if not given).
    Returns ``(x_new, r_new, d)``."""
    if W is None:
        W, H = minres_matrix(op, V, transpose)
    c = W.T @ r
    d = np.linalg.solve(H, c)
    xh = V @ d
    Axh = operators.apply_transpose(op, xh) if transpose else operators.apply(op, xh)
    return x + xh, r - Axh, d


def precond_space(op, V, precond, transpose=False):
    """Right preconditioning (Sec. 5, Example 5): the Galerkin projection of
    ``A M^{-1}`` over ``V`` uses ``c = V^T r`` and ``H = V^T A Z`` with
    ``Z = M^{-1} V``, and updates ``x += Z d``, ``r -= A Z d``.  Returns
    ``(Z, H)``."""
    Z = np.stack([precond(V[:, j]) for j in range(V.shape[1])], axis=1)
    AZ = operators.apply_transpose(op, Z) if transpose else operators.apply(op, Z)
    return Z, V.T @ AZ


def precond_projection(op, V, Z, H, x, r, transpose=False):
    """One projection of the preconditioned system (see :func:`precond_space`)."""
    c = V.T @ r
    d = np.linalg.solve(H, c)
    xh = Z @ d
    Axh = operators.apply_transpose(op, xh) if transpose else operators.apply(op, xh)
    return x + xh, r - Axh, d


def projector(op, V, H, transpose=False, projection="galerkin", Z=None):
    """The projection step of the solvers as a function ``(x, r) -> (x, r, d)``:
    Galerkin with the given ``H = V^T A V``, MinRes (its ``W`` and ``H``
    formed here once), or, with ``Z = M^{-1} V``, the preconditioned one
    (``H = V^T A Z`` given)."""
    if Z is not None:
        return lambda x, r: precond_projection(op, V, Z, H, x, r, transpose)
    if projection == "minres":
        W, Hm = minres_matrix(op, V, transpose)
        return lambda x, r: minres_projection(op, V, x, r, transpose, W, Hm)
    if projection != "galerkin":
        raise ValueError(projection)
    return lambda x, r: galerkin(op, V, H, x, r, transpose=transpose)
