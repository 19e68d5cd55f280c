"""Gradients of a least-squares loss through the solve (plain FP64).
Test infrastructure only.

This is an extension of the method (the paper has no adjoint).  For
``A(k) u = b`` with ``A(k)`` the divergence-form operator of
``operators.div_k`` and ``L = 1/2 ||u - u*||^2``:

* ``lambda = A^{-T} (u - u*)`` (the adjoint solve; the paper's deflated
  BiCGStab applied to ``A^T`` with left eigenvectors, i.e. eigenvectors of
  ``A_c^T`` from GMRES-DR on the coarse transpose);
* ``dL/db = lambda``;
* ``dL/dk_c = -lambda^T (dA/dk_c) u``.  Each grid edge ``e = (p, q)``
  contributes ``(k_e / h^2)(u_p - u_q)`` to row p and the opposite to row q,
  and ``k_e`` is the mean of the two cells that share the edge, so
  ``dL/dk_c = -sum over the four sides e of cell c of
  (1/2) h^-2 (lambda_p - lambda_q)(u_p - u_q)``, with ``u = lambda = 0`` on
  boundary nodes.  The convection term does not depend on ``k``.
"""
from __future__ import annotations

import numpy as np


def grad_k(lam, u, dims):
    """``dL/dk`` per cell, shape ``(n_y + 1, n_x + 1)``, for a 2-D grid with
    square cells of side ``h_x`` by ``h_y``.

    A horizontal side (along x) carries the x-flux coefficient ``1/h_x^2``;
    a vertical side the y-flux ``1/h_y^2``."""
    nx, ny = dims
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    # node values including the zero boundary ring: shape (ny + 2, nx + 2)
    L = np.zeros((ny + 2, nx + 2))
    U = np.zeros((ny + 2, nx + 2))
    L[1:-1, 1:-1] = np.asarray(lam).reshape(ny, nx)
    U[1:-1, 1:-1] = np.asarray(u).reshape(ny, nx)
    # x-edges: between node (j, i) and (j, i+1), for node rows j = 0..ny+1
    ex = (L[:, 1:] - L[:, :-1]) * (U[:, 1:] - U[:, :-1]) / (hx * hx)   # (ny+2, nx+1)
    # y-edges: between node (j, i) and (j+1, i)
    ey = (L[1:, :] - L[:-1, :]) * (U[1:, :] - U[:-1, :]) / (hy * hy)   # (ny+1, nx+2)
    # cell (cj, ci) has x-sides on node rows cj and cj+1, y-sides on node columns ci and ci+1
    g = ex[:-1, :] + ex[1:, :] + ey[:, :-1] + ey[:, 1:]
    return -0.5 * g


def loss(u, ustar):
    d = np.asarray(u) - np.asarray(ustar)
    return 0.5 * float(d @ d)
