"""Fine-grid deflation space from moved coarse vectors (plain FP64).
Test infrastructure only.

Phase 1 of the Sec. 3 algorithm moves the coarse approximate eigenvectors to
the fine grid; the projection box of Sec. 2.2 needs an orthonormal ``V``
spanning them (step 1) and ``H = V^T A V`` (step 2).  ``V`` is the Q factor
of the thin QR of ``P W_c`` with a positive diagonal in R (the unique thin QR,
so any correct orthonormalisation with that sign convention agrees with it).
"""
from __future__ import annotations

import numpy as np

from . import transfer
from .projection import projection_matrix


def orthonormalize(W):
    """Thin QR ``W = Q R`` with ``diag(R) > 0``; returns Q."""
    Q, R = np.linalg.qr(W)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s


def deflation_space(fine_op, Wc, coarse_dims, transpose=False):
    """``V = qr(P W_c).Q`` and ``H = V^T A V``.  Returns ``(V, H)``."""
    PW = transfer.prolongate(Wc, coarse_dims)
    V = orthonormalize(PW)
    H = projection_matrix(fine_op, V, transpose=transpose)
    return V, H
