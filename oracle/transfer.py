"""Coarse <-> fine grid transfer (plain FP64).  Test infrastructure only.

The method moves the coarse-grid solution and approximate eigenvectors to the
fine grid "with spline interpolation or prolongation" (Sec. 3, text before
the Two-grid Deflated GMRES box, and its step 1).  The spline type is not
given; the reading used here is the linear spline: bilinear (2-D) /
trilinear (3-D) interpolation on nested grids with ``h_c = 2 h_f``.

Nested grids: per axis ``n_f = 2 n_c + 1``; coarse node ``I`` (1-based)
coincides with fine node ``2I``.  One-dimensional prolongation: a fine node
on a coarse node copies it (weight 1); a fine node between two coarse nodes
takes half of each (weight 1/2); coarse nodes 0 and ``n_c + 1`` are boundary
nodes with value zero.  In 2-D/3-D the operator is the tensor product.

Evaluation order (fixed so that results are reproducible to the last bit):
apply the 1-D operator along x first, then along y, then along z; inside the
1-D operator multiply each contributor by its weight and add contributors in
increasing index order.  The weights are powers of two, so every product is
exact.

Restriction is full weighting, ``R = P^T / 2^d``; in 1-D it is
``v_c[I] = 1/4 v_f[2I-1] + 1/2 v_f[2I] + 1/4 v_f[2I+1]`` (1-based), added in
that order.  It forms a coarse right-hand side from a fine one (a reading:
the paper samples an analytic right-hand side on each grid).
"""
from __future__ import annotations

import numpy as np


def _prolong_axis(v, axis):
    """1-D linear-spline prolongation along ``axis`` (length n_c -> 2 n_c + 1)."""
    v = np.moveaxis(v, axis, -1)
    nc = v.shape[-1]
    out = np.zeros(v.shape[:-1] + (2 * nc + 1,), dtype=v.dtype)
    # fine 0-based index 2I+1 coincides with coarse 0-based I
    out[..., 1::2] = v
    # fine 0-based index 2I sits between coarse I-1 and I (zero outside)
    pad = np.zeros(v.shape[:-1] + (nc + 2,), dtype=v.dtype)
    pad[..., 1:-1] = v
    out[..., 0::2] = 0.5 * pad[..., :-1] + 0.5 * pad[..., 1:]
    return np.moveaxis(out, -1, axis)


def _restrict_axis(v, axis):
    """1-D full weighting along ``axis`` (length 2 n_c + 1 -> n_c)."""
    v = np.moveaxis(v, axis, -1)
    nf = v.shape[-1]
    assert nf % 2 == 1
    out = 0.25 * v[..., 0:-2:2] + 0.5 * v[..., 1::2] + 0.25 * v[..., 2::2]
    return np.moveaxis(out, -1, axis)


def prolongate(vc, coarse_dims):
    """``v_f = P v_c`` for a vector (length n_c) or a block (n_c, s)."""
    vc = np.asarray(vc, dtype=np.float64)
    if vc.ndim == 2:
        return np.stack([prolongate(vc[:, j], coarse_dims) for j in range(vc.shape[1])], axis=1)
    g = vc.reshape(tuple(reversed(coarse_dims)))
    d = len(coarse_dims)
    for a in range(d):  # x (last array axis) first, then y, then z
        g = _prolong_axis(g, -1 - a)
    return g.reshape(-1)


def restrict(vf, fine_dims):
    """``v_c = P^T v_f / 2^d`` for a vector (length n_f) or a block (n_f, s)."""
    vf = np.asarray(vf, dtype=np.float64)
    if vf.ndim == 2:
        return np.stack([restrict(vf[:, j], fine_dims) for j in range(vf.shape[1])], axis=1)
    g = vf.reshape(tuple(reversed(fine_dims)))
    d = len(fine_dims)
    for a in range(d):
        g = _restrict_axis(g, -1 - a)
    return g.reshape(-1)


def coarse_dims_of(fine_dims):
    return tuple((d - 1) // 2 for d in fine_dims)
