"""Discretised PDE operators (plain FP64).  Test infrastructure only.

The paper (Sec. 1) solves ``A x = b`` from finite-difference discretisations
of PDEs on the unit square/cube with zero Dirichlet boundary values.
Example 1 (Sec. 3) uses the 2-D convection-diffusion operator
``-exp(5xy)(u_xx + u_yy) + 40 u_x + 40 u_y``; Example 3 (Sec. 4.2) the same
operator on a 127x127 grid.  The workloads of this project additionally use
``-Lap(u) + beta.grad(u) + sigma u`` in 2-D and 3-D and the divergence-form
``-div(k grad u) + beta.grad(u)`` with a per-cell coefficient ``k``.

Conventions (readings where the paper is silent, listed in the design notes):

* interior grid ``n_x x n_y (x n_z)``, spacing ``h_a = 1/(n_a + 1)`` per axis;
* unknown ordering lexicographic with x fastest: a vector of length
  ``n = n_x n_y n_z`` reshapes in C order to ``(n_z, n_y, n_x)``;
* centred second differences and centred first differences, matrix NOT
  scaled by ``h^2``;
* neighbours outside the domain are dropped (zero Dirichlet data).

An operator is a set of per-row stencil coefficients: ``C`` (centre) and
``W, E`` (x-1, x+1), ``S, N`` (y-1, y+1), ``D, U`` (z-1, z+1).  Each is a
Python float (constant) or an array of the grid's shape.  Row ``p`` of
``A x`` is ``C_p x_p + sum_o c_o(p) x_{p+o}``.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# offset name -> (axis in the C-ordered grid array, step)
#   axis -1 is x, -2 is y, -3 is z
OFFSETS = {
    "W": (-1, -1), "E": (-1, +1),
    "S": (-2, -1), "N": (-2, +1),
    "D": (-3, -1), "U": (-3, +1),
}
MIRROR = {"W": "E", "E": "W", "S": "N", "N": "S", "D": "U", "U": "D"}


class StencilOp:
    """A 5-point (2-D) or 7-point (3-D) stencil operator with zero Dirichlet
    boundary.  ``dims`` is ``(n_x, n_y)`` or ``(n_x, n_y, n_z)``."""

    def __init__(self, dims, coef, kind="const", params=None):
        self.dims = tuple(int(d) for d in dims)
        self.dim = len(self.dims)
        assert self.dim in (2, 3)
        self.shape = tuple(reversed(self.dims))  # C-order array shape
        self.n = int(np.prod(self.dims))
        self.h = tuple(1.0 / (d + 1) for d in self.dims)
        self.coef = dict(coef)
        self.kind = kind
        self.params = dict(params or {})

    @property
    def names(self):
        return ["C", "W", "E", "S", "N"] + (["D", "U"] if self.dim == 3 else [])

    def coef_array(self, name):
        """Coefficient ``name`` as a full array of the grid shape."""
        c = self.coef[name]
        return np.broadcast_to(np.asarray(c, dtype=np.float64), self.shape).copy()


def _shift(xg, axis, step):
    """Value of grid function ``xg`` at the neighbour ``p + step`` along
    ``axis`` for every point ``p``; zero where that neighbour is outside."""
    out = np.zeros_like(xg)
    src = [slice(None)] * xg.ndim
    dst = [slice(None)] * xg.ndim
    if step > 0:
        src[axis] = slice(step, None)
        dst[axis] = slice(None, -step)
    else:
        src[axis] = slice(None, step)
        dst[axis] = slice(-step, None)
    out[tuple(dst)] = xg[tuple(src)]
    return out


def apply(op: StencilOp, x):
    """``y = A x`` for one vector (length n) or a block (n, s) of vectors."""
    x = np.asarray(x)
    if x.ndim == 2:
        return np.stack([apply(op, x[:, j]) for j in range(x.shape[1])], axis=1)
    xg = x.reshape(op.shape)
    y = op.coef["C"] * xg
    for name in op.names[1:]:
        axis, step = OFFSETS[name]
        y = y + op.coef[name] * _shift(xg, axis, step)
    return y.reshape(-1)


def apply_transpose(op: StencilOp, x):
    """``y = A^T x``.  Entry ``(A^T)_{p,q} = A_{q,p}``: for the neighbour
    ``q = p + o`` of ``p`` it is row q's coefficient for offset ``-o``."""
    x = np.asarray(x)
    if x.ndim == 2:
        return np.stack([apply_transpose(op, x[:, j]) for j in range(x.shape[1])], axis=1)
    xg = x.reshape(op.shape)
    y = op.coef["C"] * xg
    for name in op.names[1:]:
        axis, step = OFFSETS[name]
        # row q = p + step uses coefficient MIRROR[name] to reach p
        prod = op.coef[MIRROR[name]] * xg
        y = y + _shift(np.broadcast_to(prod, op.shape), axis, step)
    return y.reshape(-1)


def to_csr(op: StencilOp):
    """The operator as an explicit scipy CSR matrix (rows/cols lexicographic)."""
    n = op.n
    idx = np.arange(n).reshape(op.shape)
    rows, cols, vals = [idx.reshape(-1)], [idx.reshape(-1)], [op.coef_array("C").reshape(-1)]
    for name in op.names[1:]:
        axis, step = OFFSETS[name]
        nb = _shift(idx + 1, axis, step) - 1  # -1 marks "outside"
        c = op.coef_array(name)
        mask = nb >= 0
        rows.append(idx[mask])
        cols.append(nb[mask])
        vals.append(c[mask])
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    A.sum_duplicates()
    return A


def norm1(op: StencilOp):
    """``||A||_1`` (maximum absolute column sum) of the explicit matrix."""
    return float(abs(to_csr(op)).sum(axis=0).max())


# ---------------------------------------------------------------------------
# constructors
# ---------------------------------------------------------------------------

def const_cd(dims, beta=(0.0, 0.0, 0.0), sigma=0.0):
    """``-Lap(u) + beta.grad(u) + sigma u`` with constant ``beta``: centre
    ``sum_a 2/h_a^2 + sigma``; along axis a the lower neighbour gets
    ``-1/h_a^2 - beta_a/(2 h_a)`` and the upper ``-1/h_a^2 + beta_a/(2 h_a)``."""
    dims = tuple(dims)
    d = len(dims)
    beta = tuple(beta) + (0.0,) * (3 - len(beta))
    h = [1.0 / (m + 1) for m in dims]
    coef = {"C": sum(2.0 / (ha * ha) for ha in h) + sigma}
    lo, hi = ["W", "S", "D"], ["E", "N", "U"]
    for a in range(d):
        coef[lo[a]] = -1.0 / (h[a] * h[a]) - beta[a] / (2.0 * h[a])
        coef[hi[a]] = -1.0 / (h[a] * h[a]) + beta[a] / (2.0 * h[a])
    return StencilOp(dims, coef, kind="const",
                     params={"beta": beta[:d], "sigma": sigma})


def example1_operator(n):
    """The operator of Examples 1-3 (Sec. 3, Sec. 4.2):
    ``-exp(5xy)(u_xx + u_yy) + 40 u_x + 40 u_y`` on an ``n x n`` interior
    grid, non-divergence form, the diffusion coefficient taken at the node."""
    h = 1.0 / (n + 1)
    xs = h * np.arange(1, n + 1)
    X, Y = np.meshgrid(xs, xs, indexing="xy")  # shape (n_y, n_x): X varies along columns
    a = np.exp(5.0 * X * Y)
    coef = {
        "C": 4.0 * a / (h * h),
        "W": -a / (h * h) - 40.0 / (2 * h),
        "E": -a / (h * h) + 40.0 / (2 * h),
        "S": -a / (h * h) - 40.0 / (2 * h),
        "N": -a / (h * h) + 40.0 / (2 * h),
    }
    return StencilOp((n, n), coef, kind="example1")


def div_k(dims, kcell, beta=(0.0, 0.0), sigma=0.0):
    """2-D ``-div(k grad u) + beta.grad(u) + sigma u`` with ``k`` given per
    primal cell.  ``kcell`` has shape ``(n_y + 1, n_x + 1)``: cell ``(cj, ci)``
    is the square between node columns ``ci, ci+1`` and node rows ``cj, cj+1``
    (nodes numbered 0..n+1 including the boundary).  A grid edge takes the
    arithmetic mean of the two cells that have it as a side; the flux form
    gives centre ``sum_e k_e / h^2`` and neighbour ``-k_e / h^2``."""
    nx, ny = dims
    kcell = np.asarray(kcell, dtype=np.float64)
    assert kcell.shape == (ny + 1, nx + 1)
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    # interior node (i, j), 1-based, sits at array index [j-1, i-1].
    # cells touching it: [j-1, i-1] (SW), [j-1, i] (SE), [j, i-1] (NW), [j, i] (NE)
    k_sw = kcell[:-1, :-1]
    k_se = kcell[:-1, 1:]
    k_nw = kcell[1:, :-1]
    k_ne = kcell[1:, 1:]
    ke_e = 0.5 * (k_se + k_ne)  # edge to (i+1, j): cells below and above it
    ke_w = 0.5 * (k_sw + k_nw)  # edge to (i-1, j)
    ke_n = 0.5 * (k_nw + k_ne)  # edge to (i, j+1): cells left and right of it
    ke_s = 0.5 * (k_sw + k_se)  # edge to (i, j-1)
    coef = {
        "C": (ke_e + ke_w) / (hx * hx) + (ke_n + ke_s) / (hy * hy) + sigma,
        "W": -ke_w / (hx * hx) - beta[0] / (2 * hx),
        "E": -ke_e / (hx * hx) + beta[0] / (2 * hx),
        "S": -ke_s / (hy * hy) - beta[1] / (2 * hy),
        "N": -ke_n / (hy * hy) + beta[1] / (2 * hy),
    }
    return StencilOp(dims, coef, kind="div_k",
                     params={"kcell": kcell, "beta": tuple(beta), "sigma": sigma})


def coarse_kcell(kcell):
    """Coarse cell coefficient: geometric mean of the 2x2 fine cells it covers
    (fine grid ``n_f = 2 n_c + 1`` has ``2 (n_c + 1)`` cells per axis)."""
    k = np.asarray(kcell, dtype=np.float64)
    assert k.shape[0] % 2 == 0 and k.shape[1] % 2 == 0
    lg = np.log(k)
    return np.exp(0.25 * (lg[0::2, 0::2] + lg[0::2, 1::2] + lg[1::2, 0::2] + lg[1::2, 1::2]))


def coarsen(op: StencilOp):
    """The same PDE on the coarse grid with ``h_c = 2 h_f`` (``n_c = (n_f-1)/2``)."""
    for d in op.dims:
        assert d % 2 == 1, "fine grid sizes must be odd"
    cdims = tuple((d - 1) // 2 for d in op.dims)
    if op.kind == "const":
        return const_cd(cdims, op.params["beta"], op.params["sigma"])
    if op.kind == "div_k":
        return div_k(cdims, coarse_kcell(op.params["kcell"]), op.params["beta"], op.params["sigma"])
    if op.kind == "example1":
        return example1_operator(cdims[0])
    raise ValueError(op.kind)
