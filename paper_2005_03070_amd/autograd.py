"""Two-grid solver object and a differentiable solve.

``TwoGridSolver`` strings the phases of the two-grid algorithm together
(Sec. 3 algorithm box, phase 1 and phase 3; Sec. 4.1 for BiCGStab): the
coarse operator, GMRES-DR on the coarse grid, moving its vectors and solution
to the fine grid, and the deflated fine solve.  With ``transpose=True`` every
phase uses ``A^T``: GMRES-DR on ``A_c^T`` yields left eigenvectors of
``A_c``, which deflate the adjoint system.

``DeflatedSolve`` is a ``torch.autograd.Function`` for
``u = A(k)^{-1} b`` with ``A(k)`` the divergence-form operator built from the
per-cell coefficient ``k``: the backward pass solves ``A^T lambda = dL/du``
with the same two-grid method on the transpose and returns
``dL/db = lambda`` and ``dL/dk`` from the edge formula (libtgdk's
tgdk_adjoint_grad_k).
"""
from __future__ import annotations

import torch

from . import api


class TwoGridSolver:
    """levels: how many times the fine grid is coarsened for the coarse phase
    (1: h_c = 2 h; the paper's Examples 1-2 coarsen 511^2 to 63^2, three
    levels, and Example 4 to 127^2, two).  The coarse right-hand side is
    restricted and the coarse solution and vectors prolongated one level at a
    time; at each intermediate grid the moved vectors are orthonormalised, so
    the fine space spans P...P W_c (only the span enters the projection)."""

    def __init__(self, op, m=30, k=10, nev=None, rtolev=1e-8, coarse_rtol=1e-8, maxcyc=300,
                 store=torch.float64, transpose=False, levels=1, grids=None):
        self.op = op
        # grids: the operators from fine to coarse (for operators that cannot
        # coarsen themselves, e.g. per-row coefficient arrays); else coarsened
        self.grids = list(grids) if grids is not None else [op]
        while len(self.grids) < levels + 1:
            self.grids.append(self.grids[-1].coarsen())
        self.coarse = self.grids[-1]
        self.m, self.k, self.nev = m, k, (k if nev is None else nev)
        self.rtolev, self.coarse_rtol, self.maxcyc = rtolev, coarse_rtol, maxcyc
        self.store = store
        self.transpose = transpose
        self.defl = None
        self.setup_report = None

    def setup(self, b):
        """Phase 1: GMRES-DR on the restricted right-hand side; returns the
        prolongated coarse solution (the fine initial guess)."""
        g = self.grids
        bc = b
        for lv in range(len(g) - 1):
            bc = api.restrict(g[lv], g[lv + 1], bc)
        xc, space, rep = api.coarse_setup(self.coarse, bc, self.m, self.k, self.nev, self.rtolev,
                                          self.coarse_rtol, self.maxcyc, self.transpose)
        self.setup_report = rep
        for lv in range(len(g) - 2, -1, -1):
            space = api.defl_prolongate(space, g[lv], self.store if lv == 0 else torch.float64)
            xc = api.prolongate(g[lv + 1], g[lv], xc)
        self.defl = space
        return xc

    def solve(self, b, x0=None, **kw):
        """Phase 3 with the current deflation space (set up on the first call)."""
        if self.defl is None:
            x0 = self.setup(b)
        kw.setdefault("transpose", self.transpose)
        return api.solve(self.op, b, x0=x0, defl=self.defl, **kw)


class DeflatedSolve(torch.autograd.Function):
    """u = A(k)^{-1} b for the 2-D operator -div(k grad u) + beta.grad(u).

    cfg: TwoGridSolver arguments, plus "solve" (fine-solve keywords of both
    solves) and optionally "solve_adjoint" (keywords of the backward solve
    alone)."""

    @staticmethod
    def forward(ctx, b, kcell, dims, beta, cfg):
        cfg = dict(cfg or {})
        solve_kw = cfg.pop("solve", {})
        adjoint_kw = cfg.pop("solve_adjoint", solve_kw)  # the backward solve's own settings, if given
        op = api.Operator.div_k(tuple(dims), kcell.detach(), tuple(beta))
        fwd = TwoGridSolver(op, **cfg)
        u, reps = fwd.solve(b.detach().contiguous(), **solve_kw)
        if reps[0].status != 0:
            raise RuntimeError(f"forward solve ended with status {reps[0].status_name}")
        ctx.op = op
        ctx.cfg = cfg
        ctx.solve_kw = adjoint_kw
        ctx.reports = {"forward": reps[0], "forward_setup": fwd.setup_report}
        ctx.save_for_backward(u)
        return u

    @staticmethod
    def backward(ctx, g):
        (u,) = ctx.saved_tensors
        adj = TwoGridSolver(ctx.op, transpose=True, **ctx.cfg)
        lam, reps = adj.solve(g.detach().contiguous(), **ctx.solve_kw)
        if reps[0].status != 0:
            raise RuntimeError(f"adjoint solve ended with status {reps[0].status_name}")
        gk = api.grad_k(ctx.op, lam, u)
        return lam, gk, None, None, None
