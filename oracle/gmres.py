"""GMRES(m) cycles and GMRES(m)-Proj(k) (plain FP64).  Test infrastructure only.

GMRES(m)-Proj(k) follows the Sec. 2.2 box: alternate (A) a Galerkin
projection over the k approximate eigenvectors and (B) one cycle of GMRES(m).
Convergence is checked at the end of each cycle only (Sec. 3, Example 1).

One GMRES(m) cycle on ``A e = r``: Arnoldi ``A V_m = V_{m+1} Hbar_m`` from
``v_1 = r/||r||`` with modified Gram-Schmidt and one full
re-orthogonalisation pass, then ``y = argmin || ||r|| e_1 - Hbar_m y ||`` and
``e = V_m y``.  The least-squares problem is solved with ``numpy.linalg.lstsq``
as one library step.  A zero ``h_{j+1,j}`` ends the cycle early (the Krylov
space is invariant and ``e`` is exact).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import operators
from .projection import projector

OK, NOT_CONVERGED = 0, 1


def arnoldi(matvec, v0, m, V_init=None, H_init=None, start=0):
    """Arnoldi with MGS plus one re-orthogonalisation pass.

    Builds columns ``start+1 .. m`` of ``V`` (n x (m+1)) and columns
    ``start .. m-1`` of ``Hbar`` ((m+1) x m).  With ``start = 0`` the basis
    starts from ``v0`` (normalised).  Returns ``(V, Hbar, j_end)`` where
    ``j_end`` is the number of columns of ``Hbar`` that were completed."""
    n = v0.shape[0]
    V = np.zeros((n, m + 1)) if V_init is None else V_init
    H = np.zeros((m + 1, m)) if H_init is None else H_init
    if start == 0:
        V[:, 0] = v0 / np.linalg.norm(v0)
    for j in range(start, m):
        w = matvec(V[:, j])
        for _pass in range(2):
            for i in range(j + 1):
                hij = float(np.dot(V[:, i], w))
                H[i, j] += hij
                w = w - hij * V[:, i]
        hn = float(np.linalg.norm(w))
        H[j + 1, j] = hn
        if hn == 0.0:
            return V, H, j + 1
        V[:, j + 1] = w / hn
    return V, H, m


def gmres_cycle(matvec, r, m):
    """One GMRES(m) cycle on ``A e = r`` from ``e = 0``.

    Returns ``(e, lsq_residual_norm, steps)``."""
    beta = float(np.linalg.norm(r))
    V, H, j = arnoldi(matvec, r, m)
    rhs = np.zeros(j + 1)
    rhs[0] = beta
    y, *_ = np.linalg.lstsq(H[: j + 1, :j], rhs, rcond=None)
    res = float(np.linalg.norm(rhs - H[: j + 1, :j] @ y))
    return V[:, :j] @ y, res, j


@dataclass
class GmresReport:
    status: int = OK
    cycles: int = 0
    mvp_inner: int = 0
    mvp_boundary: int = 0
    relres_true: float = float("nan")
    nu_hist: list = field(default_factory=list)
    lsq_hist: list = field(default_factory=list)
    cycle_mvps: list = field(default_factory=list)  # steps per cycle


def gmres_proj(op, b, x0=None, V=None, H=None, rtol=1e-8, m=50, maxcyc=1000,
               transpose=False, projection="galerkin", lengths=None, precond=None, Z=None):
    """GMRES(m)-Proj(k) on ``A x = b``; ``V``/``H`` may be None (k = 0);
    ``projection="minres"`` takes the MinRes variant of the projection.
    ``lengths``: variable restarting (Sec. 4.3, Table 4.3): cycle j
    (1-based) has ``lengths[j-1]`` steps while the list lasts, then ``m``.
    ``precond`` (``v -> M^{-1} v``): right preconditioning, the cycles run on
    ``A M^{-1}`` and ``x += M^{-1} e``; the projection then needs
    ``Z = M^{-1} V`` and ``H = V^T A Z`` (``projection.precond_space``).

    The overall tolerance is ``tau = rtol * min(||b||, ||r0||)``, as for
    BiCGStab(ncyc)-Proj(k)."""
    mv = (lambda z: operators.apply_transpose(op, z)) if transpose else (lambda z: operators.apply(op, z))
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    rep = GmresReport()
    r = b - mv(x)
    rep.mvp_boundary += 1
    bnorm = float(np.linalg.norm(b))
    nu0 = float(np.linalg.norm(r))
    tau = rtol * min(bnorm, nu0)
    if nu0 <= tau:
        rep.relres_true = nu0 / bnorm if bnorm else 0.0
        return x, rep
    proj = projector(op, V, H, transpose, projection, Z) if V is not None and V.shape[1] > 0 else None
    mvc = mv if precond is None else (lambda z: mv(precond(z)))
    for icyc in range(1, maxcyc + 1):
        if proj is not None:                          # (A) projection
            x, r, _ = proj(x, r)
            rep.mvp_boundary += 1
            if float(np.linalg.norm(r)) <= tau:
                rep.cycles = icyc
                break
        mc = lengths[icyc - 1] if lengths is not None and icyc <= len(lengths) else m
        e, lsq, steps = gmres_cycle(mvc, r, mc)        # (B) one GMRES(mc) cycle
        rep.mvp_inner += steps
        rep.cycle_mvps.append(steps)
        x = x + (e if precond is None else precond(e))
        r = b - mv(x)
        rep.mvp_boundary += 1
        nu = float(np.linalg.norm(r))
        rep.nu_hist.append(nu)
        rep.lsq_hist.append(lsq)
        rep.cycles = icyc
        if nu <= tau:
            break
    else:
        rep.status = NOT_CONVERGED
    rep.relres_true = float(np.linalg.norm(b - mv(x))) / bnorm
    return x, rep
