"""BiCGStab(ncyc)-Proj(k): restarted BiCGStab with a Galerkin projection
before every cycle (plain FP64, optional FP32 inner cycles).
Test infrastructure only.

Follows Sec. 4.1, the "BiCGStab(ncyc)-Proj(k)" box, step 3:

  a) Galerkin projection over the k approximate eigenvectors;
  b) the cycle's relative tolerance ``rticyc`` is the smaller of
     ``(rtol ||r0|| / ||r||)^(1/(ncyc - icyc + 1))`` and
     ``(||r0|| / ||r||) rtol^(icyc/ncyc)``;
  c) run BiCGStab to that relative tolerance;
  d) stop once ``||r||`` is below the tolerance.

``ncyc`` is the number of cycles (so ``ncyc - 1`` restarts), not a cycle
length.  ``k = 0`` (no vectors) is plain restarted BiCGStab (Sec. 4.2,
Example 3), and ``ncyc = 1, k = 0`` is non-restarted BiCGStab.

The inner solver is the textbook Bi-CGSTAB of van der Vorst (1992), which the
paper cites; the paper ran MATLAB's implementation.  Readings where the paper
is silent:

* the shadow vector is the residual at the start of the cycle;
* the cycle tolerance is relative to the residual norm at the cycle start
  (after the projection);
* the cycle exits after the half step when ``||s||`` already meets the target;
* a breakdown (``rho = 0``, ``r^ . v = 0``, ``omega = 0`` or a non-finite
  scalar) ends the cycle, and the next restart renews the shadow vector; a
  cycle that breaks down before its first update ends the solve with status
  ``breakdown``;
* after every inner cycle the solution is updated and the true residual
  ``b - A x`` is recomputed in FP64 (the paper notes one extra operator
  application per cycle that its tables do not count);
* the overall tolerance is ``tau = rtol * min(||b||, ||r0||)``;
* if ``ncyc`` cycles are used up before convergence, further cycles run with
  relative tolerance ``tau / ||r||`` up to ``max_extra`` more, then the solve
  returns ``not_converged``.

FP32 inner cycles with FP64 refinement (an extension): the projection, the
true residual and ``x`` stay FP64; the inner BiCGStab runs on the correction
system with every vector in float32 (dot products accumulated in float64);
the cycle tolerance is floored at ``fp32_floor`` because float32 BiCGStab
cannot reach arbitrarily small relative residuals.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import operators
from .projection import projector

OK, NOT_CONVERGED, BREAKDOWN = 0, 1, 2


def cycle_tolerance(nu, nu0, tau, icyc, ncyc):
    """``rticyc`` of step 3 b) with ``rtol ||r0||`` replaced by ``tau``.

    Returns ``(rticyc, branch)`` where branch 1 is the first criterion (equal
    share of the remaining orders of magnitude) and 2 the second (at least
    ``icyc/ncyc`` of the way); ties count as branch 1.  Past ``ncyc`` the
    tolerance is ``tau / nu`` (branch 3)."""
    if icyc > ncyc:
        return tau / nu, 3
    rtol_eff = tau / nu0
    t1 = (tau / nu) ** (1.0 / (ncyc - icyc + 1))
    t2 = (nu0 / nu) * rtol_eff ** (icyc / ncyc)
    return (t1, 1) if t1 <= t2 else (t2, 2)


@dataclass
class InnerResult:
    e: np.ndarray
    iters: int
    mvps: int
    status: str  # "converged", "half", "breakdown", "maxit"
    scalars: list = field(default_factory=list)  # (rho, alpha, omega) per iteration
    resid: np.ndarray = None  # the recursive residual at exit (s after a half step, else r)


def bicgstab_inner(matvec, r0, target, maxit, dtype=np.float64):
    """Bi-CGSTAB on ``A e = r0`` from ``e = 0`` until ``||r|| <= target``.

    Vectors are held in ``dtype``; inner products are accumulated in float64.
    """
    def dot(a, b):
        return float(np.dot(a.astype(np.float64), b.astype(np.float64)))

    r = np.asarray(r0, dtype=dtype).copy()
    rhat = r.copy()
    e = np.zeros_like(r)
    p = np.zeros_like(r)
    v = np.zeros_like(r)
    rho_old = alpha = omega = 1.0
    mvps = 0
    scalars = []
    for it in range(maxit):
        rho = dot(rhat, r)
        if rho == 0.0 or not math.isfinite(rho):
            return InnerResult(e, it, mvps, "breakdown", scalars, r)
        if it == 0:
            p = r.copy()
        else:
            beta = (rho / rho_old) * (alpha / omega)
            p = (r + dtype(beta) * (p - dtype(omega) * v)).astype(dtype)
        v = matvec(p).astype(dtype)
        mvps += 1
        sigma = dot(rhat, v)
        if sigma == 0.0 or not math.isfinite(sigma):
            return InnerResult(e, it, mvps, "breakdown", scalars, r)
        alpha = rho / sigma
        s = (r - dtype(alpha) * v).astype(dtype)
        if math.sqrt(dot(s, s)) <= target:
            e = (e + dtype(alpha) * p).astype(dtype)
            scalars.append((rho, alpha, float("nan")))
            return InnerResult(e, it + 1, mvps, "half", scalars, s)
        t = matvec(s).astype(dtype)
        mvps += 1
        tt = dot(t, t)
        omega = dot(t, s) / tt if tt != 0.0 else 0.0
        scalars.append((rho, alpha, omega))
        e = (e + dtype(alpha) * p + dtype(omega) * s).astype(dtype)
        r = (s - dtype(omega) * t).astype(dtype)
        rho_old = rho
        if omega == 0.0 or not math.isfinite(omega):
            return InnerResult(e, it + 1, mvps, "breakdown", scalars, r)
        if math.sqrt(dot(r, r)) <= target:
            return InnerResult(e, it + 1, mvps, "converged", scalars, r)
    return InnerResult(e, maxit, mvps, "maxit", scalars, r)


@dataclass
class SolveReport:
    status: int = OK
    cycles: int = 0
    mvp_inner: int = 0
    mvp_boundary: int = 0
    relres_true: float = float("nan")
    nu_hist: list = field(default_factory=list)   # ||r|| after each cycle's true residual
    branches: list = field(default_factory=list)  # rticyc branch per cycle
    inner_iters: list = field(default_factory=list)
    cycle_mvps: list = field(default_factory=list)     # inner operator applications per cycle
    first_scalars: list = field(default_factory=list)  # first 8 inner (rho, alpha, omega), across cycles
    cycle_nu: list = field(default_factory=list)   # (nu, nu0, tau, icyc, ncyc) at each cycle start


def bicgstab_proj(op, b, x0=None, V=None, H=None, rtol=1e-8, ncyc=20,
                  max_extra=None, maxit_cycle=100000, precision="fp64",
                  fp32_floor=1e-4, transpose=False, projection="galerkin", progress=None):
    """BiCGStab(ncyc)-Proj(k) on ``A x = b`` (or ``A^T x = b``).

    ``V`` (n x k, orthonormal) and ``H = V^T A V`` may be None (k = 0);
    ``projection="minres"`` takes the MinRes variant of step a) (``H`` is then
    not used).  ``progress`` (optional, ``f(cycle, ||r||)``) is called after
    every cycle's true residual and changes nothing.  Returns
    ``(x, SolveReport)``."""
    mv = (lambda z: operators.apply_transpose(op, z)) if transpose else (lambda z: operators.apply(op, z))
    if max_extra is None:
        max_extra = ncyc
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    rep = SolveReport()
    r = b - mv(x)
    rep.mvp_boundary += 1
    nu0 = float(np.linalg.norm(r))
    tau = rtol * min(float(np.linalg.norm(b)), nu0)
    bnorm = float(np.linalg.norm(b))
    if nu0 <= tau or nu0 == 0.0:
        rep.relres_true = nu0 / bnorm if bnorm > 0 else 0.0
        return x, rep
    inner_dtype = np.float32 if precision == "fp32_ir" else np.float64
    proj = projector(op, V, H, transpose, projection) if V is not None and V.shape[1] > 0 else None
    icyc = 0
    while True:
        icyc += 1
        if proj is not None:                            # step a)
            x, r, _ = proj(x, r)
            rep.mvp_boundary += 1
        nu = float(np.linalg.norm(r))
        if nu <= tau:                                   # step d) (after projection)
            break
        rt, branch = cycle_tolerance(nu, nu0, tau, icyc, ncyc)   # step b)
        rep.cycle_nu.append((nu, nu0, tau, icyc, ncyc))          # what decided the branch
        if precision == "fp32_ir":
            rt = max(rt, fp32_floor)
        inner = bicgstab_inner(mv, r, rt * nu, maxit_cycle, dtype=inner_dtype)  # step c)
        rep.mvp_inner += inner.mvps
        rep.branches.append(branch)
        rep.inner_iters.append(inner.iters)
        rep.cycle_mvps.append(inner.mvps)
        if len(rep.first_scalars) < 8:
            rep.first_scalars += inner.scalars[: 8 - len(rep.first_scalars)]
        x = x + inner.e.astype(np.float64)
        r = b - mv(x)                                   # true residual, FP64
        rep.mvp_boundary += 1
        nu = float(np.linalg.norm(r))
        rep.nu_hist.append(nu)
        rep.cycles = icyc
        if progress is not None:
            progress(icyc, nu)
        if nu <= tau:                                   # step d)
            break
        if inner.status == "breakdown" and inner.iters == 0:
            rep.status = BREAKDOWN
            break
        if icyc >= ncyc + max_extra:
            rep.status = NOT_CONVERGED
            break
    rep.cycles = icyc
    rep.relres_true = float(np.linalg.norm(b - mv(x))) / bnorm
    return x, rep
