"""IDR(s)(ncyc)-Proj(k): restarted IDR(s) with a Galerkin projection before
every cycle.  Test infrastructure only.

Sec. 4.1 gives one box for BiCGStab(ncyc)-Proj(k) and IDR(ncyc)-Proj(k): the
same restarts, projection and per-cycle tolerance (step 3 a-d), with IDR in
place of BiCGStab in step c.  The paper runs the IDR code of van Gijzen and
Sonneveld with s = 4 by default, and s = 20 and s = 5 in the Sec. 5 Helmholtz
examples.  The inner solver here is the biorthogonal IDR(s) of van Gijzen and
Sonneveld (ACM TOMS 38(1), 2011), written from its description:

* a fixed n x s shadow matrix P with orthonormal columns: s seeded random
  columns (the same draw on the GPU side), orthonormalised;
* rounds of s + 1 operator applications.  Steps k = 1..s of a round build a
  direction u_k and g_k = A u_k from the current residual and the previous
  round's directions, make g_k orthogonal to p_1..p_(k-1) (which keeps
  M = P^T G lower triangular), then remove from r its component along g_k
  that leaves r orthogonal to p_1..p_k;
* the round ends with a dimension-reduction step r <- r - omega A r, where
  omega minimises ||r - omega A r||, enlarged when the angle between r and A r
  is too small (the "maintaining the convergence" choice of that paper, with
  kappa = 0.7; kappa = 0 gives the plain minimal-residual omega).

Readings where the paper is silent (the same as for BiCGStab(ncyc)-Proj(k)):
the cycle tolerance is relative to the residual after the projection; each
cycle starts IDR afresh (G = U = 0, M = I, omega = 1) from that residual with
the same P; the residual norm is tested after every update of r; a zero or
non-finite M_kk, A r, or omega ends the cycle (breakdown; a cycle that ends
before its first update ends the solve).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import operators
from .bicgstab import BREAKDOWN, NOT_CONVERGED, OK, SolveReport, cycle_tolerance
from .deflation import orthonormalize
from .projection import projector


def shadow_space(P0):
    """The shadow matrix of the paper's IDR code: its s random columns (the
    seeded draw ``P0``, n x s) orthonormalised, thin QR with diag(R) > 0."""
    return orthonormalize(np.asarray(P0, dtype=np.float64))


@dataclass
class IdrResult:
    e: np.ndarray
    mvps: int
    status: str                                   # "converged", "breakdown", "maxit"
    resnorms: list = field(default_factory=list)  # ||r|| after every update of r
    coefs: list = field(default_factory=list)     # the coefficient of that update (beta, or omega)
    kinds: list = field(default_factory=list)     # 0 after a step, 1 after a dimension reduction
    round_resnorms: list = field(default_factory=list)  # ||r|| after every dimension reduction
    checks: list = field(default_factory=list)    # per round: (max |upper(P^T G)|, max |P^T r| before the reduction)


def idrs_inner(matvec, r0, target, P, maxit, kappa=0.7, dtype=np.float64, check=False):
    """IDR(s) on ``A e = r0`` from ``e = 0`` until ``||r|| <= target``.

    Vectors are held in ``dtype`` (inner products and the small s x s
    systems in float64); ``P`` is n x s.  ``maxit`` bounds the operator
    applications."""
    def dot(a, b):
        return float(np.dot(np.asarray(a, np.float64), np.asarray(b, np.float64)))

    def norm(a):
        return math.sqrt(dot(a, a))

    n, s = P.shape
    P64 = np.asarray(P, np.float64)
    r = np.asarray(r0, dtype=dtype).copy()
    e = np.zeros_like(r)
    G = np.zeros((n, s), dtype=dtype)
    U = np.zeros((n, s), dtype=dtype)
    M = np.eye(s)
    om = 1.0
    mvps = 0
    res = IdrResult(e, 0, "maxit")
    if norm(r) <= target:
        res.status = "converged"
        return res
    while mvps < maxit:
        f = P64.T @ np.asarray(r, np.float64)
        for k in range(s):
            # c from the lower-triangular system M[k:, k:] c = f[k:]
            c = np.linalg.solve(np.tril(M[k:, k:]), f[k:])
            v = (r - (G[:, k:].astype(np.float64) @ c)).astype(dtype)
            uk = (U[:, k:].astype(np.float64) @ c + om * v.astype(np.float64)).astype(dtype)
            gk = np.asarray(matvec(uk)).astype(dtype)
            mvps += 1
            for i in range(k):
                alpha = dot(P64[:, i], gk) / M[i, i]
                gk = (gk - dtype(alpha) * G[:, i]).astype(dtype)
                uk = (uk - dtype(alpha) * U[:, i]).astype(dtype)
            G[:, k] = gk
            U[:, k] = uk
            M[k:, k] = [dot(P64[:, i], gk) for i in range(k, s)]
            if M[k, k] == 0.0 or not math.isfinite(M[k, k]):
                res.status = "breakdown"
                res.e, res.mvps = e, mvps
                return res
            beta = f[k] / M[k, k]
            r = (r - dtype(beta) * gk).astype(dtype)
            e = (e + dtype(beta) * uk).astype(dtype)
            nr = norm(r)
            res.resnorms.append(nr)
            res.coefs.append(beta)
            res.kinds.append(0)
            if nr <= target:
                res.status = "converged"
                res.e, res.mvps = e, mvps
                return res
            if k + 1 < s:
                f[k + 1:] = f[k + 1:] - beta * M[k + 1:, k]
            if mvps >= maxit:
                res.e, res.mvps = e, mvps
                return res
        if check:
            upper = np.triu(P64.T @ G.astype(np.float64), 1)
            res.checks.append((float(np.abs(upper).max(initial=0.0)),
                               float(np.abs(P64.T @ np.asarray(r, np.float64)).max())))
        # dimension reduction
        t = np.asarray(matvec(r)).astype(dtype)
        mvps += 1
        tt = dot(t, t)
        ts = dot(t, r)
        if tt == 0.0 or ts == 0.0 or not math.isfinite(ts / tt):
            res.status = "breakdown"
            res.e, res.mvps = e, mvps
            return res
        om = ts / tt
        rho = abs(ts) / (math.sqrt(tt) * norm(r))
        if rho < kappa:
            om = om * kappa / rho
        e = (e + dtype(om) * r).astype(dtype)
        r = (r - dtype(om) * t).astype(dtype)
        nr = norm(r)
        res.resnorms.append(nr)
        res.coefs.append(om)
        res.kinds.append(1)
        res.round_resnorms.append(nr)
        if nr <= target:
            res.status = "converged"
            res.e, res.mvps = e, mvps
            return res
    res.e, res.mvps = e, mvps
    return res


def idrs_proj(op, b, P, x0=None, V=None, H=None, rtol=1e-8, ncyc=20, max_extra=None, maxit_cycle=100000,
              precision="fp64", fp32_floor=1e-4, kappa=0.7, transpose=False, projection="galerkin",
              precond=None, Z=None):
    """IDR(s)(ncyc)-Proj(k) on ``A x = b`` with shadow matrix ``P`` (n x s).

    ``V`` (n x k, orthonormal) and ``H = V^T A V`` may be None (k = 0).
    ``precond`` (``v -> M^{-1} v``): right preconditioning; the inner cycles
    run on ``A M^{-1}`` and ``x += M^{-1} e``; the projection then needs
    ``Z = M^{-1} V`` and ``H = V^T A Z`` (``projection.precond_space``).
    Returns ``(x, SolveReport)``; ``first_scalars`` holds, for the first
    updates of r in the first cycle, (||r||, coefficient, 1 at a dimension
    reduction else 0)."""
    mv = (lambda z: operators.apply_transpose(op, z)) if transpose else (lambda z: operators.apply(op, z))
    if max_extra is None:
        max_extra = ncyc
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    rep = SolveReport()
    r = b - mv(x)
    rep.mvp_boundary += 1
    nu0 = float(np.linalg.norm(r))
    bnorm = float(np.linalg.norm(b))
    tau = rtol * min(bnorm, nu0)
    if nu0 <= tau or nu0 == 0.0:
        rep.relres_true = nu0 / bnorm if bnorm > 0 else 0.0
        return x, rep
    inner_dtype = np.float32 if precision == "fp32_ir" else np.float64
    Pin = np.asarray(P, dtype=inner_dtype)
    proj = projector(op, V, H, transpose, projection, Z) if V is not None and V.shape[1] > 0 else None
    mvc = mv if precond is None else (lambda z: mv(precond(z)))
    icyc = 0
    while True:
        icyc += 1
        if proj is not None:                            # step a)
            x, r, _ = proj(x, r)
            rep.mvp_boundary += 1
        nu = float(np.linalg.norm(r))
        if nu <= tau:
            break
        rt, branch = cycle_tolerance(nu, nu0, tau, icyc, ncyc)   # step b)
        rep.cycle_nu.append((nu, nu0, tau, icyc, ncyc))          # what decided the branch
        if precision == "fp32_ir":
            rt = max(rt, fp32_floor)
        inner = idrs_inner(mvc, r, rt * nu, Pin, maxit_cycle, kappa=kappa, dtype=inner_dtype)  # step c)
        rep.mvp_inner += inner.mvps
        if icyc == 1:
            rep.first_scalars = list(zip(inner.resnorms, inner.coefs, inner.kinds))[:8]
        rep.branches.append(branch)
        rep.inner_iters.append(inner.mvps)
        rep.cycle_mvps.append(inner.mvps)
        x = x + (inner.e.astype(np.float64) if precond is None else precond(inner.e.astype(np.float64)))
        r = b - mv(x)                                    # true residual, FP64
        rep.mvp_boundary += 1
        nu = float(np.linalg.norm(r))
        rep.nu_hist.append(nu)
        rep.cycles = icyc
        if nu <= tau:                                    # step d)
            break
        if inner.status == "breakdown" and inner.mvps <= 1:
            rep.status = BREAKDOWN
            break
        if icyc >= ncyc + max_extra:
            rep.status = NOT_CONVERGED
            break
    rep.cycles = icyc
    rep.relres_true = float(np.linalg.norm(b - mv(x))) / bnorm
    return x, rep


__all__ = ["shadow_space", "idrs_inner", "idrs_proj", "IdrResult", "OK", "BREAKDOWN", "NOT_CONVERGED"]
