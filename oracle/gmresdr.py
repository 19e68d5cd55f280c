"""GMRES-DR(m,k): GMRES with deflated restarting (plain FP64).
Test infrastructure only.

The paper uses GMRES-DR on the coarse grid to solve the coarse system and at
the same time compute the eigenpairs with smallest eigenvalues (Sec. 2.1;
phase 1 of the Sec. 3 algorithm).  A cycle works in
``span{y_1..y_k, r0, A r0, ..., A^(m-k-1) r0}`` where the ``y_i`` are the
harmonic Ritz vectors of the previous cycle.  The paper only summarises the
method; the steps below are those of the published GMRES-DR (Morgan 2002),
written from its description:

1. The first cycle is GMRES(m) from the initial guess: Arnoldi
   ``A V_m = V_{m+1} Hbar_m``, ``y = argmin ||c - Hbar_m y||`` with
   ``c = beta e_1``, ``x += V_m y``, and the least-squares residual
   ``q = c - Hbar_m y`` (the true residual is ``V_{m+1} q``).
2. Harmonic Ritz pairs of ``A`` w.r.t. ``range(V_m)``: solve
   ``H_m^T f = e_m`` and take the eigenpairs ``(theta, g)`` of
   ``H_m + h_{m+1,m}^2 f e_m^T``.  Keep the k with smallest ``|theta|``.
3. ``P_{k+1}``: the columns ``g_i`` (real and imaginary parts for a complex
   pair) padded with a zero row, then ``q``; orthonormalised by QR.
4. Restart: ``V_{k+1} <- V_{m+1} P_{k+1}``,
   ``Hbar_k <- P_{k+1}^T Hbar_m P_k``; the new least-squares right-hand side
   is ``c = P_{k+1}^T q``.
5. Arnoldi continues from ``v_{k+1}`` (re-orthogonalised against
   ``v_1..v_k``) out to dimension m; solve the least-squares problem with the
   full ``Hbar_m``; update ``x`` and ``q``.
6. At the end of a cycle the eigen-residual of each harmonic Ritz pair is
   ``||Hbar_m g - rho [g; 0]||`` with ``||g|| = 1`` and the Rayleigh quotient
   ``rho = g^H H_m g`` (because ``A V_m g = V_{m+1} Hbar_m g``); it is divided
   by ``||A||_1`` (a reading: the paper's "residual norm below 1e-8" is taken
   relative to the matrix norm because the unscaled operator has norm
   ``~8/h^2``).  Residuals are computed only at cycle ends (Sec. 3, Ex. 1).
7. Stop when the linear residual is below ``rtol ||b||`` and the ``nev``
   smallest pairs are converged, or after ``maxcyc`` cycles.  The returned
   basis ``W`` is the first k columns of ``V_{m+1} P_{k+1}`` built from the
   last cycle, i.e. an orthonormal basis of the span of the final harmonic
   Ritz vectors (only the span matters for the Galerkin projection).

Selection (a reading): sort by ``|theta|``, then by real part, then complex
pairs with positive imaginary part first; if the k-th kept value is one half
of a conjugate pair its partner is kept too (k+1 vectors for that restart).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import operators
from .gmres import arnoldi


def harmonic_ritz(Hbar, m):
    """All harmonic Ritz pairs of an (m+1) x m upper-Hessenberg-like matrix.

    Returns ``(theta, G)`` with ``G[:, i]`` the coefficient vector of pair i."""
    Hm = Hbar[:m, :m]
    hm = Hbar[m, m - 1]
    em = np.zeros(m)
    em[-1] = 1.0
    f = np.linalg.solve(Hm.T, em)
    M = Hm + (hm * hm) * np.outer(f, em)
    theta, G = np.linalg.eig(M)
    return theta, G


def select_smallest(theta, k):
    """Indices of the k harmonic Ritz values to keep (see module docstring).
    Returns a list of indices; complex pairs appear as (index of the value
    with positive imaginary part) followed by its conjugate's index."""
    order = sorted(range(len(theta)),
                   key=lambda i: (abs(theta[i]), theta[i].real, -np.sign(theta[i].imag)))
    chosen = []
    used = set()
    for i in order:
        if len(chosen) >= k:
            break
        if i in used:
            continue
        if abs(theta[i].imag) > 0:
            # find the conjugate partner
            cands = [j for j in range(len(theta)) if j not in used and j != i
                     and abs(theta[j] - np.conj(theta[i])) <= 1e-12 * max(1.0, abs(theta[i]))]
            j = min(cands, key=lambda j: abs(theta[j] - np.conj(theta[i]))) if cands else None
            ip, jn = (i, j) if theta[i].imag > 0 else (j, i)
            chosen.append(ip)
            used.add(ip)
            if jn is not None:
                chosen.append(jn)
                used.add(jn)
        else:
            chosen.append(i)
            used.add(i)
    return chosen


def real_basis(theta, G, chosen):
    """Real columns spanning the chosen harmonic Ritz vectors: ``g`` for a
    real value, ``Re g`` and ``Im g`` for a conjugate pair."""
    cols = []
    i = 0
    while i < len(chosen):
        a = chosen[i]
        if abs(theta[a].imag) > 0:
            cols.append(G[:, a].real)
            cols.append(G[:, a].imag)
            i += 2
        else:
            cols.append(G[:, a].real)
            i += 1
    return np.stack(cols, axis=1)


def eigen_residuals(Hbar, m, theta, G, idx):
    """``||Hbar g - rho [g;0]||`` for ``||g|| = 1``, ``rho = g^H H_m g``."""
    out = []
    for i in idx:
        g = G[:, i] / np.linalg.norm(G[:, i])
        rho = np.vdot(g, Hbar[:m, :m] @ g)
        res = Hbar @ g - rho * np.concatenate([g, [0.0]])
        out.append(float(np.linalg.norm(res)))
    return np.array(out)


@dataclass
class DRReport:
    cycles: int = 0
    mvps: int = 0
    relres: float = float("nan")
    nconv: int = 0
    theta: np.ndarray = None
    eigres: np.ndarray = None
    lin_hist: list = field(default_factory=list)


def gmres_dr(op, b, m, k, nev=None, rtolev=1e-8, rtol=1e-8, maxcyc=300,
             transpose=False, x0=None, precond=None, progress=None):
    """GMRES-DR(m,k) on ``A x = b``.  Returns ``(x, W, report)`` where ``W``
    (n x k') is an orthonormal basis of the final k harmonic Ritz vectors
    (k' = k, or k+1 if a conjugate pair straddles position k).

    ``precond`` (a function ``v -> M^{-1} v``): right preconditioning (Sec. 5,
    Example 5): the cycles run on ``A M^{-1}`` from ``u = 0`` (``x0`` must be
    None), the kept vectors are harmonic Ritz vectors of ``A M^{-1}`` and the
    solution is ``x = M^{-1} u``.

    ``progress`` (optional, ``f(cycle, nconv)``) is called after every
    cycle; it sees the counts only and changes nothing."""
    mv0 = (lambda z: operators.apply_transpose(op, z)) if transpose else (lambda z: operators.apply(op, z))
    assert precond is None or x0 is None
    mv = mv0 if precond is None else (lambda z: mv0(precond(z)))
    nev = k if nev is None else nev
    anorm = operators.norm1(op)
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    rep = DRReport()
    bnorm = float(np.linalg.norm(b))
    r = b - mv(x)
    beta = float(np.linalg.norm(r))
    # cycle 1: GMRES(m)
    V, Hbar, j = arnoldi(mv, r, m)
    assert j == m, "invariant subspace found in the first cycle"
    rep.mvps += m
    c = np.zeros(m + 1)
    c[0] = beta
    for cyc in range(1, maxcyc + 1):
        y, *_ = np.linalg.lstsq(Hbar, c, rcond=None)
        x = x + V[:, :m] @ y
        q = c - Hbar @ y
        rep.lin_hist.append(float(np.linalg.norm(q)))
        theta, G = harmonic_ritz(Hbar, m)
        chosen = select_smallest(theta, k)
        ev_idx = chosen[:nev]
        res = eigen_residuals(Hbar, m, theta, G, ev_idx) / anorm
        nconv = int(np.sum(res <= rtolev))
        rep.cycles = cyc
        rep.nconv = nconv
        rep.theta = theta[chosen]
        rep.eigres = eigen_residuals(Hbar, m, theta, G, chosen) / anorm
        done = (np.linalg.norm(q) <= rtol * bnorm) and nconv >= nev
        if progress is not None:
            progress(cyc, nconv)
        # restart (also done after the last cycle to form W)
        Gr = real_basis(theta, G, chosen)
        kk = Gr.shape[1]
        Pk1 = np.zeros((m + 1, kk + 1))
        Pk1[:m, :kk] = Gr
        Pk1[:, kk] = q
        Pk1, R = np.linalg.qr(Pk1)
        Pk1 = Pk1 * np.sign(np.where(np.diag(R) == 0, 1.0, np.diag(R)))
        Vnew = V @ Pk1
        if done or cyc == maxcyc:
            W = Vnew[:, :kk].copy()
            break
        Hnew = np.zeros((m + 1, m))
        Hnew[: kk + 1, :kk] = Pk1.T @ Hbar @ Pk1[:m, :kk]
        cnew = np.zeros(m + 1)
        cnew[: kk + 1] = Pk1.T @ q
        Vn = np.zeros((n, m + 1))
        Vn[:, : kk + 1] = Vnew
        # re-orthogonalise v_{k+1} against v_1..v_k (twice), keep H consistent
        for _ in range(2):
            coef = Vn[:, :kk].T @ Vn[:, kk]
            Vn[:, kk] -= Vn[:, :kk] @ coef
        Vn[:, kk] /= np.linalg.norm(Vn[:, kk])
        V, Hbar, j = arnoldi(mv, Vn[:, kk], m, V_init=Vn, H_init=Hnew, start=kk)
        rep.mvps += m - kk
        c = cnew
    if precond is not None:
        x = precond(x)
    rep.relres = float(np.linalg.norm(b - mv0(x))) / bnorm
    return x, W, rep
