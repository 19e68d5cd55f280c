"""Arnoldi-E(m,k): improvement of approximate eigenvectors on the fine grid
(step 2 of the Two-grid Deflated GMRES and BiCGStab boxes, Sec. 3 and 4.1;
Sec. 2.3).  Test infrastructure only.

The paper names Arnoldi-E as a restarted Arnoldi method that can start from
given approximate eigenvectors, and runs it optionally on the fine grid to
improve the vectors moved from the coarse grid (Sec. 5, Table 5.1: 10 cycles of
Arnoldi-E(150,100), or cycles until the first 80 vectors have residual norms
below 1e-3).  Its steps are not printed there; the reading used here (the same
on the GPU) is:

* Rayleigh-Ritz on the current subspace gives approximate eigenpairs
  ``(theta_i, y_i)``, ordered and kept as GMRES-DR keeps its harmonic Ritz
  values (smallest ``|theta|`` first, a conjugate pair kept whole); the
  residual norm of a pair is ``||A y - theta y|| / ||A||_1`` with ``||y|| = 1``.
* A cycle starts a Krylov subspace from the first of the ``nev`` leading
  approximate eigenvectors whose residual norm exceeds ``tol`` (its real part,
  normalised), runs ``m - k`` Arnoldi steps from it, appends a real basis of the
  ``k`` kept vectors orthonormalised against the Krylov basis (two classical
  Gram-Schmidt passes; a vector that loses all but 1e-8 of its norm is
  dropped, which drops the start vector itself), and applies Rayleigh-Ritz
  on the whole subspace: the ``k`` leading pairs are kept.
* Each basis vector of a cycle is multiplied by A once (the operator
  applications counted per cycle equal the subspace dimension).
* The improvement stops when the ``nev`` leading pairs have residual norm
  ``<= tol``, or after ``maxcyc`` cycles.  The result is an orthonormal basis
  of the span of the kept vectors (only the span matters for the projection).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import operators
from .gmres import arnoldi
from .gmresdr import real_basis, select_smallest


@dataclass
class ArnoldiEReport:
    cycles: int = 0
    mvps: int = 0
    nconv: int = 0
    theta: np.ndarray = None      # kept Ritz values, in keeping order
    eigres: np.ndarray = None     # their residual norms (relative to ||A||_1)
    eigres_start: np.ndarray = None
    res_hist: list = field(default_factory=list)   # max residual of the nev leading pairs per cycle


def _orthonormal(Z):
    Q, R = np.linalg.qr(Z)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s


def _rayleigh_ritz(Q, W, k, anorm):
    """Ritz pairs of A on range(Q) (orthonormal Q, W = A Q): the k kept ones
    (indices in keeping order), their residual norms, and the coefficient
    vectors."""
    B = Q.T @ W
    theta, G = np.linalg.eig(B)
    chosen = select_smallest(theta, k)
    res = []
    for i in chosen:
        g = G[:, i] / np.linalg.norm(G[:, i])
        r = W @ g - theta[i] * (Q @ g)
        res.append(float(np.linalg.norm(r)) / anorm)
    return theta, G, chosen, np.array(res)


def arnoldi_e(op, Y0, m, nev=None, tol=1e-8, maxcyc=100, transpose=False):
    """Improve the approximate eigenvectors spanning ``Y0`` (n x k) of ``A``
    (``A^T`` if ``transpose``).  Returns ``(V, ArnoldiEReport)`` with ``V``
    an orthonormal n x k' basis of the improved span."""
    mv = (lambda z: operators.apply_transpose(op, z)) if transpose else (lambda z: operators.apply(op, z))
    # ||M||_1 of the operator applied (for A^T: the largest absolute row sum of A)
    anorm = float(abs(operators.to_csr(op)).sum(axis=1 if transpose else 0).max())
    Y = _orthonormal(np.asarray(Y0, dtype=np.float64))
    k = Y.shape[1]
    nev = k if nev is None else min(nev, k)
    p = m - k
    assert p >= 1, "m must exceed k"
    rep = ArnoldiEReport()
    W = mv(Y)
    rep.mvps += k
    theta, G, chosen, res = _rayleigh_ritz(Y, W, k, anorm)
    rep.eigres_start = res[:nev].copy()
    Q = Y
    for cyc in range(maxcyc + 1):
        lead = res[:nev]
        rep.theta = theta[chosen]
        rep.eigres = res
        rep.nconv = int(np.sum(lead <= tol))
        if np.all(lead <= tol) or cyc == maxcyc:
            break
        rep.cycles = cyc + 1
        # start vector: the first leading pair that has not converged
        s = chosen[int(np.argmax(lead > tol))]
        start = (Q @ G[:, s]).real
        if np.linalg.norm(start) <= 1e-8 * np.linalg.norm(Q @ G[:, s]):
            start = (Q @ G[:, s]).imag
        # Krylov part: p Arnoldi steps from the start vector
        K, _, j = arnoldi(mv, start, p)
        K = K[:, : j + 1]
        K = K[:, np.linalg.norm(K, axis=0) > 0]   # an invariant subspace ends the basis early
        # the kept vectors (real basis), orthonormalised against K and each other
        Z = Q @ real_basis(theta, G, chosen)
        cols = [K]
        for c in range(Z.shape[1]):
            z = Z[:, c].copy()
            z0 = np.linalg.norm(z)
            Qc = np.concatenate(cols, axis=1)
            for _ in range(2):
                z -= Qc @ (Qc.T @ z)
            nz = np.linalg.norm(z)
            if nz > 1e-8 * z0:
                cols.append((z / nz)[:, None])
        Q = np.concatenate(cols, axis=1)
        W = mv(Q)
        rep.mvps += Q.shape[1]
        theta, G, chosen, res = _rayleigh_ritz(Q, W, k, anorm)
        rep.res_hist.append(float(res[:nev].max()))
    V = _orthonormal(Q @ real_basis(theta, G, chosen))
    return V, rep


__all__ = ["arnoldi_e", "ArnoldiEReport"]
