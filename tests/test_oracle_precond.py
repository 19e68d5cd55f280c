"""Pins of the oracle's right-preconditioned paths (Sec. 5, Example 5:
multigrid on the positively shifted Laplacian preconditions the Helmholtz
operator on both grids): the preconditioned projection leaves V^T r = 0,
preconditioned GMRES-Proj and IDR-Proj reach the direct solution of the
Helmholtz system, the preconditioned coarse GMRES-DR finds eigenvalues of
A M^{-1} (dense eig of the explicitly assembled product) and its solution
solves the original coarse system."""
import numpy as np
import scipy.sparse.linalg as spl

import workloads as W
from oracle import operators as O, multigrid as MG, projection as PR, gmres as OG, idr as OI, gmresdr as GDR
from oracle import deflation as OD, transfer as T

KAPPA = 20.0


def _helmholtz(dims):
    op = O.const_cd(dims, (0.0,) * len(dims), sigma=-KAPPA * KAPPA)
    ops = MG.levels(O.const_cd(dims, (0.0,) * len(dims), sigma=KAPPA * KAPPA))
    return op, (lambda v: MG.mg_apply(ops, v, cycles=2, nu=2))


def test_preconditioned_projection_and_solvers():
    op, pre = _helmholtz((63, 63))
    b = W.rhs(op.n, 91)
    xs = spl.spsolve(O.to_csr(op).tocsc(), b)
    opc = O.coarsen(op)
    w, vr = np.linalg.eig(O.to_csr(opc).toarray())
    Vc = np.real(vr[:, np.argsort(np.abs(w))[:20]])
    V, _ = OD.deflation_space(op, Vc, opc.dims)
    Z, H = PR.precond_space(op, V, pre)
    r = W.rhs(op.n, 92)
    _, r1, _ = PR.precond_projection(op, V, Z, H, np.zeros(op.n), r)
    assert np.abs(V.T @ r1).max() <= 1e-10 * np.linalg.norm(r)
    x1, g = OG.gmres_proj(op, b, V=V, H=H, Z=Z, rtol=1e-10, m=40, precond=pre)
    P = OI.shadow_space(W.shadow_draw(op.n, 4, 93).T)
    x2, i = OI.idrs_proj(op, b, P, V=V, H=H, Z=Z, rtol=1e-10, precond=pre)
    x3, i0 = OI.idrs_proj(op, b, P, rtol=1e-10)
    for x, rep in ((x1, g), (x2, i)):
        assert rep.status == 0 and rep.relres_true <= 1e-10
        assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 1e-7
    assert i.mvp_inner < i0.mvp_inner


def test_preconditioned_gmres_dr_finds_eigenvalues_of_A_Minv():
    op, pre = _helmholtz((31, 31))
    b = W.rhs(op.n, 94)
    x, Wk, rep = GDR.gmres_dr(op, b, m=40, k=12, nev=6, rtolev=1e-8, rtol=1e-10, maxcyc=300, precond=pre)
    assert rep.relres <= 1e-9
    A = O.to_csr(op).toarray()
    Minv = np.stack([pre(np.eye(op.n)[:, j]) for j in range(op.n)], axis=1)
    ev = np.linalg.eigvals(A @ Minv)
    for t in rep.theta[:6]:
        assert np.min(np.abs(ev - t)) <= 1e-6 * np.abs(t)
    # the kept basis spans approximate eigenvectors of A M^{-1}: Ritz values of it agree
    B = Wk.T @ (A @ (Minv @ Wk))
    rv = np.linalg.eigvals(B)
    for t in rep.theta[:6]:
        assert np.min(np.abs(rv - t)) <= 1e-5 * np.abs(t)
