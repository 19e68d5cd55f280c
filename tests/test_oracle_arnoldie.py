"""Pins of the oracle's Arnoldi-E eigenvector improvement against facts
outside the oracle: closed-form eigenvalues of the convection-diffusion
operator, exact eigenvectors (no cycle needed), dense numpy eigenvalues for an
operator with complex conjugate pairs, and the improvement of moved
coarse-grid vectors."""
import numpy as np
import pytest

import workloads as W
from oracle import operators as O, arnoldie as AE, gmresdr as GDR, deflation as OD, transfer as T


def _tri(n, beta):
    h = 1.0 / (n + 1)
    w, e = -1 / h**2 - beta / (2 * h), -1 / h**2 + beta / (2 * h)
    j = np.arange(1, n + 1)
    lam = 2.0 / h**2 - 2.0 * np.sqrt(w * e) * np.cos(j * np.pi * h)
    i = np.arange(1, n + 1)[:, None]
    right = np.sqrt(w / e) ** i * np.sin(i * j[None, :] * np.pi * h)
    left = np.sqrt(w / e) ** (-i) * np.sin(i * j[None, :] * np.pi * h)
    return lam, right, left


def _closed_form(dims, beta, count):
    """The `count` smallest eigenvalues, right eigenvectors (unit) and the
    eigenvalue condition numbers ||u|| ||v|| / |u^T v| (2-D)."""
    (lx, rx, ux), (ly, ry, uy) = _tri(dims[0], beta[0]), _tri(dims[1], beta[1])
    pairs = sorted(((lx[a] + ly[b_], a, b_) for a in range(dims[0]) for b_ in range(dims[1])))[:count]
    lam = np.array([p[0] for p in pairs])
    vecs = np.stack([np.kron(ry[:, b_], rx[:, a]) for _, a, b_ in pairs], axis=1)
    lefts = np.stack([np.kron(uy[:, b_], ux[:, a]) for _, a, b_ in pairs], axis=1)
    kappa = np.linalg.norm(vecs, axis=0) * np.linalg.norm(lefts, axis=0) / np.abs(np.sum(vecs * lefts, axis=0))
    return lam, vecs / np.linalg.norm(vecs, axis=0), kappa


@pytest.mark.parametrize("beta", [(0.0, 0.0), (20.0, 10.0)])
def test_converges_to_closed_form_eigenvalues(beta):
    """From perturbed eigenvectors (1e-2 noise) of the 8 smallest
    eigenvalues, Arnoldi-E(24,8) brings the 6 leading pairs below residual
    norm 1e-11; their values are the closed-form eigenvalues: to 1e-11 for
    the symmetric operator, within 10 kappa(lambda) ||r|| for the
    nonsymmetric one (kappa from the closed-form left and right vectors)."""
    dims = (31, 27)
    op = O.const_cd(dims, beta)
    anorm = O.norm1(op)
    lam, vecs, kappa = _closed_form(dims, beta, 8)
    noise = W.rng(1).standard_normal(vecs.shape)
    Y0 = vecs + 1e-2 * noise / np.linalg.norm(noise, axis=0)
    V, rep = AE.arnoldi_e(op, Y0, m=24, nev=6, tol=1e-11, maxcyc=300)
    assert rep.eigres_start.max() > 1e-4
    assert rep.cycles >= 1 and np.all(rep.eigres[:6] <= 1e-11)
    order = np.argsort(rep.theta[:6].real)
    got = rep.theta[:6][order]
    assert np.abs(got.imag).max() <= 1e-8 * lam[0]
    if beta == (0.0, 0.0):
        np.testing.assert_allclose(got.real, lam[:6], rtol=1e-11)
    else:
        bound = 10 * kappa[:6] * rep.eigres[:6][order] * anorm
        assert np.all(np.abs(got.real - lam[:6]) <= bound)
    np.testing.assert_allclose(V.T @ V, np.eye(V.shape[1]), atol=1e-12)
    # the span holds the eigenvectors
    for c in range(6):
        v = vecs[:, c]
        assert np.linalg.norm(v - V @ (V.T @ v)) <= 1e-6


def test_exact_eigenvectors_need_no_cycle():
    dims, beta = (21, 19), (15.0, -5.0)
    op = O.const_cd(dims, beta)
    lam, vecs, kappa = _closed_form(dims, beta, 5)
    V, rep = AE.arnoldi_e(op, vecs, m=15, nev=5, tol=1e-10)
    assert rep.cycles == 0 and rep.mvps == 5
    np.testing.assert_allclose(np.sort(rep.theta.real), lam, rtol=1e-12 * kappa.max())


def test_transpose_reaches_the_same_eigenvalues():
    """A^T has A's eigenvalues: from random vectors the 4 leading Ritz values
    of A^T match the closed forms within 10 kappa(lambda) ||r||."""
    dims, beta = (25, 21), (30.0, 10.0)
    op = O.const_cd(dims, beta)
    lam, _, kappa = _closed_form(dims, beta, 6)
    Y0 = W.rng(2).standard_normal((op.n, 6))
    V, rep = AE.arnoldi_e(op, Y0, m=40, nev=4, tol=1e-9, maxcyc=400, transpose=True)
    assert np.all(rep.eigres[:4] <= 1e-9)
    anorm_t = float(abs(O.to_csr(op)).sum(axis=1).max())
    order = np.argsort(rep.theta[:4].real)
    bound = 10 * kappa[:4] * rep.eigres[:4][order] * anorm_t
    assert np.all(np.abs(rep.theta[:4][order].real - lam[:4]) <= bound)


def test_complex_pairs_against_dense_eigenvalues():
    """Strong convection (cell Peclet number above 1) gives complex
    conjugate eigenvalues: the nev leading ones (a pair kept whole) match
    numpy's dense eigenvalues of smallest modulus."""
    dims, beta = (15, 13), (90.0, 0.0)
    op = O.const_cd(dims, beta)
    w = np.linalg.eigvals(O.to_csr(op).toarray())
    ref = w[np.argsort(np.abs(w))]
    assert np.abs(ref[:6].imag).max() > 1.0
    Y0 = W.rng(3).standard_normal((op.n, 8))
    V, rep = AE.arnoldi_e(op, Y0, m=40, nev=6, tol=1e-10, maxcyc=400)
    assert np.all(rep.eigres[:6] <= 1e-10)
    got = rep.theta[:6]
    for z in got:
        assert np.min(np.abs(ref[:8] - z)) <= 1e-8 * np.abs(ref[0])
    assert np.abs(np.sort(np.abs(got)) - np.sort(np.abs(ref[:6]))).max() <= 1e-8 * np.abs(ref[5])


def test_improves_moved_coarse_vectors():
    """The workflow's phase 2: coarse GMRES-DR vectors of the small workload
    moved to the fine grid have residual norms above 1e-6; Arnoldi-E(30,10)
    brings the 8 leading ones below 1e-8, counting one operator application
    per basis vector per cycle."""
    c = W.CONFIGS["C1"]
    op = O.const_cd(c["n"], c["beta"])
    opc = O.coarsen(op)
    b = W.rhs(op.n, c["seed"])
    _, Wc, _ = GDR.gmres_dr(opc, T.restrict(b, op.dims), c["m"], c["k"], c["nev"], c["rtolev"], 1e-8, 300)
    V0, _ = OD.deflation_space(op, Wc, opc.dims)
    V, rep = AE.arnoldi_e(op, V0, m=30, nev=8, tol=1e-8, maxcyc=100)
    assert rep.eigres_start.max() > 1e-6
    assert rep.cycles >= 1 and np.all(rep.eigres[:8] <= 1e-8)
    assert rep.res_hist[-1] <= 1e-8
    assert rep.mvps >= V0.shape[1] + rep.cycles * (30 - V0.shape[1])
