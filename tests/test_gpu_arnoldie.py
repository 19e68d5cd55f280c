"""GPU parity of the Arnoldi-E(m,k) eigenvector improvement
(tgdk_defl_improve) against closed forms and the oracle (oracle/arnoldie.py),
through the C-ABI: converged values of symmetric, nonsymmetric and transposed
operators, complex conjugate pairs against dense eigenvalues, and the
two-grid workflow's phase 2 (moved coarse vectors improved on the fine grid
make the deflated solve cheaper)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import operators as O, arnoldie as AE

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"


def tg():
    import paper_2005_03070_amd as m
    return m


def _t(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


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
    (lx, rx, ux), (ly, ry, uy) = _tri(dims[0], beta[0]), _tri(dims[1], beta[1])
    pairs = sorted(((lx[a] + ly[b_], a, b_) for a in range(dims[0]) for b_ in range(dims[1])))[:count]
    lam = np.array([p[0] for p in pairs])
    vecs = np.stack([np.kron(ry[:, b_], rx[:, a]) for _, a, b_ in pairs], axis=1)
    lefts = np.stack([np.kron(uy[:, b_], ux[:, a]) for _, a, b_ in pairs], axis=1)
    kappa = np.linalg.norm(vecs, axis=0) * np.linalg.norm(lefts, axis=0) / np.abs(np.sum(vecs * lefts, axis=0))
    return lam, vecs / np.linalg.norm(vecs, axis=0), kappa


def _perturbed(vecs, seed):
    noise = W.rng(seed).standard_normal(vecs.shape)
    return vecs + 1e-2 * noise / np.linalg.norm(noise, axis=0)


@pytest.mark.parametrize("beta", [(0.0, 0.0), (20.0, 10.0)])
def test_improve_converges_to_closed_form(beta):
    """Arnoldi-E(24,8) from perturbed eigenvectors: the 6 leading values are
    the closed forms (1e-11 symmetric; within 10 kappa ||r|| otherwise); the
    oracle takes the same number of cycles (within one); the improved space
    holds the eigenvectors."""
    dims = (31, 27)
    oop = O.const_cd(dims, beta)
    lam, vecs, kappa = _closed_form(dims, beta, 8)
    Y0 = _perturbed(vecs, 1)
    op = tg().Operator.const_cd(dims, beta)
    space = tg().defl_from_basis(op, _t(Y0.T))
    imp, rep = space.improve(m=24, nev=6, tol=1e-11, maxcyc=300)
    _, orep = AE.arnoldi_e(oop, Y0, m=24, nev=6, tol=1e-11, maxcyc=300)
    assert rep["cycles"] >= 1 and abs(rep["cycles"] - orep.cycles) <= 1
    assert rep["nconv"] == 6 and np.all(rep["eigres"][:6] <= 1e-11)
    np.testing.assert_allclose(rep["eigres_start"], orep.eigres_start, rtol=1e-8)
    order = np.argsort(rep["theta"][:6].real)
    got = rep["theta"][:6][order].real
    if beta == (0.0, 0.0):
        np.testing.assert_allclose(got, lam[:6], rtol=1e-11)
    else:
        bound = 10 * kappa[:6] * rep["eigres"][:6][order] * O.norm1(oop)
        assert np.all(np.abs(got - lam[:6]) <= bound)
    V, H = imp.basis()
    V = V.cpu().numpy().T
    np.testing.assert_allclose(V.T @ V, np.eye(V.shape[1]), atol=1e-12)
    for c in range(6):
        assert np.linalg.norm(vecs[:, c] - V @ (V.T @ vecs[:, c])) <= 1e-6


def test_improve_transpose_and_complex_pairs():
    """A^T space: the leading values match A's closed forms within the kappa
    bound.  Strong convection: complex conjugate pairs match dense numpy
    eigenvalues of smallest modulus."""
    dims, beta = (25, 21), (30.0, 10.0)
    oop = O.const_cd(dims, beta)
    lam, _, kappa = _closed_form(dims, beta, 6)
    op = tg().Operator.const_cd(dims, beta)
    space = tg().defl_from_basis(op, _t(W.rng(2).standard_normal((6, oop.n))), transpose=True)
    imp, rep = space.improve(m=40, nev=4, tol=1e-9, maxcyc=400)
    assert np.all(rep["eigres"][:4] <= 1e-9)
    anorm_t = float(abs(O.to_csr(oop)).sum(axis=1).max())
    order = np.argsort(rep["theta"][:4].real)
    bound = 10 * kappa[:4] * rep["eigres"][:4][order] * anorm_t
    assert np.all(np.abs(rep["theta"][:4][order].real - lam[:4]) <= bound)
    dims, beta = (15, 13), (90.0, 0.0)
    oop = O.const_cd(dims, beta)
    w = np.linalg.eigvals(O.to_csr(oop).toarray())
    ref = w[np.argsort(np.abs(w))]
    assert np.abs(ref[:6].imag).max() > 1.0
    op = tg().Operator.const_cd(dims, beta)
    space = tg().defl_from_basis(op, _t(W.rng(3).standard_normal((8, oop.n))))
    imp, rep = space.improve(m=40, nev=6, tol=1e-10, maxcyc=400)
    assert np.all(rep["eigres"][:6] <= 1e-10)
    for z in rep["theta"][:6]:
        assert np.min(np.abs(ref[:8] - z)) <= 1e-8 * np.abs(ref[0])
    assert np.abs(rep["theta"][:6].imag).max() > 1.0


def test_phase2_improvement_makes_the_deflated_solve_cheaper():
    """Two-grid workflow on the small workload: coarse GMRES-DR(30,10) on the
    GPU, vectors moved to the fine grid, Arnoldi-E(30,10) until the 8
    leading pairs are below 1e-8; BiCGStab(20)-Proj(10) then needs fewer
    inner operator applications than with the unimproved space, and reaches
    the same solution."""
    c = W.CONFIGS["C1"]
    op = tg().Operator.const_cd(c["n"], c["beta"])
    b = _t(W.rhs(op.n, c["seed"]))
    coarse = op.coarsen()
    xc, cspace, _ = tg().coarse_setup(coarse, tg().restrict(op, coarse, b), c["m"], c["k"], c["nev"],
                                      c["rtolev"], 1e-8, 300)
    space = tg().defl_prolongate(cspace, op)
    x0 = tg().prolongate(coarse, op, xc)
    imp, rep = space.improve(m=30, nev=8, tol=1e-8, maxcyc=100)
    assert rep["eigres_start"].max() > 1e-6 and rep["cycles"] >= 1
    assert np.all(rep["eigres"][:8] <= 1e-8)
    x1, r1 = tg().solve(op, b, x0=x0, defl=space, rtol=1e-10)
    x2, r2 = tg().solve(op, b, x0=x0, defl=imp, rtol=1e-10)
    assert r1[0].status == 0 and r2[0].status == 0
    assert r2[0].mvp_inner < r1[0].mvp_inner
    assert float(torch.linalg.vector_norm(x1 - x2) / torch.linalg.vector_norm(x1)) <= 1e-8


def test_improve_argument_errors():
    op = tg().Operator.const_cd((15, 13), (5.0, 0.0))
    space = tg().defl_from_basis(op, _t(W.rng(4).standard_normal((5, op.n))))
    for kw in (dict(m=5), dict(m=257), dict(m=20, nev=6), dict(m=20, tol=0.0), dict(m=20, maxcyc=-1)):
        with pytest.raises(tg()._lib.TgdkError):
            space.improve(**kw)
