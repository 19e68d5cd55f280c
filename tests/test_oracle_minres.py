"""Pins of the oracle's MinRes projection (the variant the paper notes after
the Sec. 2.2 box) and of variable GMRES cycle lengths (Sec. 4.3, Table 4.3),
against facts outside the oracle: numpy's SVD least-squares solution, the
orthogonality of the residual to AV, invariance under a change of basis of
span(V), an explicitly transposed CSR operator, closed forms and direct
solves."""
import numpy as np
import scipy.sparse.linalg as spl

import workloads as W
from oracle import operators as O, projection as PR, deflation as OD, bicgstab as OB, gmres as OG, idr as OI


def _space(oop, cdims, k, seed):
    Wc = W.rng(seed).standard_normal((int(np.prod(cdims)), k))
    return OD.deflation_space(oop, Wc, cdims)


def test_minres_projection_is_least_squares():
    """d minimises ||r - A V d||: equal to numpy's SVD least squares; the new
    residual is orthogonal to AV and no longer than r or than Galerkin's."""
    oop = O.const_cd((31, 23), (30.0, 10.0))
    V, H = _space(oop, (15, 11), 7, 3)
    x = W.rhs(oop.n, 4)
    r = W.rhs(oop.n, 5)
    AV = O.to_csr(oop) @ V
    d_ls, *_ = np.linalg.lstsq(AV, r, rcond=None)
    x1, r1, d = PR.minres_projection(oop, V, x, r)
    np.testing.assert_allclose(d, d_ls, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(r1, r - AV @ d_ls, rtol=1e-9, atol=1e-12 * np.linalg.norm(r))
    np.testing.assert_allclose(x1, x + V @ d_ls, rtol=1e-12)
    assert np.abs(AV.T @ r1).max() <= 1e-10 * np.linalg.norm(AV) * np.linalg.norm(r)
    xg, rg, _ = PR.galerkin(oop, V, H, x, r)
    assert np.linalg.norm(r1) <= np.linalg.norm(r) and np.linalg.norm(r1) <= np.linalg.norm(rg) * (1 + 1e-12)


def test_minres_invariant_under_change_of_basis():
    oop = O.const_cd((19, 17), (10.0, 20.0))
    V, _ = _space(oop, (9, 8), 5, 6)
    M = W.rng(7).standard_normal((5, 5)) + 3 * np.eye(5)
    x, r = np.zeros(oop.n), W.rhs(oop.n, 8)
    x1, r1, _ = PR.minres_projection(oop, V, x, r)
    x2, r2, _ = PR.minres_projection(oop, V @ M, x, r)
    np.testing.assert_allclose(x2, x1, rtol=1e-9, atol=1e-13)
    np.testing.assert_allclose(r2, r1, rtol=1e-9, atol=1e-12)


def test_minres_transpose_against_explicit_transpose():
    oop = O.const_cd((21, 13), (40.0, -15.0))
    V, _ = _space(oop, (10, 6), 6, 9)
    r = W.rhs(oop.n, 10)
    ATV = O.to_csr(oop).T @ V
    d_ls, *_ = np.linalg.lstsq(ATV, r, rcond=None)
    _, r1, d = PR.minres_projection(oop, V, np.zeros(oop.n), r, transpose=True)
    np.testing.assert_allclose(d, d_ls, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(r1, r - ATV @ d_ls, rtol=1e-9, atol=1e-12 * np.linalg.norm(r))


def test_galerkin_can_grow_the_residual_minres_cannot():
    """On an indefinite Helmholtz operator with a random space, the Galerkin
    projection can lengthen the residual (H = V^T A V nearly singular); the
    MinRes projection never does."""
    oop = O.const_cd((31, 31), (0.0, 0.0), sigma=-400.0)
    grew = 0
    for seed in range(20):
        V, H = _space(oop, (15, 15), 6, 100 + seed)
        r = W.rhs(oop.n, 200 + seed)
        _, rg, _ = PR.galerkin(oop, V, H, np.zeros(oop.n), r)
        _, rm, _ = PR.minres_projection(oop, V, np.zeros(oop.n), r)
        assert np.linalg.norm(rm) <= np.linalg.norm(r)
        grew += np.linalg.norm(rg) > np.linalg.norm(r)
    assert grew >= 1


def test_solvers_with_minres_projection_reach_the_direct_solution():
    c = W.CONFIGS["C1"]
    oop = O.const_cd(c["n"], c["beta"])
    b = W.rhs(oop.n, c["seed"])
    V, H = _space(oop, (31, 31), 10, 11)
    xs = spl.spsolve(O.to_csr(oop).tocsc(), b)
    P = OI.shadow_space(W.shadow_draw(oop.n, 4, 12).T)
    runs = [OB.bicgstab_proj(oop, b, V=V, H=H, rtol=1e-10, projection="minres"),
            OG.gmres_proj(oop, b, V=V, H=H, rtol=1e-10, m=30, projection="minres"),
            OI.idrs_proj(oop, b, P, V=V, H=H, rtol=1e-10, projection="minres")]
    for x, rep in runs:
        assert rep.status == 0 and rep.relres_true <= 1e-10
        assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 1e-7


def test_gmres_variable_cycle_lengths():
    """Equal lengths reproduce GMRES(m); a one-step cycle is the closed-form
    minimal residual step along A r; the inner mvps are the sum of the cycle
    lengths used."""
    c = W.CONFIGS["C1"]
    oop = O.const_cd(c["n"], c["beta"])
    b = W.rhs(oop.n, c["seed"])
    x1, r1 = OG.gmres_proj(oop, b, rtol=1e-9, m=20)
    x2, r2 = OG.gmres_proj(oop, b, rtol=1e-9, m=20, lengths=[20] * 500)
    np.testing.assert_array_equal(x1, x2)
    assert r1.mvp_inner == r2.mvp_inner
    # one cycle of length 1 from x = 0: x = (r.Ar / ||Ar||^2) r
    x, rep = OG.gmres_proj(oop, b, rtol=1e-30, m=20, lengths=[1], maxcyc=1)
    Ab = O.apply(oop, b)
    np.testing.assert_allclose(x, (b @ Ab) / (Ab @ Ab) * b, rtol=1e-10)
    lengths = [int(v) for v in W.rng(13).integers(1, 41, size=300)]
    x, rep = OG.gmres_proj(oop, b, rtol=1e-9, m=40, lengths=lengths, maxcyc=300)
    assert rep.status == 0 and rep.relres_true <= 1e-9
    assert rep.mvp_inner == sum(lengths[:rep.cycles])
