"""Pins of the oracle's IDR(s)(ncyc)-Proj(k) against facts that do not come
from the oracle itself: IDR(1)'s equivalence with BiCGStab (scipy's
implementation), finite termination within n + n/s operator applications,
the biorthogonality invariants of the biorthogonal variant, and direct
solves."""
import numpy as np
import pytest
import scipy.sparse.linalg as spl

import workloads as W
from oracle import operators as O, idr as OI, deflation as OD


def _direct(op, b):
    return spl.spsolve(O.to_csr(op).tocsc(), b)


def test_idr1_equals_bicgstab():
    """IDR(1) with P = r0 / ||r0|| and the minimal-residual omega (kappa = 0)
    is mathematically BiCGStab (shadow vector r0): its residual after every
    dimension reduction equals BiCGStab's after every iteration (scipy's
    Bi-CGSTAB, true residuals of its iterates)."""
    op = O.const_cd((15, 11), (30.0, 10.0))
    b = W.rhs(op.n, 5)
    A = O.to_csr(op)
    P = (b / np.linalg.norm(b))[:, None]
    res = OI.idrs_inner(lambda z: O.apply(op, z), b, 0.0, P, 24, kappa=0.0)
    ref = []
    spl.bicgstab(A, b, rtol=1e-30, atol=0.0, maxiter=12, callback=lambda xk: ref.append(np.linalg.norm(b - A @ xk)))
    k = 8
    np.testing.assert_allclose(res.round_resnorms[:k], ref[:k], rtol=1e-7)


@pytest.mark.parametrize("s", [2, 4, 6])
def test_finite_termination(s):
    """In exact arithmetic IDR(s) finds the solution within n + n/s operator
    applications; on a mildly nonsymmetric 24-unknown system it reaches 1e-10
    within that count (strongly non-normal ones need a few more in floating
    point)."""
    op = O.const_cd((4, 6), (20.0, 10.0))
    b = W.rhs(op.n, 6)
    P = OI.shadow_space(W.shadow_draw(op.n, s, 7).T)
    res = OI.idrs_inner(lambda z: O.apply(op, z), b, 1e-10 * np.linalg.norm(b), P, 200)
    assert res.status == "converged"
    assert res.mvps <= op.n + op.n // s
    x = res.e
    assert np.linalg.norm(b - O.apply(op, x)) <= 1e-9 * np.linalg.norm(b)


def test_biorthogonality_invariants():
    """Before each dimension reduction M = P^T G is lower triangular and
    the residual is orthogonal to all s shadow vectors."""
    op = O.const_cd((31, 31), (40.0, 0.0))
    b = W.rhs(op.n, 8)
    P = OI.shadow_space(W.shadow_draw(op.n, 4, 9).T)
    res = OI.idrs_inner(lambda z: O.apply(op, z), b, 1e-8 * np.linalg.norm(b), P, 400, check=True)
    assert len(res.checks) >= 5
    scale_g = np.linalg.norm(O.apply(op, b))
    scale_r = np.linalg.norm(b)
    for upper, ptr in res.checks:
        assert upper <= 1e-10 * scale_g
        assert ptr <= 1e-10 * scale_r


def test_shadow_space_orthonormal():
    P = OI.shadow_space(W.shadow_draw(500, 4, 3).T)
    np.testing.assert_allclose(P.T @ P, np.eye(4), atol=1e-14)


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_idr_proj_solution_and_deflation(precision):
    """IDR(4)(20)-Proj(8) on the small workload with a deflation space from
    a coarse basis: the direct solve's solution; deflation cuts the inner
    operator applications."""
    c = W.CONFIGS["C1"]
    op = O.const_cd(c["n"], c["beta"])
    b = W.rhs(op.n, c["seed"])
    P = OI.shadow_space(W.shadow_draw(op.n, 4, 11).T)
    opc = O.coarsen(op)
    # a coarse basis of the lowest modes of the coarse operator (dense eig)
    Ac = O.to_csr(opc).toarray()
    w, vr = np.linalg.eig(Ac)
    idx = np.argsort(np.abs(w))[:8]
    Wc = np.real_if_close(vr[:, idx])
    Wc = np.concatenate([Wc.real, Wc.imag[:, np.abs(Wc.imag).max(axis=0) > 0]], axis=1)[:, :8]
    V, H = OD.deflation_space(op, Wc, opc.dims)
    xs = _direct(op, b)
    x0, r0 = OI.idrs_proj(op, b, P, rtol=1e-10, precision=precision)
    x1, r1 = OI.idrs_proj(op, b, P, V=V, H=H, rtol=1e-10, precision=precision)
    for x, r in ((x0, r0), (x1, r1)):
        assert r.status == 0 and r.relres_true <= 1e-10
        assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 1e-7
    assert r1.mvp_inner < r0.mvp_inner


def test_idr_proj_restart_count_and_schedule():
    """ncyc = 1 with k = 0 is plain (non-restarted) IDR(s): one cycle; with
    ncyc = 5 the cycles follow the same rticyc schedule as BiCGStab's."""
    op = O.const_cd((31, 31), (40.0, 0.0))
    b = W.rhs(op.n, 12)
    P = OI.shadow_space(W.shadow_draw(op.n, 4, 13).T)
    x, r = OI.idrs_proj(op, b, P, rtol=1e-9, ncyc=1, max_extra=0)
    assert r.cycles == 1 and r.status == 0
    x5, r5 = OI.idrs_proj(op, b, P, rtol=1e-9, ncyc=5)
    assert r5.status == 0 and 2 <= r5.cycles <= 10
    assert all(bb in (1, 2, 3) for bb in r5.branches)
