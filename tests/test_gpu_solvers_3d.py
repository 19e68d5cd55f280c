"""3-D GPU parity of the fine solve against the oracle: the z-marching phases
A and B, the 3-D cycle boundary (marching true residual with the streamed
c = V^T r pass, w = V d, marching r -= A w), FP32 inner cycles, float32-stored
deflation vectors and variable coefficients.  The grid 47 x 31 x 21 is ragged
in every direction: one partial 64-wide column, a partial last row block and
z chunks with a partial last chunk."""
import numpy as np
import pytest
import scipy.sparse.linalg as spl
import torch

import workloads as W
from oracle import operators as O, bicgstab as OB, deflation as OD

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"
DIMS = (47, 31, 21)
CDIMS = (23, 15, 10)
BETA = (30.0, 10.0, 5.0)


def tg():
    import paper_2005_03070_amd as m
    return m


def _t(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _direct(oop, b):
    return spl.spsolve(O.to_csr(oop).tocsc(), b)


def _relres(oop, b, x):
    return np.linalg.norm(b - O.apply(oop, x)) / np.linalg.norm(b)


def _var_op():
    """Nonsymmetric, diagonally dominant 7-point operator with random
    per-point coefficients (same arrays on both sides)."""
    shape = tuple(reversed(DIMS))
    rng = W.rng(77)
    names = ["C", "W", "E", "S", "N", "D", "U"]
    coef = {k: -1.0 + 0.3 * rng.standard_normal(shape) for k in names[1:]}
    coef["C"] = 6.5 + rng.random(shape)
    oop = O.StencilOp(DIMS, coef, kind="var")
    op = tg().Operator.var_stencil(DIMS, _t(np.stack([coef[k].reshape(-1) for k in names])))
    return oop, op


def _space(oop, k=8, seed=33):
    """Oracle deflation space from a seeded random coarse basis."""
    nc = int(np.prod(CDIMS))
    Wc = W.rng(seed).standard_normal((nc, k))
    return OD.deflation_space(oop, Wc, CDIMS)


def test_3d_k0_scalars_and_solution():
    """No deflation: the first (rho, alpha, omega) agree with the oracle to
    1e-12, the solution with the direct solve."""
    oop = O.const_cd(DIMS, BETA)
    b = W.rhs(oop.n, 31)
    op = tg().Operator.const_cd(DIMS, BETA)
    x, reps = tg().solve(op, _t(b), rtol=1e-10, ncyc=20)
    r = reps[0]
    xo, orep = OB.bicgstab_proj(oop, b, rtol=1e-10, ncyc=20)
    assert r.status == 0
    np.testing.assert_allclose(np.array(r.first_scalars)[:5], np.array(orep.first_scalars)[:5], rtol=1e-12)
    xg = x.cpu().numpy()
    assert _relres(oop, b, xg) <= 1e-10
    assert abs(r.relres_true - _relres(oop, b, xg)) <= 1e-12
    xs = _direct(oop, b)
    assert np.linalg.norm(xg - xs) / np.linalg.norm(xs) <= 1e-7
    assert abs(r.mvp_inner - orep.mvp_inner) <= 0.15 * orep.mvp_inner + 4


@pytest.mark.parametrize("precision,store", [("fp64", torch.float64), ("fp32_ir", torch.float64),
                                             ("fp32_ir", torch.float32)])
def test_3d_deflated_with_oracle_space(precision, store):
    """BiCGStab(20)-Proj(8) with the oracle's deflation space: the solution
    equals the direct solve and the oracle's run; in FP64 with float64 V the
    first scalars agree with the oracle's."""
    oop = O.const_cd(DIMS, BETA)
    b = W.rhs(oop.n, 32)
    V, H = _space(oop)
    op = tg().Operator.const_cd(DIMS, BETA)
    space = tg().defl_from_basis(op, _t(V.T), store=store)
    x, reps = tg().solve(op, _t(b), defl=space, rtol=1e-10, ncyc=20, precision=precision)
    r = reps[0]
    xo, orep = OB.bicgstab_proj(oop, b, V=V, H=H, rtol=1e-10, ncyc=20, precision=precision)
    xg = x.cpu().numpy()
    assert r.status == 0 and _relres(oop, b, xg) <= 1e-10
    xs = _direct(oop, b)
    assert np.linalg.norm(xg - xs) / np.linalg.norm(xs) <= 1e-7
    assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) <= 1e-7
    assert abs(r.mvp_inner - orep.mvp_inner) <= 0.2 * orep.mvp_inner + 6
    assert r.mvp_boundary == orep.mvp_boundary or abs(r.cycles - orep.cycles) <= 2
    if precision == "fp64" and store == torch.float64:
        np.testing.assert_allclose(np.array(r.first_scalars)[:5], np.array(orep.first_scalars)[:5], rtol=1e-10)


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_3d_variable_coefficients_deflated(precision):
    """Per-point coefficient arrays (the run-time coefficient path of the
    marching kernels) with deflation: the solution equals the direct solve."""
    oop, op = _var_op()
    b = W.rhs(oop.n, 34)
    V, H = _space(oop, k=6, seed=35)
    space = tg().defl_from_basis(op, _t(V.T))
    x, reps = tg().solve(op, _t(b), defl=space, rtol=1e-10, ncyc=20, precision=precision)
    xg = x.cpu().numpy()
    assert reps[0].status == 0 and _relres(oop, b, xg) <= 1e-10
    xs = _direct(oop, b)
    assert np.linalg.norm(xg - xs) / np.linalg.norm(xs) <= 1e-7
    xo, orep = OB.bicgstab_proj(oop, b, V=V, H=H, rtol=1e-10, ncyc=20, precision=precision)
    assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) <= 1e-7


def test_3d_batched_and_single_agree():
    """Two right-hand sides on one 3-D space solved together: each column
    is bit-identical to its solve in a group of one."""
    oop = O.const_cd(DIMS, BETA)
    B = np.stack([W.rhs(oop.n, s) for s in (40, 41)])
    V, H = _space(oop)
    op = tg().Operator.const_cd(DIMS, BETA)
    space = tg().defl_from_basis(op, _t(V.T))
    X, reps = tg().solve(op, _t(B), defl=space, rtol=1e-10, ncyc=20, precision="fp32_ir")
    for j in range(2):
        xj, rj = tg().solve(op, _t(B[j]), defl=space, rtol=1e-10, ncyc=20, precision="fp32_ir")
        assert torch.equal(X[j], xj)
        assert reps[j].status == 0 and _relres(oop, B[j], xj.cpu().numpy()) <= 1e-10
