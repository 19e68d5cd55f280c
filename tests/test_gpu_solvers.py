"""GPU parity of the solvers (BiCGStab(ncyc)-Proj(k), GMRES(m)-Proj(k),
GMRES-DR, deflation spaces, FP32 refinement, batching, adjoint) against the
oracle, through the C-ABI."""
import numpy as np
import pytest
import scipy.sparse.linalg as spl
import torch

import workloads as W
from oracle import operators as O, transfer as T, bicgstab as OB, gmres as OG, gmresdr as ODR
from oracle import deflation as OD, adjoint as ADJ

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"


def tg():
    import paper_2005_03070_amd as m
    return m


def _t(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _c1():
    c = W.CONFIGS["C1"]
    oop = O.const_cd(c["n"], c["beta"])
    b = W.rhs(oop.n, c["seed"])
    return c, oop, b


def _direct(oop, b, transpose=False):
    A = O.to_csr(oop).tocsc()
    return spl.spsolve(A.T.tocsc() if transpose else A, b)


def _true_relres(oop, b, x, transpose=False):
    r = b - (O.apply_transpose(oop, x) if transpose else O.apply(oop, x))
    return np.linalg.norm(r) / np.linalg.norm(b)


def test_bicgstab_k0_matches_oracle_scalars_and_solution():
    """Restarted BiCGStab without deflation on the small workload: the first
    iterations' (rho, alpha, omega) agree with the oracle to 1e-12, the solution
    with the direct solve, and the mvp count with the oracle's (soft)."""
    c, oop, b = _c1()
    op = tg().Operator.const_cd(c["n"], c["beta"])
    x, reps = tg().solve(op, _t(b), rtol=1e-10, ncyc=20)
    r = reps[0]
    xo, orep = OB.bicgstab_proj(oop, b, rtol=1e-10, ncyc=20)
    assert r.status == 0
    gs = np.array(r.first_scalars)
    os_ = np.array(orep.first_scalars[: len(gs)])
    assert len(gs) >= 5
    np.testing.assert_allclose(gs[:5], os_[:5], rtol=1e-12)
    xg = x.cpu().numpy()
    assert _true_relres(oop, b, xg) <= 1e-10
    assert abs(r.relres_true - _true_relres(oop, b, xg)) <= 1e-12
    xs = _direct(oop, b)
    assert np.linalg.norm(xg - xs) / np.linalg.norm(xs) <= 1e-7
    assert abs(r.mvp_inner - orep.mvp_inner) <= 0.15 * orep.mvp_inner + 4
    assert r.cycles <= orep.cycles + 3


def _oracle_space(c, oop, b, transpose=False):
    opc = O.coarsen(oop)
    bc = T.restrict(b, oop.dims)
    xc, Wc, drep = ODR.gmres_dr(opc, bc, c["m"], c["k"], nev=c["nev"], rtolev=c["rtolev"], transpose=transpose)
    V, H = OD.deflation_space(oop, Wc, opc.dims, transpose=transpose)
    return opc, xc, Wc, V, H, drep


def test_deflation_space_from_oracle_basis():
    """Stage-wise: the oracle's coarse basis W_c moved and orthonormalised on
    the GPU (prolongation + CholQR2) matches the oracle's unique thin QR, and
    H = V^T A V matches."""
    c, oop, b = _c1()
    opc, xc, Wc, V, H, _ = _oracle_space(c, oop, b)
    op = tg().Operator.const_cd(c["n"], c["beta"])
    cop = op.coarsen()
    cs = tg().defl_from_basis(cop, _t(Wc.T))
    fs = tg().defl_prolongate(cs, op)
    Vg, Hg = fs.basis()
    Vg = Vg.cpu().numpy().T
    assert np.linalg.norm(Vg.T @ Vg - np.eye(Vg.shape[1])) <= 1e-13
    assert np.abs(Vg - V).max() <= 1e-10
    np.testing.assert_allclose(Hg, H, rtol=0, atol=1e-10 * np.abs(H).max())


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_deflated_bicgstab_with_oracle_space(precision):
    """BiCGStab(20)-Proj(10) fed with the oracle's deflation space and initial
    guess: same solution as the direct solve and as the oracle's run."""
    c, oop, b = _c1()
    opc, xc, Wc, V, H, _ = _oracle_space(c, oop, b)
    x0 = T.prolongate(xc, opc.dims)
    op = tg().Operator.const_cd(c["n"], c["beta"])
    space = tg().defl_from_basis(op, _t(V.T))
    x, reps = tg().solve(op, _t(b), x0=_t(x0), defl=space, rtol=1e-10, ncyc=20, precision=precision)
    r = reps[0]
    xo, orep = OB.bicgstab_proj(oop, b, x0=x0, V=V, H=H, rtol=1e-10, ncyc=20, precision=precision)
    xg = x.cpu().numpy()
    assert r.status == 0 and _true_relres(oop, b, xg) <= 1e-10
    xs = _direct(oop, b)
    assert np.linalg.norm(xg - xs) / np.linalg.norm(xs) <= 1e-7
    assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) <= 1e-7
    assert abs(r.mvp_inner - orep.mvp_inner) <= 0.2 * orep.mvp_inner + 6
    if precision == "fp64":
        np.testing.assert_allclose(np.array(r.first_scalars)[:5], np.array(orep.first_scalars)[:5], rtol=1e-10)


def test_coarse_gmres_dr_matches_closed_form_and_oracle_span():
    """GPU GMRES-DR(30,10) on the 31^2 coarse grid: harmonic Ritz values at the
    closed-form eigenvalues, coarse solution accurate, and the span of the
    basis equals the oracle's on the converged pairs."""
    c, oop, b = _c1()
    opc_o = O.coarsen(oop)
    op = tg().Operator.const_cd(c["n"], c["beta"])
    cop = op.coarsen()
    bc = T.restrict(b, oop.dims)
    xc, space, rep = tg().coarse_setup(cop, _t(bc), 30, 10, nev=6, rtolev=1e-10, rtol=1e-10, maxcyc=300)
    assert rep.status == 0 and rep.nconv >= 6 and rep.relres <= 1e-10
    h = 1 / 32
    lx = 2 / h**2 - 2 * np.sqrt(1 / h**4 - 40.0**2 / (4 * h * h)) * np.cos(np.arange(1, 32) * np.pi * h)
    ly = 2 / h**2 - 2 / h**2 * np.cos(np.arange(1, 32) * np.pi * h)
    exact = np.sort((lx[:, None] + ly[None, :]).reshape(-1))[:6]
    np.testing.assert_allclose(np.sort(rep.theta.real)[:6], exact, rtol=2e-6)
    xs = _direct(opc_o, bc)
    assert np.linalg.norm(xc.cpu().numpy() - xs) / np.linalg.norm(xs) <= 1e-8
    Vg, _ = space.basis()
    Vg = Vg.cpu().numpy().T
    xo, Wo, orep = ODR.gmres_dr(opc_o, bc, 30, 10, nev=6, rtolev=1e-10, rtol=1e-10)
    # converged eigenvectors of the oracle's space lie in the GPU space
    AW = O.apply(opc_o, Wo)
    th, G = np.linalg.eig(Wo.T @ AW)
    for i in np.argsort(np.abs(th))[:6]:
        y = Wo @ G[:, i]
        y = y / np.linalg.norm(y)
        assert np.linalg.norm(y - Vg @ (Vg.T @ y)) <= 1e-5


def test_two_grid_pipeline_small_workload():
    """Full GPU pipeline (coarse GMRES-DR, prolongation, BiCGStab(20)-Proj(10))
    on the small workload reaches the direct solution."""
    c, oop, b = _c1()
    op = tg().Operator.const_cd(c["n"], c["beta"])
    solver = tg().TwoGridSolver(op, m=c["m"], k=c["k"], nev=c["nev"], rtolev=c["rtolev"])
    x, reps = solver.solve(_t(b), rtol=1e-10, ncyc=20)
    xg = x.cpu().numpy()
    assert reps[0].status == 0 and _true_relres(oop, b, xg) <= 1e-10
    xs = _direct(oop, b)
    assert np.linalg.norm(xg - xs) / np.linalg.norm(xs) <= 1e-7
    # second right-hand side: no new setup (Sec. 4.1, Example 2)
    b2 = W.rhs(oop.n, 77)
    x2, reps2 = solver.solve(_t(b2), rtol=1e-10, ncyc=20)
    assert reps2[0].status == 0 and _true_relres(oop, b2, x2.cpu().numpy()) <= 1e-10


def test_gmres_proj_matches_oracle():
    c, oop, b = _c1()
    opc, xc, Wc, V, H, _ = _oracle_space(c, oop, b)
    x0 = T.prolongate(xc, opc.dims)
    op = tg().Operator.const_cd(c["n"], c["beta"])
    space = tg().defl_from_basis(op, _t(V.T))
    x, reps = tg().solve(op, _t(b), x0=_t(x0), defl=space, method="gmres", m3=30, rtol=1e-10)
    xo, orep = OG.gmres_proj(oop, b, x0=x0, V=V, H=H, rtol=1e-10, m=30)
    r = reps[0]
    xg = x.cpu().numpy()
    assert r.status == 0 and _true_relres(oop, b, xg) <= 1e-10
    assert r.cycles == orep.cycles
    assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) <= 1e-7


# one cycle runs every basis width p = 1 .. m + 1 through the Gram-Schmidt
# passes: m = 128 covers 1 to 32 columns per wave and the chunked kernel
# beyond 128 columns; n = 1457 is not a multiple of the 64-row blocks
@pytest.mark.parametrize("m", [20, 64, 128])
def test_gmres_first_cycle_equals_oracle_cycle(m):
    """One GMRES(m) cycle (CGS2 on the GPU, MGS2 in the oracle) gives the same
    iterate to rounding."""
    oop = O.const_cd((47, 31), (30.0, 10.0))
    b = W.rhs(oop.n, 12)
    op = tg().Operator.const_cd((47, 31), (30.0, 10.0))
    x, reps = tg().solve(op, _t(b), method="gmres", m3=m, rtol=1e-30, max_extra=1)
    xo, _ = OG.gmres_proj(oop, b, rtol=1e-30, m=m, maxcyc=1)
    assert reps[0].status == 1  # not converged after the single allowed cycle
    assert np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo) <= 1e-10


def test_batched_rhs_independent_of_grouping():
    """Right-hand sides on one deflation space solved in one group: every
    system runs its own state machine with its own reductions, so a column is
    bit-identical whichever group it is solved in, including a group of one
    (which launches the step kernel with its descriptor in the kernel
    arguments instead of the device-side descriptor table)."""
    dims, beta = (127, 127), (100.0, 0.0)
    op = tg().Operator.const_cd(dims, beta)
    oop = O.const_cd(dims, beta)
    n = op.n
    B = np.stack([W.rhs(n, s) for s in (100, 101, 102, 103)])
    Wb = np.stack([W.rhs(n, 500 + i) for i in range(6)])
    space = tg().defl_from_basis(op, _t(Wb))
    for precision in ("fp64", "fp32_ir"):
        X, reps = tg().solve(op, _t(B), defl=space, rtol=1e-9, ncyc=10, precision=precision)
        for pair in ((0, 2), (3, 1)):
            Xp, rp = tg().solve(op, _t(B[list(pair)]), defl=space, rtol=1e-9, ncyc=10, precision=precision)
            for i, j in enumerate(pair):
                assert torch.equal(X[j], Xp[i]), (precision, j)
                assert reps[j].mvp_inner == rp[i].mvp_inner
        for j in range(4):
            xj, rj = tg().solve(op, _t(B[j]), defl=space, rtol=1e-9, ncyc=10, precision=precision)
            assert torch.equal(X[j], xj), (precision, j)
            assert reps[j].mvp_inner == rj[0].mvp_inner
            assert reps[j].status == 0 and reps[j].relres_true <= 1e-9
            assert _true_relres(oop, B[j], X[j].cpu().numpy()) <= 1e-9


def test_instances_bit_identical_to_solo():
    """Uneven instances in one grouped launch: each equals its solo solve."""
    specs = [((63, 63), 10.0, 200), ((95, 41), 60.0, 201), ((31, 127), 120.0, 202)]
    ops = [tg().Operator.const_cd(d, (bx, 0.0)) for d, bx, _ in specs]
    bs = [_t(W.rhs(o.n, s)) for o, (_, _, s) in zip(ops, specs)]
    spaces = [tg().defl_from_basis(o, _t(np.stack([W.rhs(o.n, 900 + i) for i in range(4)]))) for o in ops]
    xs, reps = tg().solve_instances(ops, spaces, bs, rtol=1e-9, ncyc=10)
    for j, o in enumerate(ops):
        xj, rj = tg().solve(o, bs[j], defl=spaces[j], rtol=1e-9, ncyc=10)
        assert torch.equal(xs[j], xj)
        assert reps[j].status == 0
        oop = O.const_cd(specs[j][0], (specs[j][1], 0.0))
        assert _true_relres(oop, bs[j].cpu().numpy(), xj.cpu().numpy()) <= 1e-9


def test_adjoint_gradients_against_oracle():
    """DeflatedSolve backward: dL/db = A^-T (u - u*) and dL/dk from the edge
    formula, both against dense oracle computations."""
    dims, beta = (31, 31), (60.0, 0.0)
    k = W.kfield(dims, 5)
    b = W.rhs(dims[0] * dims[1], 7)
    ustar = W.rhs(dims[0] * dims[1], 6)
    bt = _t(b).requires_grad_(True)
    kt = _t(k).requires_grad_(True)
    cfg = {"m": 20, "k": 6, "rtolev": 1e-6, "solve": {"rtol": 1e-12, "ncyc": 20}}
    u = tg().DeflatedSolve.apply(bt, kt, dims, beta, cfg)
    L = 0.5 * ((u - _t(ustar)) ** 2).sum()
    L.backward()
    oop = O.div_k(dims, k, beta)
    A = O.to_csr(oop).toarray()
    uo = np.linalg.solve(A, b)
    lam = np.linalg.solve(A.T, uo - ustar)
    gk = ADJ.grad_k(lam, uo, dims)
    assert np.linalg.norm(u.detach().cpu().numpy() - uo) / np.linalg.norm(uo) <= 1e-9
    np.testing.assert_allclose(bt.grad.cpu().numpy(), lam, rtol=0, atol=1e-8 * np.abs(lam).max())
    np.testing.assert_allclose(kt.grad.cpu().numpy(), gk, rtol=0, atol=1e-7 * np.abs(gk).max())


def test_breakdown_on_skew_operator():
    """Pure centred convection (skew-symmetric): status breakdown, no hang.
    r^.A r0 vanishes for a skew-symmetric A; with integer right-hand-side
    entries and coefficients (45 = 10 / (2h)) every product and partial sum
    is an exact integer, so sigma is exactly zero in any summation order."""
    dims = (8, 8)
    h = 1 / 9
    n = 64
    coef = np.zeros((5, n))
    coef[1] = -10 / (2 * h)
    coef[2] = 10 / (2 * h)
    assert coef[2, 0] == 45.0
    op = tg().Operator.var_stencil(dims, _t(coef))
    b = np.round(2.0 * W.rhs(n, 3))
    assert np.any(b != 0.0)
    x, reps = tg().solve(op, _t(b), rtol=1e-8, ncyc=5)
    assert reps[0].status == 2


def test_not_converged_keeps_valid_iterate():
    oop = O.const_cd((31, 31), (40.0, 0.0))
    b = W.rhs(oop.n, 8)
    op = tg().Operator.const_cd((31, 31), (40.0, 0.0))
    x, reps = tg().solve(op, _t(b), rtol=1e-12, ncyc=3, max_extra=0, maxit_cycle=5)
    assert reps[0].status == 1 and reps[0].cycles == 3
    rr = _true_relres(oop, b, x.cpu().numpy())
    assert rr < 1.0 and abs(rr - reps[0].relres_true) <= 1e-12


def test_nonfinite_rhs_is_an_error():
    import paper_2005_03070_amd._lib as L
    op = tg().Operator.const_cd((15, 15), (10.0, 0.0))
    b = W.rhs(op.n, 1)
    b[7] = np.nan
    with pytest.raises(L.TgdkError) as ei:
        tg().solve(op, _t(b), rtol=1e-8)
    assert ei.value.code == L.E_NONFINITE


def test_zero_rhs_returns_zero():
    op = tg().Operator.const_cd((15, 15), (10.0, 0.0))
    x, reps = tg().solve(op, torch.zeros(op.n, dtype=torch.float64, device=DEV), rtol=1e-8)
    assert reps[0].status == 0 and reps[0].cycles == 0
    assert torch.count_nonzero(x) == 0


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_headline_size_residual(precision):
    """Headline 1023^2 size (beta = 100) in the benchmark's launch shape,
    without deflation: the true residual recomputed by the oracle meets the
    tolerance, and the reported residual agrees with it."""
    c = W.CONFIGS["C2"]
    oop = O.const_cd(c["n"], c["beta"])
    b = W.rhs(oop.n, c["seed"])
    op = tg().Operator.const_cd(c["n"], c["beta"])
    x, reps = tg().solve(op, _t(b), rtol=1e-8, ncyc=20, precision=precision, max_extra=40)
    rr = _true_relres(oop, b, x.cpu().numpy())
    assert reps[0].status == 0 and rr <= 1e-8
    assert abs(rr - reps[0].relres_true) <= 1e-3 * rr
