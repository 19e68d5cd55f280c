"""GPU parity of the multigrid preconditioner and the right-preconditioned
solvers (Sec. 5, Example 5: multigrid on the positively shifted Laplacian
preconditions the Helmholtz operator on both grids) against the oracle,
through the C-ABI: V-cycles (2-D and 3-D, several cycle and sweep counts),
the preconditioned deflation space and IDR-Proj (first scalars), GMRES-Proj,
the preconditioned coarse GMRES-DR (eigenvalues of A M^{-1}), the whole
preconditioned two-grid pipeline, and the rejected combinations."""
import numpy as np
import pytest
import scipy.sparse.linalg as spl
import torch

import workloads as W
from oracle import operators as O, multigrid as MG, projection as PR, idr as OI, gmresdr as GDR
from oracle import deflation as OD

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"
KAPPA = 20.0


def tg():
    import paper_2005_03070_amd as m
    return m


def _t(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


# grids whose coarse tail runs in one workgroup from level 1 (63^2, 15^3,
# 31 x 15 x 7 with an odd sweep count), from level 0 (31^2: the whole
# hierarchy; 7^2: every level small enough for the single-wave passes), after
# a non-square fine level (65 x 33 -> 32 x 16, no single-wave levels), and
# not at all (64^2: one level, too large for the tail, 20 sweeps as global
# passes)
@pytest.mark.parametrize("dims,sigma,cycles,nu", [((63, 63), 400.0, 2, 2), ((31, 31), 900.0, 1, 1),
                                                  ((15, 15, 15), 100.0, 3, 2), ((31, 15, 7), 50.0, 2, 3),
                                                  ((65, 33), 400.0, 2, 1), ((64, 64), 300.0, 2, 2),
                                                  ((7, 7), 100.0, 2, 2)])
def test_multigrid_matches_oracle(dims, sigma, cycles, nu):
    oop = O.const_cd(dims, (0.0,) * len(dims), sigma=sigma)
    ops = MG.levels(oop)
    op = tg().Operator.const_cd(dims, (0.0,) * len(dims), sigma=sigma)
    mg = tg().Multigrid(op, cycles=cycles, nu=nu)
    assert mg.levels == len(ops)
    X = np.stack([W.rhs(oop.n, 10 + j) for j in range(2)])
    Y = mg.apply(_t(X)).cpu().numpy()
    for j in range(2):
        ref = MG.mg_apply(ops, X[j], cycles=cycles, nu=nu)
        np.testing.assert_allclose(Y[j], ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())


def _helm(dims):
    oop = O.const_cd(dims, (0.0,) * len(dims), sigma=-KAPPA * KAPPA)
    ops = MG.levels(O.const_cd(dims, (0.0,) * len(dims), sigma=KAPPA * KAPPA))
    op = tg().Operator.const_cd(dims, (0.0,) * len(dims), sigma=-KAPPA * KAPPA)
    mg = tg().Multigrid(tg().Operator.const_cd(dims, (0.0,) * len(dims), sigma=KAPPA * KAPPA), cycles=2, nu=2)
    return oop, (lambda v: MG.mg_apply(ops, v, cycles=2, nu=2)), op, mg


def test_preconditioned_space_and_idr_first_scalars():
    """Oracle V (20 coarse eigenvectors moved), each side forms Z = M^{-1} V
    and H = V^T A Z with its own multigrid: H agrees to 1e-10; IDR(4)-Proj(20)
    on A M^{-1} has the oracle's first scalars to 1e-9 and the direct
    solution; GMRES(40)-Proj(20) too."""
    oop, pre, op, mg = _helm((63, 63))
    b = W.rhs(oop.n, 95)
    xs = spl.spsolve(O.to_csr(oop).tocsc(), b)
    opc = O.coarsen(oop)
    w, vr = np.linalg.eig(O.to_csr(opc).toarray())
    V, _ = OD.deflation_space(oop, np.real(vr[:, np.argsort(np.abs(w))[:20]]), opc.dims)
    Z, H = PR.precond_space(oop, V, pre)
    space = tg().defl_from_basis(op, _t(V.T)).precond(mg)
    _, Hg = space.basis()
    np.testing.assert_allclose(Hg, H, rtol=1e-10, atol=1e-10 * np.abs(H).max())
    draw = W.shadow_draw(oop.n, 4, 96)
    x, r = tg().solve_idr(op, _t(b), s=4, shadow=_t(draw), defl=space, rtol=1e-10, precond=mg)
    xo, orep = OI.idrs_proj(oop, b, OI.shadow_space(draw.T), V=V, H=H, Z=Z, rtol=1e-10, precond=pre)
    assert r.status == 0 and orep.status == 0
    np.testing.assert_allclose(np.array(r.first_scalars)[:, :2], np.array(orep.first_scalars)[:, :2], rtol=1e-9)
    xg = x.cpu().numpy()
    assert np.linalg.norm(xg - xs) / np.linalg.norm(xs) <= 1e-7
    x2, r2 = tg().solve(op, _t(b), defl=space, method="gmres", m3=40, rtol=1e-10, precond=mg)
    assert r2[0].status == 0
    assert np.linalg.norm(x2.cpu().numpy() - xs) / np.linalg.norm(xs) <= 1e-7


def test_preconditioned_two_grid_pipeline():
    """Coarse GMRES-DR(40,12) on A_c M_c^{-1} (multigrid on the coarse grid):
    its kept values match the oracle's preconditioned run (1e-6) and its
    solution solves the coarse system; moved to the fine grid and
    preconditioned there, IDR(4)-Proj reaches the direct solution with fewer
    operator applications than without deflation."""
    oop, pre, op, mg = _helm((63, 63))
    b = _t(W.rhs(oop.n, 97))
    coarse = op.coarsen()
    dims_c = coarse.dims
    oopc, prec, _, _ = _helm(dims_c)
    mgc = tg().Multigrid(tg().Operator.const_cd(dims_c, (0.0, 0.0), sigma=KAPPA * KAPPA), cycles=2, nu=2)
    bc = tg().restrict(op, coarse, b)
    xc, cspace, srep = tg().coarse_setup(coarse, bc, 40, 12, 6, 1e-8, 1e-10, 300, precond=mgc)
    _, _, orep = GDR.gmres_dr(oopc, bc.cpu().numpy(), 40, 12, 6, 1e-8, 1e-10, 300, precond=prec)
    assert srep.relres <= 1e-9
    for t in orep.theta[:6]:
        assert np.min(np.abs(srep.theta - t)) <= 1e-6 * np.abs(t)
    space = tg().defl_prolongate(cspace, op).precond(mg)
    x0 = tg().prolongate(coarse, op, xc)
    draw = _t(W.shadow_draw(oop.n, 4, 98))
    x, r = tg().solve_idr(op, b, s=4, shadow=draw, x0=x0, defl=space, rtol=1e-10, precond=mg)
    xn, rn = tg().solve_idr(op, b, s=4, shadow=draw, x0=x0, rtol=1e-10, precond=mg)
    xs = spl.spsolve(O.to_csr(oop).tocsc(), b.cpu().numpy())
    assert r.status == 0 and np.linalg.norm(x.cpu().numpy() - xs) / np.linalg.norm(xs) <= 1e-7
    assert rn.status == 0 and r.mvp_inner < rn.mvp_inner


def test_rejected_combinations():
    oop, pre, op, mg = _helm((31, 31))
    b = _t(W.rhs(oop.n, 99))
    space = tg().defl_from_basis(op, _t(W.rng(5).standard_normal((4, oop.n))))
    pspace = space.precond(mg)
    err = tg()._lib.TgdkError
    with pytest.raises(err):
        tg().solve(op, b, precond=mg)                      # BiCGStab has no preconditioning
    with pytest.raises(err):
        tg().solve(op, b, defl=pspace, method="gmres")      # preconditioned space, plain solve
    with pytest.raises(err):
        tg().solve(op, b, defl=space, method="gmres", precond=mg)  # plain space, preconditioned solve
    with pytest.raises(err):
        tg().solve_idr(op, b, precond=mg, precision="fp32_ir")
    with pytest.raises(err):
        pspace.minres()
    coef = _t(np.stack([np.full(oop.n, v) for v in (4.0, -1.0, -1.0, -1.0, -1.0)]))
    with pytest.raises(err):
        tg().Multigrid(tg().Operator.var_stencil((31, 31), coef))  # constant coefficients only


def test_multigrid_graph_replays_match_eager():
    """The captured HIP graph, replayed several times with other eager work
    and synchronisations in between, gives the eager kernels' bits every
    time (2-D and 3-D)."""
    for dims, sigma in (((127, 127), 400.0), ((15, 15, 15), 100.0)):
        op = tg().Operator.const_cd(dims, (0.0,) * len(dims), sigma=sigma)
        g = tg().Multigrid(op, cycles=2, nu=2, graph=True)
        e = tg().Multigrid(op, cycles=2, nu=2, graph=False)
        for j in range(4):
            x = _t(W.rhs(op.n, 20 + j))
            yg = g.apply(x)
            torch.cuda.synchronize()
            _ = op.apply(x)
            ye = e.apply(x)
            torch.cuda.synchronize()
            assert torch.equal(yg, ye)
