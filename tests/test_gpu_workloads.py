"""GPU checks at the full sizes of the workloads (the 1023^2 two-grid
pipeline the benchmark times, the two 511^2 Helmholtz workloads, 3-D 255^3, 32 batched right-hand sides and 16
uneven instances, the 1023^2 adjoint).  The oracle
cannot solve these sizes in seconds, so each check uses properties that hold
at any size: the true residual recomputed by the oracle's operator on the
CPU, agreement with the single-system solves, and directional derivatives."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import operators as O, adjoint as ADJ, transfer as T, multigrid as MG

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"


def tg():
    import paper_2005_03070_amd as m
    return m


def _t(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _relres(oop, b, x, transpose=False):
    r = b - (O.apply_transpose(oop, x) if transpose else O.apply(oop, x))
    return np.linalg.norm(r) / np.linalg.norm(b)


def test_headline_pipeline_full_size():
    """The 1023^2 pipeline in the benchmark's configuration: coarse
    GMRES-DR(80,30) on 511^2, the moved space, BiCGStab(20)-Proj(30) in FP64
    from the prolongated coarse solution.  The prolongated initial guess is
    the oracle's prolongation of the GPU's coarse solution bit for bit; the
    moved V is orthonormal; sampled entries of H = V^T A V equal the oracle
    operator's products; the true residual recomputed by the oracle meets
    1e-8 and matches the reported one."""
    c = W.CONFIGS["C2"]
    oop = O.const_cd(c["n"], c["beta"])
    b = W.rhs(oop.n, c["seed"])
    op = tg().Operator.const_cd(c["n"], c["beta"])
    cop = op.coarsen()
    bt = _t(b)
    xc, cspace, srep = tg().coarse_setup(cop, tg().restrict(op, cop, bt), c["m"], c["k"], c["nev"], c["rtolev"],
                                         1e-8, 300)
    assert srep.nconv >= c["nev"]
    x0 = tg().prolongate(cop, op, xc)
    assert np.array_equal(x0.cpu().numpy(), T.prolongate(xc.cpu().numpy(), cop.dims))
    space = tg().defl_prolongate(cspace, op)
    Vg, Hg = space.basis()
    V = Vg.cpu().numpy().T                      # n x k
    k = V.shape[1]
    assert k >= c["k"]
    assert np.abs(V.T @ V - np.eye(k)).max() <= 1e-12
    for i, j in ((0, 0), (0, k - 1), (k - 1, 0), (k // 2, k // 3), (k - 1, k - 1)):
        hij = float(V[:, i] @ O.apply(oop, V[:, j]))
        assert abs(Hg[i, j] - hij) <= 1e-11 * np.abs(Hg).max()
    x, reps = tg().solve(op, bt, x0=x0, defl=space, rtol=c["rtol"], ncyc=c["ncyc"])
    rr = _relres(oop, b, x.cpu().numpy())
    assert reps[0].status == 0 and rr <= c["rtol"]
    assert abs(rr - reps[0].relres_true) <= 1e-3 * rr


def test_helmholtz_workloads_full_size():
    """The paper's Examples 4 and 5 as printed: -Lap(u) - 100^2 u on 511^2,
    coarse grid 127^2 (two levels).  Example 4: coarse GMRES-DR(200,150)
    until 120 pairs converge, IDR(20)(20)-Proj(150).  Example 5: the
    multigrid on -Lap + 100^2 equals the oracle's V-cycles element by element
    at full size (1e-11); GMRES-DR(150,100) on A_c M_c^-1 until 80 pairs
    converge and the preconditioned IDR(5)(5)-Proj(100).  Both solves: the
    true residual recomputed by the oracle meets 1e-10."""
    for name in ("H1", "H2"):
        c = W.CONFIGS[name]
        oop = O.const_cd(c["n"], c["beta"], sigma=c["sigma"])
        b = W.rhs(oop.n, c["seed"])
        op = tg().Operator.const_cd(c["n"], c["beta"], sigma=c["sigma"])
        grids = [op]
        for _ in range(c["levels"]):
            grids.append(grids[-1].coarsen())
        cop = grids[-1]
        bt = _t(b)
        mg = mgc = None
        if name == "H2":
            shifted = O.const_cd(c["n"], c["beta"], sigma=-c["sigma"])
            mg = tg().Multigrid(tg().Operator.const_cd(c["n"], c["beta"], sigma=-c["sigma"]),
                                cycles=c["mg_cycles"], nu=c["mg_nu"])
            ref = MG.mg_apply(MG.levels(shifted), b, cycles=c["mg_cycles"], nu=c["mg_nu"])
            got = mg.apply(bt).cpu().numpy()
            np.testing.assert_allclose(got, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())
            mgc = tg().Multigrid(tg().Operator.const_cd(cop.dims, c["beta"], sigma=-c["sigma"]),
                                 cycles=c["mg_cycles"], nu=c["mg_nu"])
        bc = bt
        for lv in range(c["levels"]):
            bc = tg().restrict(grids[lv], grids[lv + 1], bc)
        xc, space, srep = tg().coarse_setup(cop, bc, c["m"], c["k"], c["nev"], c["rtolev"], c["rtol"], c["maxcyc"],
                                            precond=mgc)
        assert srep.nconv >= c["nev"], (name, srep.cycles, srep.nconv)
        for lv in range(c["levels"] - 1, -1, -1):
            space = tg().defl_prolongate(space, grids[lv])
            xc = tg().prolongate(grids[lv + 1], grids[lv], xc)
        if mg is not None:
            space = space.precond(mg)
        assert space.k >= c["k"]
        s = c["s"]
        shadow = _t(W.shadow_draw(op.n, s, c["seed"] + s))
        x, rep = tg().solve_idr(op, bt, s=s, shadow=shadow, x0=xc, defl=space, rtol=c["rtol"], ncyc=c["ncyc"],
                                max_extra=20, precond=mg)
        rr = _relres(oop, b, x.cpu().numpy())
        print(f"{name}: GMRES-DR {srep.cycles} cycles, {srep.nconv} converged; IDR({s}) {rep.mvp_inner} mvps, "
              f"{rep.cycles} cycles, relres {rr:.2e}", flush=True)
        assert rep.status == 0 and rr <= c["rtol"], (name, rep.status, rr)


def test_3d_255_fp32_inner_with_fp32_stored_vectors():
    """255^3 (n = 16.6 M), 7-point, coarse 127^3 GMRES-DR, 40 vectors stored in
    float32, FP32 inner cycles with FP64 refinement: true residual <= 1e-8."""
    c = W.CONFIGS["C3"]
    op = tg().Operator.const_cd(c["n"], c["beta"])
    b = W.rhs(op.n, c["seed"])
    solver = tg().TwoGridSolver(op, m=c["m"], k=c["k"], nev=c["nev"], rtolev=c["rtolev"], maxcyc=c["maxcyc"],
                                store=torch.float32)
    x, reps = solver.solve(_t(b), rtol=1e-8, ncyc=20, precision="fp32_ir", max_extra=40)
    r = reps[0]
    assert solver.defl.k >= c["k"] and solver.defl.store == 1
    oop = O.const_cd(c["n"], c["beta"])
    rr = _relres(oop, b, x.cpu().numpy())
    assert r.status == 0 and rr <= 1e-8, (r.status_name, rr)
    assert abs(rr - r.relres_true) <= 1e-3 * rr


def test_batched_32_rhs_511():
    """32 right-hand sides on 511^2 sharing a 30-vector space, FP32 inner
    cycles: each meets the tolerance, and two columns equal their solves in a
    batch of two and alone bit for bit."""
    c = W.CONFIGS["C4"]
    op = tg().Operator.const_cd(c["n"], c["beta"])
    B = W.rhs_block(op.n, c["seeds"]).T.copy()
    solver = tg().TwoGridSolver(op, m=c["m"], k=c["k"], nev=c["nev"], rtolev=c["rtolev"], maxcyc=300)
    solver.setup(_t(B[0]))
    Bt = _t(B)
    X, reps = solver.solve(Bt, rtol=1e-8, ncyc=20, precision="fp32_ir")
    oop = O.const_cd(c["n"], c["beta"])
    Xh = X.cpu().numpy()
    for j in range(32):
        assert reps[j].status == 0
        assert _relres(oop, B[j], Xh[j]) <= 1e-8
    X2, _ = solver.solve(Bt[[0, 17]].contiguous(), rtol=1e-8, ncyc=20, precision="fp32_ir")
    assert torch.equal(X2[0], X[0]) and torch.equal(X2[1], X[17])
    x17, _ = solver.solve(Bt[17].contiguous(), rtol=1e-8, ncyc=20, precision="fp32_ir")
    assert torch.equal(x17, X[17])


def test_sixteen_uneven_instances():
    """16 instances N = 127..511, beta = 10..200, each with its own coarse
    GMRES-DR(80,30) space, solved in grouped launches; each meets the
    tolerance."""
    c = W.CONFIGS["C4"]
    insts = W.uneven_instances()
    ops, spaces, bs, x0s, oops = [], [], [], [], []
    for d in insts:
        N, beta = d["N"], d["beta"]
        op = tg().Operator.const_cd((N, N), (beta, 0.0))
        b = _t(W.rhs(op.n, d["seed"]))
        s = tg().TwoGridSolver(op, m=c["m"], k=c["k"], nev=c["nev"], rtolev=c["rtolev"], maxcyc=300)
        x0s.append(s.setup(b))
        ops.append(op)
        spaces.append(s.defl)
        bs.append(b)
        oops.append(O.const_cd((N, N), (beta, 0.0)))
    assert sum(o.n for o in ops) == 1850696
    xs, reps = tg().solve_instances(ops, spaces, bs, x0s=x0s, rtol=1e-8, ncyc=20, precision="fp32_ir")
    for j in range(16):
        assert reps[j].status == 0
        assert _relres(oops[j], bs[j].cpu().numpy(), xs[j].cpu().numpy()) <= 1e-8


def test_adjoint_1023_directional_derivatives():
    """-div(k grad u) + 60 u_x on 1023^2: the adjoint gradients agree with
    central differences of the loss along random directions in b and in k,
    each perturbed solve reaching 1e-12."""
    c = W.CONFIGS["C5"]
    dims = c["n"]
    n = dims[0] * dims[1]
    k = W.kfield(dims, c["kseed"])
    b = W.rhs(n, c["bseed"])
    ustar = W.rhs(n, c["bstar_seed"]) * 1e-4
    beta = c["beta"]
    cfg = {"m": c["m"], "k": c["k"], "nev": c["nev"], "rtolev": c["rtolev"], "maxcyc": 300,
           "solve": {"rtol": 1e-12, "ncyc": 20, "max_extra": 60}}
    bt = _t(b).requires_grad_(True)
    kt = _t(k).requires_grad_(True)
    u = tg().DeflatedSolve.apply(bt, kt, dims, beta, cfg)
    L = 0.5 * ((u - _t(ustar)) ** 2).sum()
    L.backward()
    gb, gk = bt.grad.cpu().numpy(), kt.grad.cpu().numpy()
    # the gradient kernel against the oracle's formula on the GPU's u and lambda
    op = tg().Operator.div_k(dims, _t(k), beta)
    lam, _ = tg().solve(op, _t(u.detach().cpu().numpy() - ustar), transpose=True, rtol=1e-12, max_extra=200)
    g_or = ADJ.grad_k(lam.cpu().numpy(), u.detach().cpu().numpy(), dims)
    assert np.abs(gk - g_or).max() <= 1e-6 * np.abs(g_or).max()

    def loss(bb, kk):
        opx = tg().Operator.div_k(dims, _t(kk), beta)
        x, r = tg().solve(opx, _t(bb), rtol=1e-12, max_extra=200)
        assert r[0].status == 0
        d = x.cpu().numpy() - ustar
        return 0.5 * float(d @ d)

    rng = np.random.default_rng(c["dir_seed"])
    db = rng.standard_normal(n)
    eps = 1e-3 * np.linalg.norm(b) / np.linalg.norm(db)
    fd = (loss(b + eps * db, k) - loss(b - eps * db, k)) / (2 * eps)
    assert abs(fd - gb @ db) <= 1e-5 * abs(fd)
    dk = rng.standard_normal(k.shape) * k
    epsk = 1e-4
    fdk = (loss(b, k + epsk * dk) - loss(b, k - epsk * dk)) / (2 * epsk)
    assert abs(fdk - (gk * dk).sum()) <= 1e-4 * abs(fdk)
