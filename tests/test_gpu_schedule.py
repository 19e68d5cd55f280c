"""The cycle schedule of the Sec. 4.1 box on the GPU: the criterion that sets
each cycle's tolerance (step 3 b) against the oracle's, with criterion 2
forced; resuming a solve at a cycle boundary (icyc0, nu0); a rank-deficient
moved basis."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import operators as O, bicgstab as OB, idr as OI, deflation as OD, projection as OP

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"


def tg():
    import paper_2005_03070_amd as m
    return m


def _t(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _decided(cycle_nu, margin=1e-9):
    """Indices of the cycles whose two criteria differ by more than `margin`
    (relative): there the branch does not depend on rounding.  The last
    scheduled cycle is an exact tie in real arithmetic (both give tau/nu)."""
    out = []
    for i, (nu, nu0, tau, icyc, ncyc) in enumerate(cycle_nu):
        if icyc > ncyc:
            out.append(i)
            continue
        t1 = (tau / nu) ** (1.0 / (ncyc - icyc + 1))
        t2 = (nu0 / nu) * (tau / nu0) ** (icyc / ncyc)
        if abs(t1 - t2) > margin * max(t1, t2):
            out.append(i)
    return out


def _space(oop, k, seed):
    """A seeded random orthonormal basis: a poor deflation space."""
    Wb = W.rng(seed).standard_normal((oop.n, k))
    V = OD.orthonormalize(Wb)
    return Wb, V, OP.projection_matrix(oop, V)


CASES = [((63, 63), (40.0, 0.0), 0, 3), ((63, 63), (40.0, 0.0), 4, 3), ((63, 63), (40.0, 0.0), 4, 5),
         ((47, 31, 21), (50.0, 20.0, 10.0), 4, 3)]


@pytest.mark.parametrize("dims,beta,k,maxit", CASES)
def test_bicgstab_branches_match_oracle_with_criterion_2_forced(dims, beta, k, maxit):
    """Cycles capped at `maxit` inner iterations end above their targets, so
    later cycles start above the geometric schedule and criterion 2 sets
    their tolerance.  The per-cycle criteria (the report's cycle_branch)
    equal the oracle's on every cycle where the two criteria are not a
    rounding-level tie; at least five criterion-2 cycles are compared."""
    oop = O.const_cd(dims, beta)
    b = W.rhs(oop.n, 3)
    op = tg().Operator.const_cd(dims, beta)
    V = H = None
    space = None
    if k:
        Wb, V, H = _space(oop, k, 103)
        space = tg().defl_from_basis(op, _t(Wb.T))
    kw = dict(rtol=1e-8, ncyc=10, maxit_cycle=maxit, max_extra=0)
    xo, orep = OB.bicgstab_proj(oop, b, V=V, H=H, **kw)
    x, reps = tg().solve(op, _t(b), defl=space, **kw)
    r = reps[0]
    assert r.status == orep.status == 1 and r.cycles == orep.cycles == 10
    got = r.cycle_branch[:r.cycles]
    want = orep.branches
    idx = _decided(orep.cycle_nu)
    assert sum(1 for i in idx if want[i] == 2) >= 5
    assert [got[i] for i in idx] == [want[i] for i in idx], (got, want)
    assert sum(1 for v in got if v == 2) == r.branch[2]
    # the iterate after the ten capped cycles agrees with the oracle's
    assert np.linalg.norm(x.cpu().numpy() - xo) <= 1e-9 * np.linalg.norm(xo)


def test_idr_branches_match_oracle_with_criterion_2_forced():
    """The same for IDR(4)-Proj(4): capped cycles force criterion 2 and the
    host-driven drivers' cycle start (shared with BiCGStab's) logs it."""
    dims, beta, k = (63, 63), (40.0, 0.0), 4
    oop = O.const_cd(dims, beta)
    b = W.rhs(oop.n, 3)
    op = tg().Operator.const_cd(dims, beta)
    Wb, V, H = _space(oop, k, 103)
    space = tg().defl_from_basis(op, _t(Wb.T))
    s = 4
    draw = W.shadow_draw(oop.n, s, 9)
    P = OI.shadow_space(draw.T)
    kw = dict(rtol=1e-8, ncyc=10, maxit_cycle=6, max_extra=0)
    xo, orep = OI.idrs_proj(oop, b, P, V=V, H=H, **kw)
    x, r = tg().solve_idr(op, _t(b), s=s, shadow=_t(draw), defl=space, **kw)
    assert r.cycles == orep.cycles == 10
    idx = _decided(orep.cycle_nu)
    want = orep.branches
    assert sum(1 for i in idx if want[i] == 2) >= 5
    assert [r.cycle_branch[i] for i in idx] == [want[i] for i in idx], (r.cycle_branch[:10], want)


@pytest.mark.parametrize("dims,beta,precision", [((255, 255), (100.0, 0.0), "fp64"),
                                                 ((255, 255), (100.0, 0.0), "fp32_ir"),
                                                 ((47, 31, 21), (50.0, 20.0, 10.0), "fp64")])
def test_resume_equals_uninterrupted_bit_for_bit(dims, beta, precision):
    """A solve stopped after j cycles (max_cycles_call) and resumed with
    icyc0 = j and the first call's nu0 ends with the same x, bit for bit, as
    the uninterrupted solve; the cycle counts and the criteria of the
    resumed cycles are those of the uninterrupted run."""
    op = tg().Operator.const_cd(dims, beta)
    cop = op.coarsen()
    b = _t(W.rhs(op.n, 5))
    xc, cspace, _ = tg().coarse_setup(cop, tg().restrict(op, cop, b), 30, 8, 6, 1e-6, 1e-8, 60)
    space = tg().defl_prolongate(cspace, op)
    x0 = tg().prolongate(cop, op, xc)
    kw = dict(defl=space, rtol=1e-10, ncyc=12, precision=precision)
    xu, ru = tg().solve(op, b, x0=x0, **kw)
    assert ru[0].status == 0 and ru[0].cycles > 6
    j = 4
    x1, r1 = tg().solve(op, b, x0=x0, max_cycles_call=j, **kw)
    assert r1[0].status == 1 and r1[0].cycles == j
    x2, r2 = tg().solve(op, b, x0=x1, icyc0=j, nu0=r1[0].nu0, **kw)
    assert r2[0].status == 0 and r2[0].cycles == ru[0].cycles
    assert torch.equal(x2, xu)
    assert r2[0].cycle_branch[j:ru[0].cycles] == ru[0].cycle_branch[j:ru[0].cycles]
    assert r1[0].cycle_branch[:j] == ru[0].cycle_branch[:j]
    assert r2[0].mvp_inner + r1[0].mvp_inner == ru[0].mvp_inner


def test_resume_rejects_bad_arguments():
    op = tg().Operator.const_cd((31, 31), (10.0, 0.0))
    b = _t(W.rhs(op.n, 1))
    from paper_2005_03070_amd._lib import TgdkError
    with pytest.raises(TgdkError):
        tg().solve(op, b, icyc0=2)           # a resumed solve needs the iterate
    with pytest.raises(TgdkError):
        tg().solve(op, b, x0=b, icyc0=-1)
    with pytest.raises(TgdkError):
        tg().solve(op, b, x0=b, nu0=-1.0)


def test_duplicated_coarse_column_is_singular():
    """A moved basis with two equal columns is rank deficient: building the
    space fails with TGDK_E_SINGULAR from the Cholesky QR, on the coarse grid
    and for a fine basis; the context stays usable and a solve afterwards is
    finite and converges."""
    from paper_2005_03070_amd._lib import TgdkError, E_SINGULAR
    op = tg().Operator.const_cd((63, 63), (40.0, 0.0))
    cop = op.coarsen()
    Wc = W.rng(4).standard_normal((6, cop.n))
    Wc[4] = Wc[1]
    with pytest.raises(TgdkError) as ei:
        tg().defl_from_basis(cop, _t(Wc))
    assert ei.value.code == E_SINGULAR
    Wf = W.rng(5).standard_normal((6, op.n))
    Wf[5] = Wf[0]
    with pytest.raises(TgdkError) as ei:
        tg().defl_from_basis(op, _t(Wf))
    assert ei.value.code == E_SINGULAR
    b = _t(W.rhs(op.n, 1))
    x, reps = tg().solve(op, b, rtol=1e-8)
    assert reps[0].status == 0 and bool(torch.isfinite(x).all())
    oop = O.const_cd((63, 63), (40.0, 0.0))
    xb = x.cpu().numpy()
    assert np.linalg.norm(W.rhs(op.n, 1) - O.apply(oop, xb)) <= 1e-8 * np.linalg.norm(W.rhs(op.n, 1))
