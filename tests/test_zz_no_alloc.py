"""The no-allocation entry point tgdk_solve_noalloc against tgdk_solve: the
same BiCGStab(ncyc)-Proj(k) solves, with the library's workspace in its fixed
per-device scratch, give the same solutions bit for bit; two calls in a row,
the second on a smaller input; no device memory is allocated during a call;
a call larger than the scratch is rejected and leaves x untouched."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"


def tg():
    import paper_2005_03070_amd as m
    return m


def _problem(N, beta, seeds):
    op = tg().Operator.const_cd((N, N), (beta, 0.0))
    B = torch.tensor(np.stack([W.rhs(op.n, s) for s in seeds]), device=DEV)
    solver = tg().TwoGridSolver(op, m=30, k=8, nev=6, rtolev=1e-6, maxcyc=60)
    x0 = solver.setup(B[0].contiguous())
    return op, solver.defl, B, torch.stack([x0] * len(seeds)).contiguous()


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_noalloc_equals_solve_on_two_calls(precision):
    cases = [(511, 100.0, (21, 22, 23)), (255, 60.0, (24,))]   # the second call is smaller
    for N, beta, seeds in cases:
        op, space, B, X0 = _problem(N, beta, seeds)
        kw = dict(x0=X0, defl=space, rtol=1e-9, ncyc=20, precision=precision)
        x_ref, r_ref = tg().solve(op, B, **kw)
        out = torch.empty_like(B)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        x_na, r_na = tg().solve_noalloc(op, B, out=out, **kw)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0          # nothing allocated by the call
        assert torch.equal(x_na, x_ref), (N, precision)
        for a, b in zip(r_na, r_ref):
            assert a.status == b.status == 0
            assert (a.cycles, a.mvp_inner, a.mvp_boundary, a.vops) == (b.cycles, b.mvp_inner, b.mvp_boundary, b.vops)
            assert a.relres_true == b.relres_true and a.relres_true <= 1e-9


def test_noalloc_rejects_a_solve_larger_than_the_scratch():
    from paper_2005_03070_amd._lib import TgdkError, E_INVALID
    op = tg().Operator.const_cd((1023, 1023), (100.0, 0.0))    # 80 n bytes > 64 MiB in FP64
    b = torch.tensor(W.rhs(op.n, 2), device=DEV)
    out = torch.full_like(b, 7.0)
    with pytest.raises(TgdkError) as ei:
        tg().solve_noalloc(op, b, out=out, rtol=1e-8)
    assert ei.value.code == E_INVALID and "scratch" in str(ei.value)
    assert bool((out == 7.0).all())
    # float32 inner cycles need 48 n bytes: this one fits and converges
    x, r = tg().solve_noalloc(op, b, rtol=1e-8, precision="fp32_ir", max_extra=40)
    assert r[0].status == 0 and r[0].relres_true <= 1e-8
