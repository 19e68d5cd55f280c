"""Example 5 of Sec. 5 (the Helmholtz problem with multigrid preconditioning
on both grids): GMRES(100)-Proj(100) on the GPU against the oracle's first
ten cycles (tests/golden/example5_gmres_oracle.json, written by
tests/golden/make_example5_gmres.py from the oracle alone).

The whole pipeline runs as the benchmark runs it: the coarse GMRES-DR(150,100)
on A_c M_c^-1 takes as many cycles as the oracle's (within 3: its 80th pair
converges at the edge of the tolerance), and the true relative residual at
the end of cycles 1, 2, 5 and 10 is the oracle's within 2e-3 relative (the
two coarse spaces agree to their eigen-residuals, about 1e-10, in the 80
converged pairs and less closely in the 20 kept vectors that have not
converged; measured: within 3e-4).  With linearly interpolated vectors the
residual stalls near 3e-3 on both sides, so the test also records that the
tenth cycle stays above 1e-3."""
import json
import os

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "example5_gmres_oracle.json")))


def tg():
    import paper_2005_03070_amd as m
    return m


def test_example5_gmres_proj_first_cycles_match_oracle():
    c = W.CONFIGS["H2"]
    shift = -c["sigma"]
    op = tg().Operator.const_cd(c["n"], c["beta"], sigma=c["sigma"])
    b = torch.tensor(W.rhs(op.n, c["seed"]), device=DEV)
    mg = tg().Multigrid(tg().Operator.const_cd(c["n"], c["beta"], sigma=shift), cycles=c["mg_cycles"], nu=c["mg_nu"])
    grids = [op]
    for _ in range(c["levels"]):
        grids.append(grids[-1].coarsen())
    mgc = tg().Multigrid(tg().Operator.const_cd(grids[-1].dims, c["beta"], sigma=shift), cycles=c["mg_cycles"],
                         nu=c["mg_nu"])
    bc = b
    for lv in range(c["levels"]):
        bc = tg().restrict(grids[lv], grids[lv + 1], bc)
    xc, space, srep = tg().coarse_setup(grids[-1], bc, c["m"], c["k"], c["nev"], c["rtolev"], c["rtol"], c["maxcyc"],
                                        precond=mgc)
    print(f"coarse GMRES-DR: {srep.cycles} cycles (oracle {GOLD['coarse_cycles']})", flush=True)
    assert abs(srep.cycles - GOLD["coarse_cycles"]) <= 3
    for lv in range(c["levels"] - 1, -1, -1):
        space = tg().defl_prolongate(space, grids[lv])
        xc = tg().prolongate(grids[lv + 1], grids[lv], xc)
    space = space.precond(mg)
    assert space.k == GOLD["k"]
    nb = float(torch.linalg.norm(b))
    got = {}
    for j in (1, 2, 5, 10):
        x, reps = tg().solve(op, b, x0=xc, defl=space, method="gmres", m3=c["m3"], rtol=c["rtol"], max_extra=j,
                             precond=mg)
        assert reps[0].mvp_inner == j * c["m3"]
        got[j] = float(torch.linalg.norm(b - op.apply(x))) / nb
        ref = GOLD["relres_after_cycle"][j - 1]
        print(f"cycle {j}: relres {got[j]:.5e} (oracle {ref:.5e})", flush=True)
        np.testing.assert_allclose(got[j], ref, rtol=2e-3)
    assert got[10] > 1e-3
