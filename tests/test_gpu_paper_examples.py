"""The paper's Example 2 run as printed on the GPU (Sec. 4.1, Table 4.1;
operator, grids and coarse phase of Sec. 3, Example 1), against the paper's
own operator counts.

The operator -exp(5xy)(u_xx + u_yy) + 40 u_x + 40 u_y has per-row
coefficients (the oracle's `example1_operator`, passed to the library as a
VAR_STENCIL operator on each grid 511^2, 255^2, 127^2, 63^2); the coarse grid
h = 1/64 is three nested levels below h = 1/512, so the coarse right-hand
side is restricted and the moved vectors and coarse solution prolongated
level by level.  GMRES-DR(150,100) runs until 80 pairs have converged;
BiCGStab(ncyc)-Proj(100) solves to rtol 1e-10 for every ncyc of Table 4.1.

The paper's "residual norm below 1e-8" does not say how its matrix is
scaled; the eigen-residual 1e-10 relative to ||A||_1 reproduces its
coarse phase: 109 cycles and 5513 products here against the paper's 107 and
5450 (Sec. 3, Example 1), so that is the setting here.  The paper ran
MATLAB's BiCGStab, whose exit rules differ from the textbook iteration here,
and interpolated with splines of unstated degree (linear here), so the
fine counts are a soft band, as for Table 4.2: every ncyc >= 20 within 20 %
of the printed value, and the table's shape: ncyc = 5 and 10 need more
products than ncyc = 20, at most twice the printed count."""
import json
import os

import numpy as np
import pytest
import torch

import workloads as W
from oracle import operators as O

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table_4_1_example2.json")))


def tg():
    import paper_2005_03070_amd as m
    return m


def _t(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _var_op(n):
    oop = O.example1_operator(n)
    coef = np.stack([oop.coef_array(k).reshape(-1) for k in ("C", "W", "E", "S", "N")])
    return oop, tg().Operator.var_stencil((n, n), _t(coef))


def test_example2_table_4_1_counts():
    sizes = [511, 255, 127, 63]
    pairs = [_var_op(n) for n in sizes]
    oop, op = pairs[0]
    h = 1.0 / 512
    xs = h * np.arange(1, 512)
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    f = (np.sin(X) * np.cos(X) * np.exp(X * Y)).reshape(-1)
    b = f / np.linalg.norm(f)
    m, k, nev = GOLD["gmresdr"]
    solver = tg().TwoGridSolver(op, m=m, k=k, nev=nev, rtolev=1e-10, maxcyc=400, levels=3,
                                grids=[p[1] for p in pairs])
    bt = _t(b)
    x0 = solver.setup(bt)
    rep0 = solver.setup_report
    assert rep0.nconv >= nev and solver.defl.k >= k
    got = {}
    for ncyc, paper, used in zip(GOLD["ncyc"], GOLD["mvps"], GOLD["cycles_used"]):
        x, reps = tg().solve(op, bt, x0=x0, defl=solver.defl, ncyc=ncyc, rtol=GOLD["rtol"], max_extra=ncyc)
        r = reps[0]
        rr = np.linalg.norm(b - O.apply(oop, x.cpu().numpy())) / np.linalg.norm(b)
        got[ncyc] = r.mvp_inner
        print(f"ncyc {ncyc}: {r.mvp_inner} mvps (paper {paper}), {r.cycles} cycles (paper {used}), "
              f"relres {rr:.2e}", flush=True)
        assert r.status == 0 and rr <= GOLD["rtol"]
    print(f"coarse GMRES-DR({m},{k}): {rep0.cycles} cycles, {rep0.mvps} mvps (paper: 107 cycles, 5450 mvps "
          f"for 80 pairs)", flush=True)
    assert abs(rep0.cycles - 107) <= 0.2 * 107
    for ncyc, paper in zip(GOLD["ncyc"], GOLD["mvps"]):
        if ncyc >= 20:
            assert abs(got[ncyc] - paper) <= 0.2 * paper, (ncyc, got[ncyc], paper)
        else:
            assert got[20] < got[ncyc] <= 2 * paper, (ncyc, got[ncyc], paper)
