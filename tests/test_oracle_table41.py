"""The oracle's whole deflated pipeline against the paper's own counts: the
Example 2 problem of Sec. 4.1 (operator, grids and coarse phase of Sec. 3,
Example 1) run by the oracle alone, against Table 4.1 and the coarse figures
of Example 1 (tests/golden/table_4_1_example2.json).

The coarse GMRES-DR(150,100) runs on 63^2, three nested levels below the
511^2 fine grid, until 80 pairs have a relative eigen-residual below 1e-10
(the reading that reproduces the paper's 107 cycles; its own scaling is not
stated); the kept vectors are prolongated level by level and
orthonormalised, and BiCGStab(ncyc)-Proj(100) solves to rtol 1e-10.  The
band is the one the GPU test holds: the coarse cycles and the fine counts
for ncyc = 20 and 100 within 20 % of the printed values, ncyc = 5 above
ncyc = 20 and at most twice its printed count.

About ten minutes of CPU time, so it runs only with TGDK_SLOW=1."""
import json
import os

import numpy as np
import pytest

from oracle import bicgstab, deflation, gmresdr, operators as O, projection, transfer

pytestmark = [pytest.mark.slow,
              pytest.mark.skipif(os.environ.get("TGDK_SLOW") != "1", reason="about 10 min; set TGDK_SLOW=1")]

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table_4_1_example2.json")))


def test_oracle_example2_table_4_1_band():
    sizes = [511, 255, 127, 63]
    ops = [O.example1_operator(n) for n in sizes]
    h = 1.0 / 512
    xs = h * np.arange(1, 512)
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    f = (np.sin(X) * np.cos(X) * np.exp(X * Y)).reshape(-1)
    b = f / np.linalg.norm(f)
    bc = b
    for op in ops[:-1]:
        bc = transfer.restrict(bc, op.dims)
    m, k, nev = GOLD["gmresdr"]
    xc, Wc, rep0 = gmresdr.gmres_dr(ops[-1], bc, m, k, nev=nev, rtolev=1e-10, rtol=1e-8, maxcyc=400)
    assert rep0.nconv >= nev and Wc.shape[1] >= k
    assert abs(rep0.cycles - 107) <= 0.2 * 107, rep0.cycles
    Wf, x0 = Wc, xc
    for op in ops[-1:0:-1]:
        Wf = deflation.orthonormalize(transfer.prolongate(Wf, op.dims))
        x0 = transfer.prolongate(x0, op.dims)
    V = Wf
    H = projection.projection_matrix(ops[0], V)
    got = {}
    for ncyc in (5, 20, 100):
        x, rep = bicgstab.bicgstab_proj(ops[0], b, x0=x0, V=V, H=H, rtol=GOLD["rtol"], ncyc=ncyc, max_extra=ncyc)
        assert rep.status == bicgstab.OK
        assert np.linalg.norm(b - O.apply(ops[0], x)) <= GOLD["rtol"] * np.linalg.norm(b)
        got[ncyc] = rep.mvp_inner
        print(f"oracle ncyc {ncyc}: {rep.mvp_inner} mvps, {rep.cycles} cycles", flush=True)
    print(f"oracle coarse GMRES-DR({m},{k}): {rep0.cycles} cycles, {rep0.mvps} mvps", flush=True)
    printed = dict(zip(GOLD["ncyc"], GOLD["mvps"]))
    for ncyc in (20, 100):
        assert abs(got[ncyc] - printed[ncyc]) <= 0.2 * printed[ncyc], (ncyc, got[ncyc], printed[ncyc])
    assert got[20] < got[5] <= 2 * printed[5], got
