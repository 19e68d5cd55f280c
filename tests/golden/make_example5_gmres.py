"""Writes example5_gmres_oracle.json: the oracle's Example 5 pipeline (Sec. 5)
as the benchmark runs it, with the first ten cycles of GMRES(100)-Proj(100).

The Helmholtz operator -Lap(u) - 100^2 u on 511^2, b ~ N(0,1) (seed of the
Example 5 workload), coarse grid 127^2 two levels down; multigrid on
-Lap(u) + 100^2 u (two V-cycles, two damped Jacobi sweeps each side)
preconditions both grids from the right; GMRES-DR(150,100) on A_c M_c^-1 until
80 pairs converge; the kept vectors and the coarse solution moved up level
by level (linear interpolation, the vectors orthonormalised on each level);
Z = M^-1 V and H = V^T A Z; then GMRES(100)-Proj(100) from the moved
solution.  Records ||b - A x|| / ||b|| at the end of each of the first ten
cycles.  Calls only oracle/ and the seeded inputs; about ten minutes on
one core.  Run from the repository root: python tests/golden/make_example5_gmres.py"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import deflation as D, gmres, gmresdr, multigrid as MG, operators as O, projection as P, transfer as T  # noqa: E402
import workloads as W  # noqa: E402

CYCLES = 10


def main():
    c = W.CONFIGS["H2"]
    fine = O.const_cd(c["n"], c["beta"], sigma=c["sigma"])
    mid = O.coarsen(fine)
    coarse = O.coarsen(mid)
    b = W.rhs(fine.n, c["seed"])
    bc = T.restrict(T.restrict(b, fine.dims), mid.dims)
    mf = MG.levels(O.const_cd(c["n"], c["beta"], sigma=-c["sigma"]))
    mc = MG.levels(O.const_cd(coarse.dims, c["beta"], sigma=-c["sigma"]))

    def pf(v):
        return MG.mg_apply(mf, v, cycles=c["mg_cycles"], nu=c["mg_nu"])

    def pc(v):
        return MG.mg_apply(mc, v, cycles=c["mg_cycles"], nu=c["mg_nu"])

    xc, Wc, rep = gmresdr.gmres_dr(coarse, bc, c["m"], c["k"], nev=c["nev"], rtolev=c["rtolev"], rtol=c["rtol"],
                                   maxcyc=c["maxcyc"], precond=pc)
    V = D.orthonormalize(T.prolongate(D.orthonormalize(T.prolongate(Wc, coarse.dims)), mid.dims))
    x0 = T.prolongate(T.prolongate(xc, coarse.dims), mid.dims)
    Z, H = P.precond_space(fine, V, pf)
    _, r = gmres.gmres_proj(fine, b, x0=x0, V=V, H=H, Z=Z, precond=pf, rtol=c["rtol"], m=c["m3"], maxcyc=CYCLES)
    nb = float(np.linalg.norm(b))
    out = {
        "citation": "Sec. 5, Example 5: -u_xx - u_yy - 100^2 u on 511^2 (h = 1/512), random normal right-hand "
                    "side, multigrid on the positively shifted Laplacian preconditioning both grids, "
                    "GMRES-DR(150,100) on the 127^2 coarse grid until 80 eigenpairs converge, GMRES(100)-Proj(100) "
                    "on the fine grid; values computed by the oracle (this script), not printed in the paper",
        "coarse_cycles": int(rep.cycles),
        "k": int(V.shape[1]),
        "relres_after_cycle": [float(v) / nb for v in r.nu_hist[:CYCLES]],
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "example5_gmres_oracle.json"), "w") as f:
        json.dump(out, f, indent=2)
        f.write("\n")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
