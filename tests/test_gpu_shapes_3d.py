"""The 3-D step kernel over grid shapes at and around its chunk geometry
(64-point x rows, 8-row column blocks, z chunks, the row pitch rounded up to
64): a single point, shapes smaller than one chunk, exact multiples, one past
them, thin and deep grids.  No deflation and the oracle's orthonormal basis
of a seeded random 6-vector space, FP64 and FP32 inner cycles: the first
(rho, alpha, omega) agree with the oracle's in FP64 (1e-12 without
deflation, 1e-10 with it, as the two orthonormalisations differ in
rounding), the true residual meets rtol and the solution the direct
solution (1e-7)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spl
import torch

import workloads as W
from oracle import bicgstab as OB, deflation as OD, operators as O, projection as OP

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"
SHAPES = [(1, 1, 1), (3, 2, 5), (64, 8, 4), (65, 9, 5), (63, 7, 33), (130, 3, 70), (5, 70, 6)]
BETA = (20.0, 10.0, 5.0)


def tg():
    import paper_2005_03070_amd as m
    return m


def _t(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
@pytest.mark.parametrize("k", [0, 6])
@pytest.mark.parametrize("dims", SHAPES, ids=["x".join(map(str, d)) for d in SHAPES])
def test_3d_shapes_against_oracle_and_direct(dims, k, precision):
    n = int(np.prod(dims))
    if k >= n:
        pytest.skip("space as large as the grid")
    oop = O.const_cd(dims, BETA)
    b = W.rhs(n, 41)
    op = tg().Operator.const_cd(dims, BETA)
    V = H = None
    kw = {}
    if k:
        V = OD.orthonormalize(W.rng(42).standard_normal((n, k)))
        H = OP.projection_matrix(oop, V)
        kw["defl"] = tg().defl_from_basis(op, _t(V.T))
    rtol = 1e-10
    x, reps = tg().solve(op, _t(b), rtol=rtol, ncyc=20, precision=precision, max_extra=40, **kw)
    r = reps[0]
    assert r.status == 0, r.status_name
    xo, orep = OB.bicgstab_proj(oop, b, V=V, H=H, rtol=rtol, ncyc=20, precision=precision, max_extra=40)
    m = min(3, len(r.first_scalars), len(orep.first_scalars))
    if precision == "fp64" and m:
        got, ref = np.array(r.first_scalars[:m]), np.array(orep.first_scalars[:m])
        fin = np.isfinite(ref)
        np.testing.assert_allclose(got[fin], ref[fin], rtol=1e-12 if k == 0 else 1e-10)
    xg = x.cpu().numpy()
    assert np.linalg.norm(b - O.apply(oop, xg)) <= 1.0001 * rtol * np.linalg.norm(b)
    xs = spl.spsolve(O.to_csr(oop).tocsc(), b) if n > 1 else b / O.to_csr(oop).toarray()[0, 0]
    assert np.linalg.norm(xg - xs) / np.linalg.norm(xs) <= 1e-7
