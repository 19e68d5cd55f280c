"""3-D parity where the z-marching chunks are deep.  The step kernel gives
each workgroup a column chunk and walks its z planes four at a time, the
register sets of planes z-1 .. z+2 changing roles by position.  The chunk
count follows the kernel's residency: 768 for the float64 kernel (3
workgroups per compute unit on 256 units), 1024 for float32.  On
127 x 127 x 255 that gives 11-plane chunks (the last z chunk 2) in float64
and 8-plane chunks (the last 7) in float32, so every chunk carries its loads
and its planes from one group of four to the next and ends on a partial
group; x and y are ragged too (127 = 64 + 63 columns, 15 full row blocks of
8 and one of 7), and the step kernel's own vectors are stored with row
pitch 128.  Checked against the
oracle after a fixed small number of iterations: phases A and B (no
deflation), and the cycle boundary (marching true residual with the streamed
c = V^T r, w = V d, marching r -= A w) with deflation, in FP64 and with
FP32 inner cycles."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import operators as O, bicgstab as OB, deflation as OD, projection as OP

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"
DIMS = (127, 127, 255)
BETA = (50.0, 20.0, 10.0)


def tg():
    import paper_2005_03070_amd as m
    return m


def _t(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_chunk_depth_of_this_grid():
    """The launch shapes the rest of this file relies on: 2 x 16 columns of
    64 x 8 points; chunks of 11 planes for 768 chunks in all, 8 planes for
    1024 (both carry z over a group of four and end on a partial chunk)."""
    cols = ((DIMS[0] + 63) // 64) * ((DIMS[1] + 7) // 8)
    assert cols == 32
    for target, depth, last in ((768, 11, 2), (1024, 8, 7)):
        mz = max(4, min(DIMS[2], -(-cols * DIMS[2] // target)))
        assert (mz, DIMS[2] % mz) == (depth, last)


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_deep_march_k0_scalars_and_iterate(precision):
    """One cycle of six BiCGStab iterations from x = 0: the (rho, alpha,
    omega) of every iteration and the iterate agree with the oracle (FP64:
    1e-12 and 1e-11; float32 inner vectors: 1e-5 and 1e-4)."""
    oop = O.const_cd(DIMS, BETA)
    b = W.rhs(oop.n, 51)
    op = tg().Operator.const_cd(DIMS, BETA)
    kw = dict(rtol=1e-12, ncyc=1, max_extra=0, maxit_cycle=6, precision=precision)
    x, reps = tg().solve(op, _t(b), **kw)
    xo, orep = OB.bicgstab_proj(oop, b, **kw)
    r = reps[0]
    assert r.status == orep.status == 1 and r.mvp_inner == orep.mvp_inner == 12
    tol_s, tol_x = (1e-12, 1e-11) if precision == "fp64" else (1e-5, 1e-4)
    np.testing.assert_allclose(np.array(r.first_scalars)[:6], np.array(orep.first_scalars)[:6], rtol=tol_s)
    assert _rel(x.cpu().numpy(), xo) <= tol_x


@pytest.mark.parametrize("precision,store", [("fp64", torch.float64), ("fp32_ir", torch.float64),
                                             ("fp64", torch.float32)])
def test_deep_march_deflated_cycles(precision, store):
    """Three cycles of BiCGStab(3)-Proj(6) (four inner iterations each) with
    a seeded orthonormal basis: the iterate after every boundary action of
    the three cycles agrees with the oracle's run.  With float32 storage the
    oracle uses the same rounded basis and its H."""
    oop = O.const_cd(DIMS, BETA)
    b = W.rhs(oop.n, 52)
    k = 6
    V = OD.orthonormalize(W.rng(53).standard_normal((oop.n, k)))
    op = tg().Operator.const_cd(DIMS, BETA)
    space = tg().defl_from_basis(op, _t(V.T), store=store)
    Vo = V if store == torch.float64 else V.astype(np.float32).astype(np.float64)
    H = OP.projection_matrix(oop, Vo)
    kw = dict(rtol=1e-12, ncyc=3, max_extra=0, maxit_cycle=4, precision=precision)
    x, reps = tg().solve(op, _t(b), defl=space, **kw)
    xo, orep = OB.bicgstab_proj(oop, b, V=Vo, H=H, **kw)
    r = reps[0]
    assert r.status == orep.status == 1 and r.cycles == orep.cycles == 3
    assert r.mvp_inner == orep.mvp_inner and r.mvp_boundary == orep.mvp_boundary
    tol = {("fp64", torch.float64): 1e-10, ("fp32_ir", torch.float64): 1e-4,
           ("fp64", torch.float32): 1e-8}[(precision, store)]
    assert _rel(x.cpu().numpy(), xo) <= tol
    if precision == "fp64" and store == torch.float64:
        np.testing.assert_allclose(np.array(r.first_scalars)[:4], np.array(orep.first_scalars)[:4], rtol=1e-10)
