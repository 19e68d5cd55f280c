"""GPU parity of the grid kernels (stencil, transfer, gradient) against the
oracle, through the C-ABI."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import operators as O, transfer as T, adjoint as ADJ

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

DEV = "cuda:0"


def tg():
    import paper_2005_03070_amd as m
    return m


def _t(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


@pytest.mark.parametrize("dims", [(150, 37), (64, 16), (1, 1), (3, 200), (70, 9, 11), (65, 5, 4)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_var_stencil_bitexact_on_integers(dims, dtype):
    """Integer coefficients and integer x: every sum is exact, so the GPU
    result equals the oracle bit for bit, for A and A^T, several tiles and
    ragged tails, two right-hand sides."""
    n = int(np.prod(dims))
    shape = tuple(reversed(dims))
    names = ["C", "W", "E", "S", "N"] + (["D", "U"] if len(dims) == 3 else [])
    coef = {k: W.integer_field(shape, 10 + i) for i, k in enumerate(names)}
    oop = O.StencilOp(dims, coef, kind="var")
    op = tg().Operator.var_stencil(dims, _t(np.stack([coef[k].reshape(-1) for k in names])))
    x = np.stack([W.integer_field(n, 3), W.integer_field(n, 4)])
    xt = _t(x, dtype)
    for tr in (False, True):
        y = op.apply(xt, transpose=tr).cpu().numpy().astype(np.float64)
        ref = np.stack([(O.apply_transpose if tr else O.apply)(oop, x[j]) for j in range(2)])
        assert np.array_equal(y, ref), (dims, dtype, tr)


@pytest.mark.parametrize("dims,beta", [((1023, 1023), (100.0, 0.0)), ((255, 255, 255), (50.0, 20.0, 10.0)),
                                       ((97, 33), (40.0, -5.0)), ((17, 9, 40), (3.0, 0.0, 7.0))])
def test_const_stencil_random(dims, beta):
    """Constant coefficients, random x: within a few ulps of the row sum."""
    op = tg().Operator.const_cd(dims, beta)
    oop = O.const_cd(dims, beta)
    x = W.rhs(op.n, 5)
    ref = O.apply(oop, x)
    scale = (abs(oop.coef["C"]) * 2) * np.abs(x).max()
    y64 = op.apply(_t(x)).cpu().numpy()
    assert np.abs(y64 - ref).max() <= 1e-14 * scale
    y32 = op.apply(_t(x, torch.float32)).cpu().numpy()
    assert np.abs(y32 - ref).max() <= 2e-6 * scale
    yt = op.apply(_t(x), transpose=True).cpu().numpy()
    assert np.abs(yt - O.apply_transpose(oop, x)).max() <= 1e-14 * scale


def test_div_k_operator_and_transpose():
    dims = (131, 77)
    k = W.kfield(dims, 5)
    beta = (60.0, 0.0)
    op = tg().Operator.div_k(dims, _t(k), beta)
    oop = O.div_k(dims, k, beta)
    x = W.rhs(op.n, 2)
    scale = np.abs(oop.coef["C"]).max() * 3 * np.abs(x).max()
    for tr in (False, True):
        y = op.apply(_t(x), transpose=tr).cpu().numpy()
        ref = (O.apply_transpose if tr else O.apply)(oop, x)
        assert np.abs(y - ref).max() <= 1e-13 * scale
    # coarsening: geometric mean of the 2x2 fine cells
    opc = op.coarsen()
    oopc = O.coarsen(oop)
    xc = W.rhs(opc.n, 3)
    yc = opc.apply(_t(xc)).cpu().numpy()
    assert np.abs(yc - O.apply(oopc, xc)).max() <= 1e-12 * np.abs(oopc.coef["C"]).max() * np.abs(xc).max()


@pytest.mark.parametrize("cdims", [(37, 21), (1, 1), (63, 2), (9, 6, 5), (2, 3, 1)])
def test_transfer_bitexact(cdims):
    """Prolongation and restriction on random float64 data equal the oracle
    to the bit (weights are powers of two; fixed x, y, z order)."""
    fdims = tuple(2 * d + 1 for d in cdims)
    fine = tg().Operator.const_cd(fdims)
    coarse = tg().Operator.const_cd(cdims)
    vc = np.stack([W.rhs(coarse.n, 1), W.rhs(coarse.n, 2)])
    vf = np.stack([W.rhs(fine.n, 3), W.rhs(fine.n, 4)])
    p = tg().prolongate(coarse, fine, _t(vc)).cpu().numpy()
    r = tg().restrict(fine, coarse, _t(vf)).cpu().numpy()
    for j in range(2):
        assert np.array_equal(p[j], T.prolongate(vc[j], cdims))
        assert np.array_equal(r[j], T.restrict(vf[j], fdims))


def test_grad_k_kernel():
    dims = (45, 30)
    op = tg().Operator.div_k(dims, _t(W.kfield(dims, 1)), (60.0, 0.0))
    lam, u = W.rhs(op.n, 8), W.rhs(op.n, 9)
    g = tg().grad_k(op, _t(lam), _t(u)).cpu().numpy()
    ref = ADJ.grad_k(lam, u, dims)
    assert np.abs(g - ref).max() <= 1e-13 * np.abs(ref).max()


def test_every_tile_shape_gives_identical_stencil(tmp_path, monkeypatch):
    """Each candidate tile shape of the autotuner (forced through the tune
    cache) gives bit-identical stencil output; a real tuning run picks one."""
    for dims in [(200, 90), (40, 21, 19)]:
        op = tg().Operator.const_cd(dims, (30.0, 10.0, 5.0)[: len(dims)])
        x = _t(W.rhs(op.n, 1))
        key = "gfx950 dim=%d n=%d,%d,%d dtype=0 nrhs=1" % (
            len(dims), dims[0], dims[1], dims[2] if len(dims) == 3 else 1)
        outs = []
        for tile in range(3):
            f = tmp_path / f"cache{tile}.txt"
            f.write_text(f"{key} tile={tile}\n")
            monkeypatch.setenv("TGDK_TUNE_CACHE", str(f))
            op.tune()
            outs.append(op.apply(x).cpu().numpy())
        assert all(np.array_equal(outs[0], o) for o in outs[1:])
        monkeypatch.setenv("TGDK_TUNE_CACHE", str(tmp_path / "fresh.txt"))
        ty = op.tune()
        # candidate tile heights: 2-D 16, 8, 4, 32; 3-D 4, 8, 4, 2 (timing decides)
        assert ty in ((16, 8, 4, 32) if len(dims) == 2 else (4, 8, 2))
        assert "tile=" in (tmp_path / "fresh.txt").read_text()


@pytest.mark.parametrize("pattern", ["contiguous", "march", "tiled", "march_pf2", "march_pf3"])
def test_stream_probe_runs_every_pattern_and_mix(pattern):
    """The streaming probe (a measurement utility, not a step of the method)
    on a ragged grid smaller than one chunk in x and y, more than one in z:
    every pattern and stream mix completes and reports the bytes of the
    grid's points; an unknown mix and a bad grid are refused."""
    dims = (65, 9, 7)
    for nr, nw in ((1, 1), (3, 1), (6, 4)):
        ms, nbytes = tg().stream_probe(pattern, nr, nw, dims, blocks=8, reps=2)
        pts = (128 if pattern == "contiguous" else 65) * 9 * 7
        assert ms > 0 and nbytes == (nr + nw) * pts * 8
    with pytest.raises(tg()._lib.TgdkError):
        tg().stream_probe(pattern, 2, 2, dims)
    with pytest.raises(tg()._lib.TgdkError):
        tg().stream_probe(pattern, 1, 1, (0, 9, 7))
