"""Pins of the oracle's grid transfer and Galerkin projection (CPU only)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import operators as O, transfer as T, projection as PJ, deflation as D
import workloads as W


def _p1_interp(nc):
    """1-D prolongation matrix built column by column with numpy.interp:
    the linear spline through the coarse nodes and zero boundary values."""
    nf = 2 * nc + 1
    xc = np.linspace(0, 1, nc + 2)
    xf = np.linspace(0, 1, nf + 2)[1:-1]
    cols = []
    for I in range(nc):
        vals = np.zeros(nc + 2)
        vals[I + 1] = 1.0
        cols.append(np.interp(xf, xc, vals))
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("cdims", [(5, 3), (4, 3, 2)])
def test_prolongation_is_tensor_linear_spline(cdims):
    mats = [_p1_interp(n) for n in cdims]
    P = np.ones((1, 1))
    for M in mats:  # x fastest
        P = np.kron(M, P)
    vc = np.random.default_rng(0).standard_normal(int(np.prod(cdims)))
    np.testing.assert_allclose(T.prolongate(vc, cdims), P @ vc, rtol=0, atol=1e-15)
    fdims = tuple(2 * n + 1 for n in cdims)
    vf = np.random.default_rng(1).standard_normal(int(np.prod(fdims)))
    np.testing.assert_allclose(T.restrict(vf, fdims), P.T @ vf / 2 ** len(cdims), rtol=0, atol=1e-15)


def test_prolongation_reproduces_separable_interpolant():
    """P of coarse samples of a(x) b(y) equals the product of the 1-D linear
    spline interpolants sampled at fine nodes."""
    nc = (7, 5)
    a = lambda x: np.sin(3 * x) + x**2
    b = lambda y: np.cos(2 * y) * y
    xc = [np.linspace(0, 1, n + 2) for n in nc]
    xf = [np.linspace(0, 1, 2 * n + 3) for n in nc]
    ac = a(xc[0]); ac[[0, -1]] = 0.0
    bc = b(xc[1]); bc[[0, -1]] = 0.0
    vc = np.outer(bc[1:-1], ac[1:-1]).reshape(-1)
    fa = np.interp(xf[0][1:-1], xc[0], ac)
    fb = np.interp(xf[1][1:-1], xc[1], bc)
    np.testing.assert_allclose(T.prolongate(vc, nc), np.outer(fb, fa).reshape(-1), atol=1e-15)


def test_transfer_exact_on_integers_and_adjoint():
    cdims = (6, 4, 3)
    fdims = tuple(2 * n + 1 for n in cdims)
    vc = W.integer_field(int(np.prod(cdims)), 5)
    vf = W.integer_field(int(np.prod(fdims)), 6)
    pv = T.prolongate(vc, cdims)
    assert np.array_equal(pv * 8, np.round(pv * 8))  # weights are eighths at most
    # <P vc, vf> = 2^d <vc, R vf>, exact with dyadic values
    assert (pv @ vf) == 8 * (vc @ T.restrict(vf, fdims))


def _projection_setup(seed=0):
    op = O.const_cd((13, 9), (30.0, -10.0))
    rng = np.random.default_rng(seed)
    V = D.orthonormalize(rng.standard_normal((op.n, 6)))
    H = PJ.projection_matrix(op, V)
    r = rng.standard_normal(op.n)
    x = rng.standard_normal(op.n)
    return op, V, H, x, r


def test_galerkin_condition():
    op, V, H, x, r = _projection_setup()
    x1, r1, d = PJ.galerkin(op, V, H, x, r)
    assert np.linalg.norm(V.T @ r1) < 1e-12 * np.linalg.norm(r)
    # consistency: r1 = r - A (x1 - x)
    np.testing.assert_allclose(r1, r - O.apply(op, x1 - x), atol=1e-10)


def test_galerkin_basis_invariance():
    """The projection depends only on span(V): V -> V M gives the same x."""
    op, V, H, x, r = _projection_setup(1)
    M = np.random.default_rng(7).standard_normal((6, 6)) + 3 * np.eye(6)
    V2 = V @ M
    H2 = V2.T @ O.apply(op, V2)
    x1, r1, _ = PJ.galerkin(op, V, H, x, r)
    x2, r2, _ = PJ.galerkin(op, V2, H2, x, r)
    np.testing.assert_allclose(x2, x1, atol=1e-10 * np.linalg.norm(x1))


def test_galerkin_over_exact_invariant_subspace():
    """If range(V) is an exact invariant subspace (closed-form right
    eigenvectors of a nonsymmetric operator) the projected residual is
    ``(I - V V^T) r``: every component in the subspace is removed."""
    nx, ny, bx = 15, 9, 12.0
    op = O.const_cd((nx, ny), (bx, 0.0))
    hx, hy = 1 / (nx + 1), 1 / (ny + 1)
    rho = np.sqrt((1 / hx**2 + bx / (2 * hx)) / (1 / hx**2 - bx / (2 * hx)))
    i = np.arange(1, nx + 1)
    j = np.arange(1, ny + 1)
    cols = []
    for a, c in [(1, 1), (2, 1), (1, 2), (3, 2)]:
        cols.append(np.outer(np.sin(j * c * np.pi * hy), rho**i * np.sin(i * a * np.pi * hx)).reshape(-1))
    V = D.orthonormalize(np.stack(cols, axis=1))
    H = PJ.projection_matrix(op, V)
    r = np.random.default_rng(4).standard_normal(op.n)
    _, r1, _ = PJ.galerkin(op, V, H, np.zeros(op.n), r)
    np.testing.assert_allclose(r1, r - V @ (V.T @ r), atol=1e-11 * np.linalg.norm(r))


def test_orthonormalize_unique_qr():
    Wm = np.random.default_rng(5).standard_normal((200, 7))
    Q = D.orthonormalize(Wm)
    assert np.linalg.norm(Q.T @ Q - np.eye(7)) < 1e-13
    R = Q.T @ Wm
    assert np.allclose(np.tril(R, -1), 0, atol=1e-12) and np.all(np.diag(R) > 0)
