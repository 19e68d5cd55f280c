"""Pins of the oracle's operators against closed forms and independent
constructions (CPU only)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

from oracle import operators as O
import workloads as W


def _tri_eig(n, h, w, e):
    """Closed-form eigen-decomposition of tridiag(w, 2/h^2, e), w*e > 0."""
    j = np.arange(1, n + 1)
    lam = 2.0 / h**2 - 2.0 * np.sqrt(w * e) * np.cos(j * np.pi * h)
    rho = np.sqrt(w / e)
    i = np.arange(1, n + 1)[:, None]
    right = rho**i * np.sin(i * j[None, :] * np.pi * h)
    left = rho ** (-i) * np.sin(i * j[None, :] * np.pi * h)
    return lam, right, left


def _coefs_1d(n, beta):
    h = 1.0 / (n + 1)
    return h, -1 / h**2 - beta / (2 * h), -1 / h**2 + beta / (2 * h)


@pytest.mark.parametrize("dims,beta", [((15, 11), (6.0, -9.0)), ((9, 7, 5), (5.0, 3.0, -4.0))])
def test_closed_form_eigenpairs_right_and_left(dims, beta):
    """A v = lam v for tensor products of the 1-D right eigenvectors, and
    A^T u = lam u for the left ones (a sign, axis or transpose error in the
    stencil breaks one of them)."""
    op = O.const_cd(dims, beta)
    eigs = [_tri_eig(n, *_coefs_1d(n, b)) for n, b in zip(dims, beta)]
    rng = np.random.default_rng(0)
    for _ in range(6):
        idx = [rng.integers(0, n) for n in dims]
        lam = sum(e[0][i] for e, i in zip(eigs, idx))
        vr = np.ones(1)
        vl = np.ones(1)
        for e, i in zip(eigs, idx):  # x fastest: kron(z, y, x)
            vr = np.kron(e[1][:, i], vr)
            vl = np.kron(e[2][:, i], vl)
        rr = np.linalg.norm(O.apply(op, vr) - lam * vr) / (lam * np.linalg.norm(vr))
        rl = np.linalg.norm(O.apply_transpose(op, vl) - lam * vl) / (lam * np.linalg.norm(vl))
        assert rr < 1e-13 and rl < 1e-13


def _kron_assembly(dims, beta, sigma=0.0):
    """Independent assembly: A = sum_a I (x) ... (x) T_a (x) ... (x) I."""
    mats = []
    for n, b in zip(dims, beta):
        h, w, e = _coefs_1d(n, b)
        mats.append(sp.diags([np.full(n - 1, w), np.full(n, 2 / h**2), np.full(n - 1, e)], [-1, 0, 1]))
    N = int(np.prod(dims))
    A = sigma * sp.identity(N)
    for a, T in enumerate(mats):
        left = sp.identity(int(np.prod(dims[a + 1:])))   # slower axes
        right = sp.identity(int(np.prod(dims[:a])))      # faster axes
        A = A + sp.kron(sp.kron(left, T), right)
    return A.tocsr()


@pytest.mark.parametrize("dims,beta,sigma", [((13, 8), (40.0, 10.0), 0.0), ((5, 6, 7), (50.0, 20.0, 10.0), 3.5)])
def test_apply_matches_kronecker_assembly(dims, beta, sigma):
    op = O.const_cd(dims, beta, sigma)
    A = _kron_assembly(dims, beta, sigma)
    x = np.random.default_rng(1).standard_normal(op.n)
    np.testing.assert_allclose(O.apply(op, x), A @ x, rtol=0, atol=1e-9 * abs(A).max())
    np.testing.assert_allclose(O.apply_transpose(op, x), A.T @ x, rtol=0, atol=1e-9 * abs(A).max())
    assert abs(O.to_csr(op) - A).max() < 1e-9 * abs(A).max()


def test_integer_data_apply_is_exact():
    """With integer coefficients and integer x every sum is exact."""
    dims = (10, 7)
    coef = {k: W.integer_field((7, 10), s) for s, k in enumerate("CWESN")}
    op = O.StencilOp(dims, coef, kind="var")
    x = W.integer_field(op.n, 9)
    A = O.to_csr(op)
    assert np.array_equal(O.apply(op, x), A @ x)
    assert np.array_equal(O.apply_transpose(op, x), A.T @ x)


def test_smallest_eigenvalues_of_workload_operator():
    """The sparse operator of the small workload has the closed-form smallest
    eigenvalues (shift-invert Arnoldi on the explicit matrix)."""
    op = O.const_cd((63, 63), (40.0, 0.0))
    lam_x = _tri_eig(63, *_coefs_1d(63, 40.0))[0]
    lam_y = _tri_eig(63, *_coefs_1d(63, 0.0))[0]
    exact = np.sort((lam_x[:, None] + lam_y[None, :]).reshape(-1))[:5]
    vals = spl.eigs(O.to_csr(op).tocsc(), k=5, sigma=0.0, return_eigenvectors=False)
    got = np.sort(vals.real)
    np.testing.assert_allclose(got, exact, rtol=1e-8)
    assert np.abs(vals.imag).max() < 1e-6 * exact[0]


def test_div_k_constant_k_is_laplacian():
    dims = (9, 12)
    op1 = O.div_k(dims, np.ones((13, 10)), beta=(7.0, -3.0), sigma=0.5)
    op2 = O.const_cd(dims, (7.0, -3.0), 0.5)
    assert abs(O.to_csr(op1) - O.to_csr(op2)).max() < 1e-9


def test_div_k_single_cell_changes_its_four_sides():
    """Raising k in one cell by dK changes exactly the couplings across that
    cell's four sides, each by dK/2 (arithmetic edge mean), with zero row sums
    of the change (flux form)."""
    nx, ny = 7, 6
    hx, hy = 1 / (nx + 1), 1 / (ny + 1)
    base = np.ones((ny + 1, nx + 1))
    cj, ci = 3, 2
    bumped = base.copy()
    bumped[cj, ci] += 2.0
    dA = (O.to_csr(O.div_k((nx, ny), bumped)) - O.to_csr(O.div_k((nx, ny), base))).toarray()
    # corners of the cell: nodes (ci, cj), (ci+1, cj), (ci, cj+1), (ci+1, cj+1) in
    # 0..n+1 numbering; interior index (i-1, j-1)
    def node(i, j):
        return (j - 1) * nx + (i - 1)
    expect = np.zeros_like(dA)
    sides = [((ci, cj), (ci + 1, cj), hx), ((ci, cj + 1), (ci + 1, cj + 1), hx),
             ((ci, cj), (ci, cj + 1), hy), ((ci + 1, cj), (ci + 1, cj + 1), hy)]
    for (i1, j1), (i2, j2), h in sides:
        c = 1.0 / (h * h)  # dK/2 = 1
        p_in = 1 <= i1 <= nx and 1 <= j1 <= ny
        q_in = 1 <= i2 <= nx and 1 <= j2 <= ny
        if p_in:
            expect[node(i1, j1), node(i1, j1)] += c
        if q_in:
            expect[node(i2, j2), node(i2, j2)] += c
        if p_in and q_in:
            expect[node(i1, j1), node(i2, j2)] -= c
            expect[node(i2, j2), node(i1, j1)] -= c
    np.testing.assert_allclose(dA, expect, atol=1e-9)


def test_div_k_energy_identity():
    """x^T A x = sum over edges k_e (x_p - x_q)^2 / h^2 when beta = 0
    (edges to the boundary use x_q = 0)."""
    nx, ny = 6, 5
    hx, hy = 1 / (nx + 1), 1 / (ny + 1)
    k = W.kfield((nx, ny), 3)
    op = O.div_k((nx, ny), k)
    x = np.random.default_rng(2).standard_normal(op.n)
    X = np.zeros((ny + 2, nx + 2))
    X[1:-1, 1:-1] = x.reshape(ny, nx)
    total = 0.0
    for j in range(ny + 2):
        for i in range(nx + 2):
            if i + 1 <= nx + 1 and 1 <= j <= ny:  # x-edge (i,j)-(i+1,j): cells (j-1,i), (j,i)
                ke = 0.5 * (k[j - 1, i] + k[j, i])
                total += ke * (X[j, i] - X[j, i + 1]) ** 2 / hx**2
            if j + 1 <= ny + 1 and 1 <= i <= nx:  # y-edge: cells (j,i-1), (j,i)
                ke = 0.5 * (k[j, i - 1] + k[j, i])
                total += ke * (X[j, i] - X[j + 1, i]) ** 2 / hy**2
    assert abs(x @ O.apply(op, x) - total) < 1e-10 * total


@pytest.mark.parametrize("make", [
    lambda: O.example1_operator(9),
    lambda: O.div_k((8, 5), W.kfield((8, 5), 4), beta=(60.0, 0.0)),
])
def test_transpose_adjoint_identity(make):
    op = make()
    rng = np.random.default_rng(3)
    x, y = rng.standard_normal(op.n), rng.standard_normal(op.n)
    lhs = O.apply(op, x) @ y
    rhs = x @ O.apply_transpose(op, y)
    assert abs(lhs - rhs) < 1e-12 * np.linalg.norm(O.apply(op, x)) * np.linalg.norm(y)


def test_example1_operator_rows():
    """Row of a node away from the boundary: -exp(5xy) times the 5-point
    Laplacian plus centred 40 u_x + 40 u_y, with x along the fast axis."""
    n = 9
    h = 1 / (n + 1)
    op = O.example1_operator(n)
    A = O.to_csr(op).toarray()
    i, j = 3, 6  # 1-based node: x = i h, y = j h
    p = (j - 1) * n + (i - 1)
    a = np.exp(5 * (i * h) * (j * h))
    assert np.isclose(A[p, p], 4 * a / h**2)
    assert np.isclose(A[p, p + 1], -a / h**2 + 20 / h)   # east: +40/(2h)
    assert np.isclose(A[p, p - 1], -a / h**2 - 20 / h)
    assert np.isclose(A[p, p + n], -a / h**2 + 20 / h)   # north
    assert np.isclose(A[p, p - n], -a / h**2 - 20 / h)


def test_coarsen_sizes_and_kcell():
    op = O.div_k((7, 7), W.kfield((7, 7), 1))
    opc = O.coarsen(op)
    assert opc.dims == (3, 3)
    k = op.params["kcell"]
    kc = opc.params["kcell"]
    assert kc.shape == (4, 4)
    assert np.isclose(kc[1, 2], (k[2, 4] * k[2, 5] * k[3, 4] * k[3, 5]) ** 0.25)
