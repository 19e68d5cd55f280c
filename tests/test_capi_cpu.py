"""CPU checks of the C-ABI boundary: the library loads, exports every symbol
the headers declare, its struct layouts match the ctypes mirrors, and the host
algebra it runs (eigen-decomposition, least squares, LU, QR) is correct."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")


def _lib():
    from paper_2005_03070_amd import _lib as L
    return L


def _declared():
    names = []
    for h in sorted(os.listdir(INCLUDE)):
        if h.endswith(".h"):
            txt = open(os.path.join(INCLUDE, h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"\b(tgdk_[a-z0-9_]+)\s*\(", txt)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = _lib()
    lib = L.lib()
    declared = _declared()
    assert len(declared) >= 25
    for name in declared:
        assert hasattr(lib, name), name
    # and the binding declares a signature for each of them
    assert sorted(n for n, _, _ in L.SIGNATURES) == declared


def test_struct_layouts_match_header(tmp_path):
    src = tmp_path / "sizes.c"
    src.write_text('#include "tgdk.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n", sizeof(tgdk_op_desc),'
                   ' sizeof(tgdk_gmresdr_params), sizeof(tgdk_gmresdr_report), sizeof(tgdk_solve_params),'
                   ' sizeof(tgdk_solve_report), offsetof(tgdk_solve_report, first_rho),'
                   ' offsetof(tgdk_gmresdr_report, seconds), offsetof(tgdk_solve_params, nu0),'
                   ' offsetof(tgdk_solve_params, icyc0), offsetof(tgdk_solve_report, cycle_branch),'
                   ' offsetof(tgdk_solve_report, vops)); return 0;}\n')
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-I", INCLUDE, str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    L = _lib()
    want = [C.sizeof(L.OpDesc), C.sizeof(L.GmresDrParams), C.sizeof(L.GmresDrReport), C.sizeof(L.SolveParams),
            C.sizeof(L.SolveReport), L.SolveReport.first_rho.offset, L.GmresDrReport.seconds.offset,
            L.SolveParams.nu0.offset, L.SolveParams.icyc0.offset, L.SolveReport.cycle_branch.offset,
            L.SolveReport.vops.offset]
    assert got == want


def test_context_creation_fails_cleanly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    L = _lib()
    h = C.c_void_p()
    rc = L.lib().tgdk_ctx_create(C.byref(h), 0, None)
    assert rc == L.E_HIP and b"device" in L.lib().tgdk_last_error()


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


@pytest.mark.parametrize("n,seed", [(5, 0), (30, 1), (81, 2)])
def test_host_eig_matches_numpy(n, seed):
    """Eigenpairs of random nonsymmetric matrices (complex pairs included):
    A x = w x for every returned pair and the eigenvalues match numpy."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    a, ap = _d(A)
    wr, wrp = _d(np.zeros(n))
    wi, wip = _d(np.zeros(n))
    Xr, Xrp = _d(np.zeros(n * n))
    Xi, Xip = _d(np.zeros(n * n))
    assert _lib().lib().tgdk_host_eig(n, ap, wrp, wip, Xrp, Xip) == 0
    w = wr + 1j * wi
    X = (Xr + 1j * Xi).reshape(n, n).T
    ref = np.linalg.eigvals(A)
    for v in w:
        assert np.min(np.abs(ref - v)) <= 1e-9 * np.abs(ref).max()
    for v in ref:
        assert np.min(np.abs(w - v)) <= 1e-9 * np.abs(ref).max()
    res = np.linalg.norm(A @ X - X * w[None, :], axis=0)
    assert res.max() <= 1e-10 * np.linalg.norm(A)
    assert np.allclose(np.linalg.norm(X, axis=0), 1.0)


def test_host_eig_hessenberg_like_harmonic_matrix():
    """The harmonic Ritz matrix shape: upper Hessenberg plus a rank-one last
    column update, with clustered eigenvalues."""
    rng = np.random.default_rng(4)
    m = 40
    H = np.triu(rng.standard_normal((m, m)), -1) + np.diag(np.linspace(1, 2, m)) * 50
    f = rng.standard_normal(m)
    M = H.copy()
    M[:, -1] += f
    a, ap = _d(M)
    wr, wrp = _d(np.zeros(m))
    wi, wip = _d(np.zeros(m))
    assert _lib().lib().tgdk_host_eig(m, ap, wrp, wip, None, None) == 0
    ref = np.linalg.eigvals(M)
    for v in wr + 1j * wi:
        assert np.min(np.abs(ref - v)) <= 1e-8 * np.abs(ref).max()


def test_host_lstsq_and_lu_and_qr():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((31, 30))
    b = rng.standard_normal(31)
    a, ap = _d(A)
    bb, bp = _d(b)
    x, xp = _d(np.zeros(30))
    r, rp = _d(np.zeros(31))
    L = _lib().lib()
    assert L.tgdk_host_lstsq(31, 30, ap, bp, xp, rp) == 0
    xr, *_ = np.linalg.lstsq(A, b, rcond=None)
    np.testing.assert_allclose(x, xr, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(r, b - A @ x, atol=1e-12)
    S = rng.standard_normal((12, 12))
    s, sp = _d(S)
    c, cp = _d(rng.standard_normal(12))
    c0 = c.copy()
    assert L.tgdk_host_lu_solve(12, sp, cp) == 0
    np.testing.assert_allclose(S @ c, c0, atol=1e-10)
    Z, zp = _d(np.zeros((3, 3)))
    assert L.tgdk_host_lu_solve(3, zp, _d(np.ones(3))[1]) == _lib().E_SINGULAR
    Q, qp = _d(np.zeros((31, 30)))
    R, rp2 = _d(np.zeros((30, 30)))
    assert L.tgdk_host_qr(31, 30, ap, qp, rp2) == 0
    np.testing.assert_allclose(Q @ R, A, atol=1e-12)
    assert np.all(np.diag(R) >= 0) and np.allclose(np.tril(R, -1), 0)
    np.testing.assert_allclose(Q.T @ Q, np.eye(30), atol=1e-12)


def test_host_eig_near_defective_stays_finite():
    """Near-defective matrices (a Jordan-like chain of nearly equal
    eigenvalues, as harmonic Ritz matrices become once pairs converge twice):
    eigenvectors must stay finite and unit-norm."""
    rng = np.random.default_rng(7)
    for n in (12, 30, 60):
        J = np.diag(np.full(n, 5.0) + 1e-13 * rng.standard_normal(n)) + np.diag(np.full(n - 1, 1e3), 1)
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        M = Q @ J @ Q.T
        a, ap = _d(M)
        wr, wrp = _d(np.zeros(n))
        wi, wip = _d(np.zeros(n))
        Xr, Xrp = _d(np.zeros(n * n))
        Xi, Xip = _d(np.zeros(n * n))
        assert _lib().lib().tgdk_host_eig(n, ap, wrp, wip, Xrp, Xip) == 0
        X = (Xr + 1j * Xi).reshape(n, n)
        assert np.all(np.isfinite(X))
        assert np.allclose(np.linalg.norm(X, axis=1), 1.0)


def test_host_qr_tiny_and_huge_columns():
    """Columns scaled by 1e-160 and 1e+150 (the GMRES-DR least-squares
    residual shrinks toward the subnormal range once the coarse system has
    converged): Q stays finite and orthonormal, Q R reproduces A."""
    rng = np.random.default_rng(9)
    A = rng.standard_normal((31, 11))
    A[:, 10] *= 1e-160
    A[:, 3] *= 1e150
    a, ap = _d(A)
    Q, qp = _d(np.zeros((31, 11)))
    R, rp = _d(np.zeros((11, 11)))
    assert _lib().lib().tgdk_host_qr(31, 11, ap, qp, rp) == 0
    assert np.all(np.isfinite(Q)) and np.all(np.isfinite(R))
    np.testing.assert_allclose(Q.T @ Q, np.eye(11), atol=1e-12)
    for j in range(11):
        np.testing.assert_allclose(Q @ R[:, j], A[:, j], rtol=0, atol=1e-12 * np.abs(A[:, j]).max())
