"""Python binding of the tgdk C-ABI.

Tensors are torch CUDA(HIP) tensors; this module only checks shapes and
dtypes and passes device pointers and the current stream to libtgdk.so.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib as L
from ._lib import check, lib

_CTX = {}


def _stream_ptr(device):
    return torch.cuda.current_stream(device).cuda_stream


def context(device=None):
    """The tgdk context for a device and its current torch stream."""
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else torch.device(device).index or 0)
    key = (dev.index, _stream_ptr(dev))
    if key not in _CTX:
        h = C.c_void_p()
        check(lib().tgdk_ctx_create(C.byref(h), dev.index, C.c_void_p(key[1])))
        _CTX[key] = (h, dev)
    return _CTX[key]


def _ptr(t, dtype=torch.float64, numel=None, what="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{what} has {t.numel()} elements, expected {numel}")
    return C.c_void_p(t.data_ptr())


class Operator:
    """A discretised operator (see include/tgdk.h, tgdk_op_desc)."""

    def __init__(self, dims, kind=L.CONST_CD, beta=(0.0, 0.0, 0.0), sigma=0.0, coef=None, device=None,
                 _handle=None):
        self.ctx, self.device = context(device)
        self.dims = tuple(int(d) for d in dims)
        self.dim = len(self.dims)
        self.n = int(np.prod(self.dims))
        self.kind = kind
        self.beta = tuple(float(b) for b in beta) + (0.0,) * (3 - len(beta))
        self.sigma = float(sigma)
        self._keep = coef
        if _handle is not None:
            self.h = _handle
            return
        d = L.OpDesc()
        d.dim = self.dim
        for a in range(3):
            d.n[a] = self.dims[a] if a < self.dim else 1
            d.beta[a] = self.beta[a]
        d.kind = kind
        d.sigma = self.sigma
        d.coef = None
        if coef is not None:
            d.coef = _ptr(coef, what="coef")
        h = C.c_void_p()
        check(lib().tgdk_op_create(self.ctx, C.byref(d), C.byref(h)))
        self.h = h

    @classmethod
    def const_cd(cls, dims, beta=(0.0, 0.0, 0.0), sigma=0.0, device=None):
        return cls(dims, L.CONST_CD, beta, sigma, None, device)

    @classmethod
    def div_k(cls, dims, kcell, beta=(0.0, 0.0), sigma=0.0):
        kcell = kcell.contiguous()
        if tuple(kcell.shape) != (dims[1] + 1, dims[0] + 1):
            raise ValueError("kcell must have shape (n_y + 1, n_x + 1)")
        return cls(dims, L.DIV_K, beta, sigma, kcell, kcell.device)

    @classmethod
    def var_stencil(cls, dims, coef):
        """coef: (2*dim+1, n) tensor, rows C, W, E, S, N(, D, U)."""
        coef = coef.contiguous()
        return cls(dims, L.VAR_STENCIL, (0.0, 0.0, 0.0), 0.0, coef, coef.device)

    def coarsen(self):
        h = C.c_void_p()
        check(lib().tgdk_op_coarsen(self.h, C.byref(h)))
        cd = tuple((d - 1) // 2 for d in self.dims)
        return Operator(cd, self.kind, self.beta, self.sigma, None, self.device, _handle=h)

    def apply(self, x, transpose=False):
        """y = A x (or A^T x) for x of shape (n,) or (nrhs, n)."""
        dt = L.F64 if x.dtype == torch.float64 else L.F32
        nrhs = 1 if x.dim() == 1 else x.shape[0]
        _ptr(x, x.dtype, self.n * nrhs, "x")
        y = torch.empty_like(x)
        check(lib().tgdk_op_apply(self.h, int(transpose), dt, C.c_void_p(x.data_ptr()),
                                  C.c_void_p(y.data_ptr()), nrhs))
        return y

    def tune(self, dtype=torch.float64, nrhs=1):
        ty = C.c_int()
        check(lib().tgdk_tune(self.ctx, self.h, L.F64 if dtype == torch.float64 else L.F32, nrhs, C.byref(ty)))
        return ty.value

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None and L._lib is not None:
                lib().tgdk_op_destroy(self.h)
                self.h = None
        except Exception:
            pass


def prolongate(coarse, fine, vc):
    ncols = 1 if vc.dim() == 1 else vc.shape[0]
    _ptr(vc, numel=coarse.n * ncols, what="vc")
    vf = torch.empty((fine.n,) if vc.dim() == 1 else (ncols, fine.n), dtype=torch.float64, device=vc.device)
    check(lib().tgdk_prolongate(coarse.h, fine.h, L.F64, C.c_void_p(vc.data_ptr()), C.c_void_p(vf.data_ptr()),
                                ncols))
    return vf


def restrict(fine, coarse, vf):
    ncols = 1 if vf.dim() == 1 else vf.shape[0]
    _ptr(vf, numel=fine.n * ncols, what="vf")
    vc = torch.empty((coarse.n,) if vf.dim() == 1 else (ncols, coarse.n), dtype=torch.float64, device=vf.device)
    check(lib().tgdk_restrict(fine.h, coarse.h, L.F64, C.c_void_p(vf.data_ptr()), C.c_void_p(vc.data_ptr()),
                              ncols))
    return vc


class DeflationSpace:
    def __init__(self, handle, op, transpose):
        self.h = handle
        self.op = op
        self.transpose = transpose
        k, st, n = C.c_int(), C.c_int(), C.c_longlong()
        check(lib().tgdk_defl_info(handle, C.byref(k), C.byref(st), C.byref(n)))
        self.k, self.store, self.n = k.value, st.value, n.value
        self.projection = "minres" if lib().tgdk_defl_projection(handle) == L.PROJ_MINRES else "galerkin"

    def precond(self, mg):
        """The space for right-preconditioned solves with M^{-1} = mg: c = V^T r,
        H = V^T A M^{-1} V, update with Z = M^{-1} V (tgdk_defl_precond)."""
        fn, user = _precond(mg)
        h = C.c_void_p()
        check(lib().tgdk_defl_precond(self.h, C.c_void_p(fn), C.c_void_p(user), C.byref(h)))
        return DeflationSpace(h, self.op, self.transpose)

    def minres(self):
        """The MinRes-projection space over the same V: H = (AV)^T AV and
        c = (AV)^T r (see include/tgdk.h, tgdk_defl_minres)."""
        h = C.c_void_p()
        check(lib().tgdk_defl_minres(self.h, C.byref(h)))
        return DeflationSpace(h, self.op, self.transpose)

    def improve(self, m, nev=None, tol=1e-8, maxcyc=100, store=torch.float64):
        """Arnoldi-E(m, k) improvement of the space's vectors on its grid (see
        include/tgdk.h, tgdk_defl_improve).  Returns (improved space, report
        dict with cycles, nconv, k_out, mvps, theta, eigres, eigres_start)."""
        p = L.ArnoldiEParams(m, self.k if nev is None else nev, maxcyc, tol)
        r = L.ArnoldiEReport()
        h = C.c_void_p()
        check(lib().tgdk_defl_improve(self.h, C.byref(p), L.F64 if store == torch.float64 else L.F32, C.byref(h),
                                      C.byref(r)))
        nk = r.k_out
        cnt = min(len(r.theta_re), nk)
        theta = np.array([complex(r.theta_re[i], r.theta_im[i]) for i in range(cnt)])
        rep = {"cycles": r.cycles, "nconv": r.nconv, "k_out": nk, "mvps": r.mvps, "seconds": r.seconds,
               "theta": theta, "eigres": np.array(r.eigres[:cnt]),
               "eigres_start": np.array(r.eigres_start[:p.nev])}
        return DeflationSpace(h, self.op, self.transpose), rep

    def basis(self):
        """(V as a (k, n) float64 tensor, H as a k x k numpy array)."""
        V = torch.empty((self.k, self.n), dtype=torch.float64, device=self.op.device)
        H = np.zeros((self.k, self.k))
        check(lib().tgdk_defl_copy(self.h, C.c_void_p(V.data_ptr()), H.ctypes.data_as(L.DP)))
        return V, H

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None and L._lib is not None:
                lib().tgdk_defl_destroy(self.h)
                self.h = None
        except Exception:
            pass


@dataclass
class SetupReport:
    status: int
    cycles: int
    nconv: int
    k_out: int
    mvps: int
    relres: float
    theta: np.ndarray
    eigres: np.ndarray
    seconds: float


def _precond(pc):
    """(function pointer, user pointer) of a right preconditioner: a Multigrid."""
    if pc is None:
        return None, None
    if not isinstance(pc, Multigrid):
        raise TypeError("precond must be a Multigrid")
    return C.cast(lib().tgdk_mg_apply, C.c_void_p).value, pc.h.value


def coarse_setup(coarse, b_c, m, k, nev=None, rtolev=1e-8, rtol=1e-8, maxcyc=300, transpose=False, precond=None):
    """GMRES-DR(m,k) on the coarse grid (on A M^{-1} with a right
    preconditioner): returns (x_c, space, SetupReport)."""
    _ptr(b_c, numel=coarse.n, what="b_c")
    x_c = torch.empty_like(b_c)
    p = L.GmresDrParams(m, k, k if nev is None else nev, maxcyc, int(transpose), rtolev, rtol)
    p.precond, p.precond_user = _precond(precond)
    rep = L.GmresDrReport()
    h = C.c_void_p()
    rc = check(lib().tgdk_coarse_setup(coarse.h, C.c_void_p(b_c.data_ptr()), C.c_void_p(x_c.data_ptr()),
                                       C.byref(p), C.byref(h), C.byref(rep)))
    kk = rep.k_out
    theta = np.array(rep.theta_re[:kk]) + 1j * np.array(rep.theta_im[:kk])
    sr = SetupReport(rc, rep.cycles, rep.nconv, kk, rep.mvps, rep.relres, theta, np.array(rep.eigres[:kk]),
                     rep.seconds)
    return x_c, DeflationSpace(h, coarse, transpose), sr


class Multigrid:
    """Geometric multigrid V-cycles for a constant-coefficient operator (see
    include/tgdk.h, tgdk_mg_create); usable as a right preconditioner."""

    def __init__(self, op, cycles=2, nu=2, graph=True):
        h = C.c_void_p()
        check(lib().tgdk_mg_create(op.h, cycles, nu, 0 if graph else 1, C.byref(h)))
        self.h, self.op = h, op
        self.levels = lib().tgdk_mg_levels(h)

    def apply(self, x):
        """M^{-1} x for x of shape (n,) or (nrhs, n), float64 on the device."""
        nrhs = 1 if x.dim() == 1 else x.shape[0]
        _ptr(x, numel=self.op.n * nrhs, what="x")
        y = torch.empty_like(x)
        check(lib().tgdk_mg_apply(self.h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), nrhs))
        return y

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None and L._lib is not None:
                lib().tgdk_mg_destroy(self.h)
                self.h = None
        except Exception:
            pass


def defl_prolongate(space, fine, store=torch.float64):
    h = C.c_void_p()
    check(lib().tgdk_defl_prolongate(space.h, fine.h, L.F64 if store == torch.float64 else L.F32, C.byref(h)))
    return DeflationSpace(h, fine, space.transpose)


def defl_from_basis(op, W, transpose=False, store=torch.float64):
    """W: (k, n) float64 tensor (k basis vectors, each contiguous)."""
    W = W.contiguous()
    k = W.shape[0]
    _ptr(W, numel=k * op.n, what="W")
    h = C.c_void_p()
    check(lib().tgdk_defl_from_basis(op.h, C.c_void_p(W.data_ptr()), k, int(transpose),
                                     L.F64 if store == torch.float64 else L.F32, C.byref(h)))
    return DeflationSpace(h, op, transpose)


@dataclass
class Report:
    status: int
    cycles: int
    iters_inner: int
    mvp_inner: int
    mvp_boundary: int
    relres_true: float
    seconds: float
    branch: list = field(default_factory=list)
    first_scalars: list = field(default_factory=list)
    cycle_mvps: list = field(default_factory=list)  # inner operator applications of the first cycles
    cycle_branch: list = field(default_factory=list)  # tolerance criterion of each of the first cycles
    nu0: float = 0.0       # ||r0|| of the schedule (pass back as nu0= to resume)
    mvp_setup: int = 0     # fine operator applications that built the deflation space
    vops: int = 0          # length-n vector operations of this call (the paper's cost model)

    @property
    def cost(self):
        """The paper's cost (Sec. 3, Example 1) without the nnz factor: the
        caller multiplies mvps by the operator's nonzeros per row."""
        return {"mvps": self.mvp_inner + self.mvp_boundary, "vops": self.vops}

    @property
    def status_name(self):
        return L.STATUS_NAMES.get(self.status, str(self.status))


def _params(method, ncyc, m3, precision, x0_given, transpose, maxit_cycle, max_extra, rtol, fp32_floor,
            icyc0=0, nu0=0.0, max_cycles_call=0):
    p = L.SolveParams()
    p.icyc0 = int(icyc0)
    p.nu0 = float(nu0)
    p.max_cycles_call = int(max_cycles_call)
    p.method = {"gmres": L.GMRES_PROJ, "idr": L.IDRS_PROJ}.get(method, L.BICGSTAB_PROJ)
    p.ncyc = ncyc
    p.m3 = m3
    p.precision = L.FP32_IR if precision == "fp32_ir" else L.FP64
    p.x0_given = int(x0_given)
    p.transpose = int(transpose)
    p.maxit_cycle = maxit_cycle
    if max_extra is None:
        max_extra = ncyc if method != "gmres" else 1000
    p.max_extra_cycles = max_extra
    p.rtol = rtol
    p.fp32_floor = fp32_floor
    return p


def _reports(reps):
    out = []
    for r in reps:
        fs = [(r.first_rho[i], r.first_alpha[i], r.first_omega[i]) for i in range(r.n_first)]
        out.append(Report(r.status, r.cycles, r.iters_inner, r.mvp_inner, r.mvp_boundary, r.relres_true,
                          r.seconds, list(r.branch), fs, [r.cycle_mvps[i] for i in range(r.n_cycle_mvps)],
                          [r.cycle_branch[i] for i in range(r.n_cycle_mvps)], r.nu0, r.mvp_setup, r.vops))
    return out


def solve(op, b, x0=None, defl=None, method="bicgstab", ncyc=20, m3=50, precision="fp64", rtol=1e-8,
          transpose=False, maxit_cycle=100000, max_extra=None, fp32_floor=1e-4, out=None, cycle_lengths=None,
          precond=None, icyc0=0, nu0=0.0, max_cycles_call=0):
    """Fine solve of A x = b (A^T x = b if transpose).  b: (n,) or (nrhs, n)
    float64.  cycle_lengths (GMRES): lengths of the first cycles, each in
    1..m3 (variable restarting).  icyc0, nu0, max_cycles_call: resuming at a
    cycle boundary (see include/tgdk.h, tgdk_solve_params).  Returns
    (x, [Report per right-hand side])."""
    nrhs = 1 if b.dim() == 1 else b.shape[0]
    _ptr(b, numel=op.n * nrhs, what="b")
    if out is None:
        out = torch.empty_like(b)
    _ptr(out, numel=op.n * nrhs, what="x")
    if x0 is not None:
        out.copy_(x0)
    p = _params(method, ncyc, m3, precision, x0 is not None, transpose, maxit_cycle, max_extra, rtol, fp32_floor,
                icyc0, nu0, max_cycles_call)
    if cycle_lengths is not None:
        lens = (C.c_int * len(cycle_lengths))(*[int(v) for v in cycle_lengths])
        p.cycle_lengths = C.cast(lens, C.POINTER(C.c_int))
        p.n_cycle_lengths = len(cycle_lengths)
    p.precond, p.precond_user = _precond(precond)
    reps = (L.SolveReport * nrhs)()
    check(lib().tgdk_solve(op.h, defl.h if defl is not None else None, C.c_void_p(b.data_ptr()),
                           C.c_void_p(out.data_ptr()), nrhs, C.byref(p), reps))
    return out, _reports(reps)


def solve_noalloc(op, b, x0=None, defl=None, ncyc=20, precision="fp64", rtol=1e-8, transpose=False,
                  maxit_cycle=100000, max_extra=None, fp32_floor=1e-4, out=None, icyc0=0, nu0=0.0,
                  max_cycles_call=0):
    """BiCGStab(ncyc)-Proj(k) through tgdk_solve_noalloc: the same solve as
    solve(method="bicgstab"), with the library's workspace in its fixed
    per-device scratch (no device allocation inside the call; `out` may be
    passed preallocated).  Returns (x, [Report per right-hand side])."""
    nrhs = 1 if b.dim() == 1 else b.shape[0]
    _ptr(b, numel=op.n * nrhs, what="b")
    if out is None:
        out = torch.empty_like(b)
    _ptr(out, numel=op.n * nrhs, what="x")
    if x0 is not None:
        out.copy_(x0)
    p = _params("bicgstab", ncyc, 0, precision, x0 is not None, transpose, maxit_cycle, max_extra, rtol, fp32_floor,
                icyc0, nu0, max_cycles_call)
    reps = (L.SolveReport * nrhs)()
    check(lib().tgdk_solve_noalloc(op.h, defl.h if defl is not None else None, C.c_void_p(b.data_ptr()),
                                   C.c_void_p(out.data_ptr()), nrhs, C.byref(p), reps))
    return out, _reports(reps)


def solve_idr(op, b, s=4, shadow=None, x0=None, defl=None, ncyc=20, precision="fp64", rtol=1e-8, kappa=0.7,
              transpose=False, maxit_cycle=100000, max_extra=None, fp32_floor=1e-4, seed=0, out=None, precond=None,
              icyc0=0, nu0=0.0, max_cycles_call=0):
    """IDR(s)(ncyc)-Proj(k) on A x = b (one right-hand side, b of shape (n,)
    float64).  shadow: (s, n) float64 device tensor, the raw columns of the
    shadow space (orthonormalised by the library); None draws s standard
    normal columns on the device from ``seed``.  Returns (x, Report)."""
    _ptr(b, numel=op.n, what="b")
    if shadow is None:
        gen = torch.Generator(device=b.device)
        gen.manual_seed(seed)
        shadow = torch.randn((s, op.n), dtype=torch.float64, device=b.device, generator=gen)
    if tuple(shadow.shape) != (s, op.n):
        raise ValueError(f"shadow must have shape ({s}, {op.n})")
    _ptr(shadow, numel=op.n * s, what="shadow")
    if out is None:
        out = torch.empty_like(b)
    _ptr(out, numel=op.n, what="x")
    if x0 is not None:
        out.copy_(x0)
    p = _params("idr", ncyc, 0, precision, x0 is not None, transpose, maxit_cycle, max_extra, rtol, fp32_floor,
                icyc0, nu0, max_cycles_call)
    p.precond, p.precond_user = _precond(precond)
    rep = L.SolveReport()
    check(lib().tgdk_solve_idr(op.h, defl.h if defl is not None else None, C.c_void_p(b.data_ptr()),
                               C.c_void_p(out.data_ptr()), s, C.c_void_p(shadow.data_ptr()), kappa, C.byref(p),
                               C.byref(rep)))
    return out, _reports([rep])[0]


def solve_instances(ops, defls, bs, x0s=None, ncyc=20, precision="fp64", rtol=1e-8, maxit_cycle=100000,
                    max_extra=None, fp32_floor=1e-4, outs=None):
    """Independent instances solved together (one launch per step covers all)."""
    ni = len(ops)
    if outs is None:
        outs = [torch.empty_like(b) for b in bs]
    for j in range(ni):
        _ptr(bs[j], numel=ops[j].n, what="b")
        if x0s is not None:
            outs[j].copy_(x0s[j])
    p = _params("bicgstab", ncyc, 0, precision, x0s is not None, False, maxit_cycle, max_extra, rtol, fp32_floor)
    ctx = ops[0].ctx
    oph = (C.c_void_p * ni)(*[o.h.value for o in ops])
    dh = (C.c_void_p * ni)(*[(d.h.value if d is not None else None) for d in defls]) if defls else None
    bp = (C.c_void_p * ni)(*[b.data_ptr() for b in bs])
    xp = (C.c_void_p * ni)(*[x.data_ptr() for x in outs])
    reps = (L.SolveReport * ni)()
    check(lib().tgdk_solve_instances(ctx, ni, oph, dh, bp, xp, C.byref(p), reps))
    return outs, _reports(reps)


def grad_k(op, lam, u):
    _ptr(lam, numel=op.n, what="lambda")
    _ptr(u, numel=op.n, what="u")
    g = torch.empty((op.dims[1] + 1, op.dims[0] + 1), dtype=torch.float64, device=u.device)
    check(lib().tgdk_adjoint_grad_k(op.h, C.c_void_p(lam.data_ptr()), C.c_void_p(u.data_ptr()),
                                    C.c_void_p(g.data_ptr())))
    return g


def stream_probe(pattern, nreads, nwrites, dims, blocks=768, reps=10, device=None):
    """Streaming ceiling for a mix of float64 streams (include/tgdk.h,
    tgdk_stream_probe): pattern "contiguous", "march", "tiled", "march_pf2" or
    "march_pf3" (the march with 2 or 3 planes of loads in flight); returns
    (ms per launch, bytes moved per launch)."""
    ctx, _ = context(device)
    d = (C.c_int * 3)(*[int(v) for v in dims])
    ms = C.c_double()
    check(lib().tgdk_stream_probe(ctx, {"contiguous": 0, "march": 1, "tiled": 2, "march_pf2": 3, "march_pf3": 4}[pattern], int(nreads), int(nwrites), d,
                                  int(blocks), int(reps), C.byref(ms)))
    nx, ny, nz = (int(v) for v in dims)
    pts = ((nx + 63) // 64 * 64 if pattern == "contiguous" else nx) * ny * nz
    return ms.value, (nreads + nwrites) * pts * 8
