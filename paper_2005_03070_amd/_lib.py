"""ctypes declarations of the tgdk C-ABI (include/tgdk.h, include/tgdk_host.h).

Argument marshalling only: every step of the solver runs in libtgdk.so.
Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtgdk.so")

OK, E_INVALID, E_NOMEM, E_HIP, E_SINGULAR, E_NONFINITE = 0, -1, -2, -3, -4, -5
NOT_CONVERGED, BREAKDOWN = 1, 2
F64, F32 = 0, 1
CONST_CD, VAR_STENCIL, DIV_K = 0, 1, 2
BICGSTAB_PROJ, GMRES_PROJ, IDRS_PROJ = 0, 1, 2
PROJ_GALERKIN, PROJ_MINRES = 0, 1
FP64, FP32_IR = 0, 1
MAX_DEFL = 256
NHIST = 8
IDR_SMAX = 32
NCYC_REPORT = 64

STATUS_NAMES = {OK: "ok", NOT_CONVERGED: "not_converged", BREAKDOWN: "breakdown",
                E_INVALID: "invalid", E_NOMEM: "nomem", E_HIP: "hip", E_SINGULAR: "singular",
                E_NONFINITE: "nonfinite"}


class OpDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("kind", C.c_int),
                ("beta", C.c_double * 3), ("sigma", C.c_double), ("coef", C.c_void_p)]


class GmresDrParams(C.Structure):
    _fields_ = [("m", C.c_int), ("k", C.c_int), ("nev", C.c_int), ("maxcyc", C.c_int),
                ("transpose", C.c_int), ("rtolev", C.c_double), ("rtol", C.c_double),
                ("precond", C.c_void_p), ("precond_user", C.c_void_p)]


class GmresDrReport(C.Structure):
    _fields_ = [("cycles", C.c_int), ("nconv", C.c_int), ("k_out", C.c_int),
                ("mvps", C.c_longlong), ("relres", C.c_double),
                ("theta_re", C.c_double * (MAX_DEFL + 1)), ("theta_im", C.c_double * (MAX_DEFL + 1)),
                ("eigres", C.c_double * (MAX_DEFL + 1)), ("seconds", C.c_double)]


class ArnoldiEParams(C.Structure):
    _fields_ = [("m", C.c_int), ("nev", C.c_int), ("maxcyc", C.c_int), ("tol", C.c_double)]


class ArnoldiEReport(C.Structure):
    _fields_ = [("cycles", C.c_int), ("nconv", C.c_int), ("k_out", C.c_int), ("mvps", C.c_longlong),
                ("theta_re", C.c_double * (MAX_DEFL + 1)), ("theta_im", C.c_double * (MAX_DEFL + 1)),
                ("eigres", C.c_double * (MAX_DEFL + 1)), ("eigres_start", C.c_double * (MAX_DEFL + 1)),
                ("seconds", C.c_double)]


class SolveParams(C.Structure):
    _fields_ = [("method", C.c_int), ("ncyc", C.c_int), ("m3", C.c_int), ("precision", C.c_int),
                ("x0_given", C.c_int), ("transpose", C.c_int), ("maxit_cycle", C.c_int),
                ("max_extra_cycles", C.c_int), ("rtol", C.c_double), ("fp32_floor", C.c_double),
                ("cycle_lengths", C.POINTER(C.c_int)), ("n_cycle_lengths", C.c_int),
                ("precond", C.c_void_p), ("precond_user", C.c_void_p),
                ("icyc0", C.c_int), ("max_cycles_call", C.c_int), ("nu0", C.c_double)]


class SolveReport(C.Structure):
    _fields_ = [("status", C.c_int), ("cycles", C.c_int), ("iters_inner", C.c_longlong),
                ("mvp_inner", C.c_longlong), ("mvp_boundary", C.c_longlong),
                ("relres_true", C.c_double), ("seconds", C.c_double), ("branch", C.c_int * 4),
                ("n_first", C.c_int), ("first_rho", C.c_double * NHIST),
                ("first_alpha", C.c_double * NHIST), ("first_omega", C.c_double * NHIST),
                ("n_cycle_mvps", C.c_int), ("cycle_mvps", C.c_int * NCYC_REPORT),
                ("cycle_branch", C.c_int * NCYC_REPORT), ("nu0", C.c_double),
                ("mvp_setup", C.c_longlong), ("vops", C.c_longlong)]


P = C.c_void_p
PP = C.POINTER(C.c_void_p)
I = C.c_int
D = C.c_double
DP = C.POINTER(C.c_double)

# (name, restype, argtypes) for every entry point of include/tgdk.h
SIGNATURES = [
    ("tgdk_last_error", C.c_char_p, []),
    ("tgdk_ctx_create", I, [PP, I, P]),
    ("tgdk_ctx_destroy", I, [P]),
    ("tgdk_ctx_num_cus", I, [P]),
    ("tgdk_ctx_time_kernel", I, [P, I]),
    ("tgdk_ctx_kernel_time", I, [P, I, DP, C.POINTER(C.c_longlong)]),
    ("tgdk_stream_probe", I, [P, I, I, I, C.POINTER(C.c_int), I, I, DP]),
    ("tgdk_op_create", I, [P, C.POINTER(OpDesc), PP]),
    ("tgdk_op_coarsen", I, [P, PP]),
    ("tgdk_op_apply", I, [P, I, I, P, P, I]),
    ("tgdk_op_info", I, [P, C.POINTER(I), C.POINTER(I), C.POINTER(C.c_longlong)]),
    ("tgdk_op_destroy", I, [P]),
    ("tgdk_prolongate", I, [P, P, I, P, P, I]),
    ("tgdk_restrict", I, [P, P, I, P, P, I]),
    ("tgdk_coarse_setup", I, [P, P, P, C.POINTER(GmresDrParams), PP, C.POINTER(GmresDrReport)]),
    ("tgdk_defl_prolongate", I, [P, P, I, PP]),
    ("tgdk_defl_from_basis", I, [P, P, I, I, I, PP]),
    ("tgdk_mg_create", I, [P, I, I, I, PP]),
    ("tgdk_mg_apply", I, [P, P, P, I]),
    ("tgdk_mg_levels", I, [P]),
    ("tgdk_mg_destroy", I, [P]),
    ("tgdk_defl_improve", I, [P, C.POINTER(ArnoldiEParams), I, PP, C.POINTER(ArnoldiEReport)]),
    ("tgdk_defl_minres", I, [P, PP]),
    ("tgdk_defl_precond", I, [P, P, P, PP]),
    ("tgdk_defl_projection", I, [P]),
    ("tgdk_defl_info", I, [P, C.POINTER(I), C.POINTER(I), C.POINTER(C.c_longlong)]),
    ("tgdk_defl_copy", I, [P, P, DP]),
    ("tgdk_defl_destroy", I, [P]),
    ("tgdk_solve", I, [P, P, P, P, I, C.POINTER(SolveParams), C.POINTER(SolveReport)]),
    ("tgdk_solve_noalloc", I, [P, P, P, P, I, C.POINTER(SolveParams), C.POINTER(SolveReport)]),
    ("tgdk_solve_idr", I, [P, P, P, P, I, P, D, C.POINTER(SolveParams), C.POINTER(SolveReport)]),
    ("tgdk_solve_instances", I, [P, I, PP, PP, PP, PP, C.POINTER(SolveParams), C.POINTER(SolveReport)]),
    ("tgdk_adjoint_grad_k", I, [P, P, P, P]),
    ("tgdk_tune", I, [P, P, I, I, C.POINTER(I)]),
    # include/tgdk_host.h
    ("tgdk_host_eig", I, [I, DP, DP, DP, DP, DP]),
    ("tgdk_host_lstsq", I, [I, I, DP, DP, DP, DP]),
    ("tgdk_host_lu_solve", I, [I, DP, DP]),
    ("tgdk_host_qr", I, [I, I, DP, DP, DP]),
]

_lib = None


class TgdkError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tgdk error {code} ({STATUS_NAMES.get(code, code)}): {msg}")
        self.code = code


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} not found: the HIP library is not built "
                "(run `python -c 'import __graft_entry__ as g; g.build()'` at the repository root)")
        L = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc, allow_soft=True):
    """Raise on a hard error; return the code otherwise."""
    if rc < 0 or (rc > 0 and not allow_soft):
        raise TgdkError(rc, lib().tgdk_last_error().decode(errors="replace"))
    return rc
