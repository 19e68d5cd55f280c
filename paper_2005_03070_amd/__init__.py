"""tgdk: two-grid deflated Krylov solvers for MI355X (gfx950).

The fine-grid hot path of Morgan, Whyte, Wilcox and Yang's two-grid deflated
Krylov method (arXiv 2005.03070) as a HIP library (libtgdk.so, C-ABI in
include/tgdk.h) with a thin Python binding.
"""
from . import _lib
from .api import (DeflationSpace, Multigrid, Operator, Report, SetupReport, coarse_setup, context, defl_from_basis,
                  defl_prolongate, grad_k, prolongate, restrict, solve, solve_idr, solve_instances, solve_noalloc,
                  stream_probe)
from .autograd import DeflatedSolve, TwoGridSolver

__all__ = ["Operator", "DeflationSpace", "Multigrid", "Report", "SetupReport", "coarse_setup", "context", "defl_from_basis",
           "defl_prolongate", "grad_k", "prolongate", "restrict", "solve", "solve_idr", "solve_instances", "solve_noalloc",
           "stream_probe",
           "DeflatedSolve",
           "TwoGridSolver"]
