// Multigrid level descriptions shared by the host walker (mg.cpp) and the
// multigrid kernels (kernels_mg.hip).
#pragma once

namespace tgdk {

// One grid level: sides (nz = 1 in 2-D), the constant stencil C, W, E, S, N,
// D, U (zero Dirichlet data outside the grid) and the damped-Jacobi factor
// omega / C.
struct MgLvl {
    int nx, ny, nz, pad_;
    double cc[7];
    double sc;
};

// The coarse tail of a hierarchy that one workgroup runs in LDS: levels
// lv[0] (the tail's finest) .. lv[nlev-1] (the coarsest); each level's z, v
// and sweep temporary t at zoff / voff / toff (doubles into the LDS array).
constexpr int MG_TAIL_MAXLEV = 12;
constexpr int MG_TAIL_LDS = 6144;   // doubles (48 KiB)
constexpr int MG_TAIL_NT = 1024;

// Levels wave_from .. nlev-1 have at most 64 points each: one wave runs
// them, ordered by wave-level fences instead of workgroup barriers.
struct MgTail {
    int dim, nlev, nu, coarsest_sweeps;
    int wave_from, pad_;
    int zoff[MG_TAIL_MAXLEV], voff[MG_TAIL_MAXLEV], toff[MG_TAIL_MAXLEV];
    MgLvl lv[MG_TAIL_MAXLEV];
};

// What one pass computes at a point of a level (s: the Jacobi factor):
//  FIRST   s v                              (the first sweep from z = 0)
//  FIRST2  z1 + s (v - A z1), z1 = s v      (the first two sweeps from z = 0)
//  SWEEP   z + s (v - A z)
//  PSWEEP  z' + s (v - A z'), z' = z + P zc (coarse correction, then a sweep)
//  RESID   v - A z
// with MG_ACC added, the pass adds its value to the output instead.
enum : int { MG_FIRST = 0, MG_FIRST2 = 1, MG_SWEEP = 2, MG_PSWEEP = 3, MG_RESID = 4, MG_ACC = 8 };

}  // namespace tgdk
