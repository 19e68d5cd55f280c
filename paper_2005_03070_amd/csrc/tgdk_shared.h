// Plain structs shared by host code and kernels.
#pragma once

#include <stdint.h>

namespace tgdk {

constexpr int MAXK = 256;   // largest deflation space / GMRES cycle length
constexpr int NHIST = 8;    // recorded first BiCGStab scalars
constexpr int NCYCLOG = 512;  // cycles whose inner iteration counts are logged
constexpr int NTILE_IDS = 4;  // tile shapes of the grid kernels (ids 0..3)

// An operator as the kernels see it (passed by value or inside DevProb).
struct DevOp {
    int dim, nx, ny, nz;
    long long n;
    int var;                 // 1: per-row coefficient arrays
    int px;                  // row pitch (x stride of y) of the step kernel's own vectors, >= nx; caller
                             // vectors (x, b), the deflation basis and coefficient arrays have pitch nx
    double cc[7];            // constant coefficients C, W, E, S, N, D, U
    const double* coef64;    // var: (2*dim+1) arrays of n, same order
    const float* coef32;
    const void* zero;        // 4 KiB of zeros (loads of out-of-domain points read here)
};

// inner cycle state
enum : int {
    IN_RUNNING = 0,
    IN_CONVERGED = 1,     // full step, ||r|| <= target (update alpha p + omega s pending)
    IN_HALF = 2,          // half step, ||s|| <= target (update alpha p pending)
    IN_BREAK_NOUPD = 3,   // breakdown, no pending update (rho or r^.v)
    IN_BREAK_FULL = 4,    // breakdown after a full step (omega or next rho)
    IN_MAXIT = 5,         // iteration limit (full update pending)
};
// solve state
enum : int { SV_RUNNING = 0, SV_CONVERGED = 1, SV_BREAKDOWN = 2, SV_NOT_CONVERGED = 3, SV_NONFINITE = 4 };
enum : int { METHOD_BICGSTAB = 0, METHOD_GMRES = 1, METHOD_IDR = 2 };

// BiCGStab step kernel: what the next launch does for a problem (StepHot::mode)
enum : int {
    M_DONE = 0,
    M_RES = 1,      // cycle end or solve start: true residual (+ c partials)
    M_A = 2,        // phase A of the next iteration (phase B partials pending)
    M_B = 3,        // phase B (phase A partials pending)
    M_REDUCE = 4,   // boundary decisions; c summed and H d = c solved
    M_APPLY = 5,    // x += upd + V d, r -= A V d, new shadow vector
    M_START = 6,    // decisions after the projection, then phase A of iteration 0
    M_APPLY0 = 7,   // no deflation: decisions, x += upd, phase A of iteration 0
    M_APPLYW = 8,   // 3-D: w = V d, x += upd + w (then M_APPLY: r -= A w)
    M_SUMC = 9,     // 3-D, float64 V: c summed and H d = c solved (the c partials came from ACT_CDOT)
};
// ... and what a launch did for it (logged for measurement)
enum : int {
    ACT_NONE = 0,
    ACT_A = 1,       // phase A of an iteration > 0
    ACT_A0 = 2,      // phase A of iteration 0
    ACT_B = 3,       // phase B
    ACT_RES = 4,     // true residual at the end of a cycle (or at the start)
    ACT_REDUCE = 5,  // projection coefficients (one workgroup)
    ACT_APPLY = 6,   // projection applied
    ACT_FIN = 7,     // last inner update folded into x
    ACT_FIN_A0 = 8,  // x update and phase A of iteration 0 (no deflation)
    ACT_APPLYW = 9,  // 3-D: w = V d and x += upd + w (the stencil part follows as ACT_APPLY)
    ACT_CDOT = 10,   // 3-D, float64 V: c = V^T r partials over contiguous ranges (after the boundary decisions)
    NACT = 11,
};

// Scalars of the step kernel's state machine, double-buffered by launch
// parity: launch s reads hot[(s + 1) & 1] and its lead workgroup writes
// hot[s & 1].
struct StepHot {
    int mode, solve_state, inner_state, first;
    int iter, icyc, pbuf, upd_any;
    double rho, rho_old, alpha, omega;
    double target2, tau, nu0, bnorm;
    double upd_a, upd_w;  // coefficients of p and s in the pending x update
};

// Per-problem solver state in device memory.  Scalars are float64.
struct SolveState {
    StepHot hot[2];
    double rho, rho_old, alpha, omega, sigma;
    double target2;          // (relative tolerance * nu)^2 of the inner cycle
    double nu, nu0, tau, bnorm;
    double rt;               // last cycle tolerance
    double rtol, fp32_floor;
    double rr_last;          // last exact ||r_inner||^2 seen by phase A
    double nu_final;         // true residual norm of the final check
    int icyc, ncyc, max_extra, maxit;
    int iter;                // completed inner iterations this cycle
    int inner_state, solve_state;
    int method, k, precision;
    int pbuf;                // buffer holding the last p (iteration parity)
    int last_inner_iters;    // iterations of the cycle that just ended
    int nhist;
    int branch[4];
    long long iters_total, mvp_inner, mvp_boundary;
    long long nproj;         // projections applied (each one boundary operator application)
    double hist[3 * NHIST];
    int cyc_iters[NCYCLOG];  // inner iterations of each finished cycle
    int cyc_end[NCYCLOG];    // inner state that ended it
    int cyc_branch[NCYCLOG];  // cycle tolerance criterion of each started cycle (1, 2, 3)
    int icyc0;               // cycles completed by earlier calls (resume); the first cycle here is icyc0 + 1
    int maxcyc_call;         // > 0: stop after this many cycles in this call
    double nu0_in;           // > 0: the initial residual norm of the resumed solve
    double d[MAXK + 1];      // projection coefficients (H d = c)
    double cvec[MAXK + 1];
};

// Host-visible status mirror (in host-mapped memory).
struct Mirror {
    int solve_state, inner_state, icyc, iter;
    int mode, slot;  // step kernel: state after launch number slot
    double rr;       // estimate of ||r_inner||^2 after the last iteration
    double rr0;      // ||r_inner||^2 at the start of the cycle
    double target2;  // squared target of the cycle
};

// One problem of a grouped launch.  All pointers are device pointers.
struct DevProb {
    DevOp op;
    int tx, ty, tz, ntiles, tile_begin;
    int k;
    int maxit;               // step kernel: inner iteration cap (the state's maxit)
    const double* b;
    double* x;
    double* r;               // outer residual, float64
    void* rin;               // inner residual (aliases r in float64 mode)
    void* rhat;
    void* p[2];
    void* v[2];
    void* r2[2];             // the inner residual r_i, double-buffered with p and v (s = r_i - alpha v_i is
                             // formed where needed, never stored)
    void* t;
    void* e;
    const void* V;           // deflation basis, column-major, leading dim ldv
    const void* Vl;          // basis of c = Vl^T r: V (Galerkin) or A V (MinRes), same layout and type
    long long ldv;
    int vtype;               // V stored as 0 float64, 1 float32
    int mcx, mcy, mz, nchunks;  // 3-D step kernel: z-marching chunks (mcx x mcy columns, mz planes deep)
    double* w;               // 3-D with deflation: w = V d (n values)
    const double* lu;        // LU factors of H (k x k, row-major), pivots
    const int* piv;
    const double* hinv;      // H^{-1} (k x k, column-major)
    SolveState* st;
    double* partial;         // tile kernels: ntiles * pstride (tile-major);
                             // step kernel: two launch-parity slots of pstride * nwg (value-major)
    int pstride;
    int nwg, wg_begin;       // step kernel: workgroups of this problem, first workgroup id
    long long pslot;         // pstride * nwg
    unsigned char* actlog;   // step kernel: action per launch (first NSLOTLOG launches), or null
    unsigned long long* tstamp;  // step kernel: start/end stamp per launch and workgroup (first NTSLOG launches), or null
    unsigned* counter;
    Mirror* mirror;
};

constexpr int NSLOTLOG = 1 << 15;
constexpr int NTSLOG = 1 << 12;

}  // namespace tgdk
