// Plain structs shared by host code and kernels.
#pragma once

#include <stdint.h>

namespace tgdk {

constexpr int MAXK = 128;   // largest deflation space / GMRES cycle length
constexpr int NHIST = 8;    // recorded first BiCGStab scalars
constexpr int NCYCLOG = 512;  // cycles whose inner iteration counts are logged

// An operator as the kernels see it (passed by value or inside DevProb).
struct DevOp {
    int dim, nx, ny, nz;
    long long n;
    int var;                 // 1: per-row coefficient arrays
    int pad_;
    double cc[7];            // constant coefficients C, W, E, S, N, D, U
    const double* coef64;    // var: (2*dim+1) arrays of n, same order
    const float* coef32;
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
enum : int { SV_RUNNING = 0, SV_CONVERGED = 1, SV_BREAKDOWN = 2, SV_NOT_CONVERGED = 3 };
enum : int { METHOD_BICGSTAB = 0, METHOD_GMRES = 1 };

// Per-problem solver state in device memory.  Scalars are float64.
struct SolveState {
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
    double hist[3 * NHIST];
    int cyc_iters[NCYCLOG];  // inner iterations of each finished cycle
    int cyc_end[NCYCLOG];    // inner state that ended it
    double d[MAXK + 1];      // projection coefficients (H d = c)
    double cvec[MAXK + 1];
};

// Host-visible status mirror (in host-mapped memory).
struct Mirror {
    int solve_state, inner_state, icyc, iter;
    double rr;       // estimate of ||r_inner||^2 after the last iteration
    double rr0;      // ||r_inner||^2 at the start of the cycle
    double target2;  // squared target of the cycle
};

// One problem of a grouped launch.  All pointers are device pointers.
struct DevProb {
    DevOp op;
    int tx, ty, tz, ntiles, tile_begin;
    int k;
    const double* b;
    double* x;
    double* r;               // outer residual, float64
    void* rin;               // inner residual (aliases r in float64 mode)
    void* rhat;
    void* p[2];
    void* v[2];
    void* s;
    void* t;
    void* e;
    const void* V;           // deflation basis, column-major, leading dim ldv
    long long ldv;
    const double* lu;        // LU factors of H (k x k, row-major), pivots
    const int* piv;
    SolveState* st;
    double* partial;         // ntiles * pstride
    int pstride;
    unsigned* counter;
    Mirror* mirror;
    // systems that share one deflation space (several right-hand sides): the
    // projection runs as matrix-core products over the block of residuals
    const double* Ccol;      // column of C = V^T R (k values), or null
    double* Dcol;            // column of D (k values): this system's d
    const double* Wcol;      // column of W = V D (n values), or null
};

}  // namespace tgdk
