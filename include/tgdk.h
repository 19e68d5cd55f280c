/*
 * tgdk -- two-grid deflated Krylov solvers for gfx950 (MI355X).
 *
 * C-ABI of the fine-grid hot path of the two-grid deflated Krylov method of
 * Morgan, Whyte, Wilcox and Yang, "Two-grid deflated Krylov methods for linear
 * equations" (arXiv 2005.03070).  The library solves A x = b (Sec. 1) for a
 * finite-difference PDE operator A on a fine grid, using approximate
 * eigenvectors computed on a coarse grid with GMRES-DR (Sec. 2.1) and moved to
 * the fine grid (Sec. 3), a Galerkin projection over them (Sec. 2.2), and
 * restarted BiCGStab with a projection before every cycle (Sec. 4.1,
 * "BiCGStab(ncyc)-Proj(k)") or GMRES(m)-Proj(k) (Sec. 2.2).
 *
 * Conventions for every entry point:
 *  - Vectors are caller-owned DEVICE memory (e.g. torch tensors), contiguous.
 *    A block of several vectors is column-major: vector j starts at
 *    ptr + j * n.  Right-hand sides and solutions are always float64.
 *  - Grid ordering is lexicographic with x fastest: point (i, j, l), 0-based,
 *    is element (l * n_y + j) * n_x + i.
 *  - Every call is ordered on the context's HIP stream.  Calls that return
 *    scalars or reports (solvers, setup) block the host until their work is
 *    complete; the others only enqueue work.
 *  - Return value: 0 OK; negative = hard error (outputs undefined, see
 *    tgdk_last_error()); positive = soft outcome, outputs valid (see the
 *    report).  Handles own their internal device workspaces.
 *    *_destroy(NULL) is a no-op.  Handles are not thread-safe.
 */
#ifndef TGDK_H
#define TGDK_H

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define TGDK_OK             0
#define TGDK_E_INVALID     -1   /* bad argument (sizes, pointers, kinds) */
#define TGDK_E_NOMEM       -2   /* device or host allocation failed */
#define TGDK_E_HIP         -3   /* a HIP runtime call failed */
#define TGDK_E_SINGULAR    -4   /* singular small matrix (H, Gram, Hessenberg) */
#define TGDK_E_NONFINITE   -5   /* NaN/Inf in an input or a residual */
#define TGDK_NOT_CONVERGED  1   /* tolerance not reached in the allowed cycles */
#define TGDK_BREAKDOWN      2   /* a Krylov breakdown stopped all progress */

/* element types */
#define TGDK_F64 0
#define TGDK_F32 1

/* operator kinds */
#define TGDK_CONST_CD    0  /* -Lap(u) + beta.grad(u) + sigma u, constant beta  */
#define TGDK_VAR_STENCIL 1  /* per-row coefficients C,W,E,S,N(,D,U) given       */
#define TGDK_DIV_K       2  /* 2-D -div(k grad u) + beta.grad(u) + sigma u,
                               k per primal cell                              */

/* solver methods and precisions */
#define TGDK_BICGSTAB_PROJ 0
#define TGDK_GMRES_PROJ    1
#define TGDK_IDRS_PROJ     2   /* tgdk_solve_idr only */
#define TGDK_FP64          0
#define TGDK_FP32_IR       1

#define TGDK_MAX_DEFL 256   /* largest GMRES(-DR) cycle length m and deflation space k (k < m for GMRES-DR) */
#define TGDK_NHIST    8     /* recorded BiCGStab scalars of the first iterations */
#define TGDK_IDR_SMAX 32    /* largest IDR shadow-space dimension s */
#define TGDK_NCYC_REPORT 64 /* cycles whose inner operator applications are reported */

/* A right preconditioner as the host-driven solvers call it: out = M^{-1} in
 * for nrhs device float64 vectors of n (column-major), enqueued on the
 * context's stream (or completed before returning); in and out do not alias.
 * Returns TGDK_OK or a negative code. */
typedef int (*tgdk_precond_fn)(void* user, const double* in, double* out, int nrhs);

/* Text of the last non-OK return on the calling thread ("" if none). */
const char* tgdk_last_error(void);

typedef struct tgdk_ctx_s*  tgdk_ctx;
typedef struct tgdk_op_s*   tgdk_op;
typedef struct tgdk_defl_s* tgdk_defl;

/* Context: a device and a HIP stream (hipStream_t passed as void*, e.g.
 * torch.cuda.current_stream().cuda_stream; NULL = the null stream).  The
 * stream is borrowed, not owned. */
int tgdk_ctx_create(tgdk_ctx* out, int device, void* hip_stream);
int tgdk_ctx_destroy(tgdk_ctx ctx);
/* Number of compute units of the context's device (for launch sizing). */
int tgdk_ctx_num_cus(tgdk_ctx ctx);
/* Measurement hook for the BiCGStab step kernel inside tgdk_solve /
 * tgdk_solve_instances (the first 4096 launches of a call): each launch's
 * duration is added to the total of what the group's first problem did in it.
 *  on = 2: durations from HIP timing events, one recorded on the context's
 *          stream before the first launch and one after every launch (the
 *          time between two events: the launch plus the gap before it);
 *  on = 1: durations from the device's constant-rate wall clock, last end
 *          minus first start of the first problem's workgroups;
 *  on = 0: off.
 * Every call clears the totals.  tgdk_ctx_kernel_time returns, for one action
 * (TGDK_STEP_*), the summed duration in ms of the launches in which the first
 * problem did it and their number; TGDK_STEP_ANY sums the launches in which it
 * did work, TGDK_STEP_ALL every launch (including those queued past the end of
 * its solve).  Actions: */
#define TGDK_STEP_NONE   0  /* nothing (the problem had finished, or another problem's launch) */
#define TGDK_STEP_A      1  /* phase A of iteration i > 0: r, e, p updates, v = A p, r^.v and ||r||^2 partials */
#define TGDK_STEP_A0     2  /* phase A of iteration 0 of a cycle (p = r) */
#define TGDK_STEP_B      3  /* phase B: s = r - alpha v, t = A s, five dot-product partials */
#define TGDK_STEP_RES    4  /* end of a cycle: r = b - A (x + update), ||r||^2 (2-D, and 3-D with a float32 V: and c = V^T r) partials */
#define TGDK_STEP_REDUCE 5  /* c summed and H d = c solved (one workgroup) */
#define TGDK_STEP_APPLY  6  /* x += update + V d, r -= A V d, new shadow vector (3-D: r -= A w only) */
#define TGDK_STEP_FIN    7  /* final update folded into x */
#define TGDK_STEP_FIN_A0 8  /* update folded into x and phase A of iteration 0 (no deflation) */
#define TGDK_STEP_APPLYW 9  /* 3-D: w = V d and x += update + w (APPLY then does r -= A w) */
#define TGDK_STEP_CDOT   10 /* 3-D with a float64 V: c = V^T r partials (after the boundary decisions; REDUCE follows) */
#define TGDK_STEP_ANY   -1
#define TGDK_STEP_ALL   -2
int tgdk_ctx_time_kernel(tgdk_ctx ctx, int on);
int tgdk_ctx_kernel_time(tgdk_ctx ctx, int action, double* total_ms, long long* launches);
/* Measurement utility, not a step of the method: the streaming rate a plain
 * kernel reaches with nreads read streams and nwrites write streams of
 * float64 (mixes 1+1, 3+1 and 6+4: a copy, the 3-D phase B, the 3-D phase A),
 * the ceilings the step kernel's phases are compared with.  The arrays are
 * dims[0] x dims[1] x dims[2] grids with the row pitch rounded up to 64 (as
 * the step kernel's own vectors), allocated and freed by the call.
 * pattern 0: each array walked grid-strided by `blocks` workgroups (copy
 * order); pattern 1: one workgroup per 64 x 8 column chunk walking its planes
 * (the marching phases' order, about `blocks` chunks, no LDS or stencil);
 * pattern 2: the same walk over arrays stored chunk by chunk, each chunk's
 * 64 x 8 plane one contiguous block (y padded to a multiple of 8 as well);
 * patterns 3 and 4: the march of pattern 1 with the loads of the next one or
 * two planes issued before a plane is stored (2 or 3 planes in flight).
 * Runs one untimed and `reps` timed launches on the context's stream;
 * *ms_per_launch = their average (HIP events).  Returns TGDK_E_INVALID for
 * other mixes or bad sizes, TGDK_E_NOMEM when the arrays do not fit. */
int tgdk_stream_probe(tgdk_ctx ctx, int pattern, int nreads, int nwrites, const int* dims, int blocks, int reps,
                      double* ms_per_launch);

/* ---------------------------------------------------------------- operators
 * The discretised operator of Sec. 1 / Sec. 3 Example 1: centred finite
 * differences on the interior grid n[0] x n[1] (x n[2]) of the unit square
 * (cube) with zero Dirichlet data, h_a = 1/(n[a]+1), matrix not scaled by h^2.
 * Row p of A x is C_p x_p + sum over neighbours q of c_{q-p}(p) x_q; neighbours
 * outside the domain are dropped.
 *  - CONST_CD: C = sum_a 2/h_a^2 + sigma; along axis a the lower neighbour
 *    has -1/h_a^2 - beta[a]/(2h_a), the upper -1/h_a^2 + beta[a]/(2h_a).
 *  - VAR_STENCIL: coef is a device array of (2*dim+1)*n float64, the arrays
 *    C, W, E, S, N (, D, U) one after the other (W/E = x-1/x+1, S/N = y-1/y+1,
 *    D/U = z-1/z+1).  Copied.
 *  - DIV_K (dim 2 only): coef is a device array of (n[0]+1)*(n[1]+1) float64
 *    per-cell k, cell (cj, ci) at coef[cj*(n[0]+1) + ci] between node columns
 *    ci, ci+1 and node rows cj, cj+1 (boundary nodes numbered 0 and n+1).  A
 *    grid edge takes the mean of the two cells sharing it; centre
 *    sum_e k_e/h^2 + sigma, neighbour -k_e/h^2 plus centred convection.  Copied.
 * tgdk_op_create fails with TGDK_E_INVALID for n[a] < 1, dim not 2 or 3, or a
 * NULL coef where one is needed. */
typedef struct {
    int dim;
    int n[3];
    int kind;
    double beta[3];
    double sigma;
    const double* coef;
} tgdk_op_desc;

int tgdk_op_create(tgdk_ctx ctx, const tgdk_op_desc* desc, tgdk_op* out);
/* The same PDE on the coarse grid h_c = 2 h_f (n_c = (n_f - 1)/2 per axis;
 * every n_f must be odd and >= 3).  CONST_CD keeps beta and sigma; DIV_K takes
 * the geometric mean of the 2x2 (2x2x2) fine cells; VAR_STENCIL cannot be
 * coarsened (TGDK_E_INVALID). */
int tgdk_op_coarsen(tgdk_op fine, tgdk_op* coarse);
/* y = A x (transpose = 0) or y = A^T x (transpose = 1) for nrhs column
 * vectors; x and y device arrays of nrhs*n elements of type dtype
 * (TGDK_F64/TGDK_F32); x and y must not overlap.  Enqueue only. */
int tgdk_op_apply(tgdk_op op, int transpose, int dtype, const void* x, void* y, int nrhs);
/* Number of unknowns n and dimensions of an operator. */
int tgdk_op_info(tgdk_op op, int* dim, int* n_per_axis /* [3] */, long long* n);
int tgdk_op_destroy(tgdk_op op);

/* ----------------------------------------------------------- grid transfer
 * Coarse-to-fine transfer of Sec. 3 ("spline interpolation or
 * prolongation"), read as the linear spline: vf = P vc with bilinear
 * (trilinear) weights 1, 1/2, 1/4 (, 1/8) on nested grids n_f = 2 n_c + 1.
 * Restriction is full weighting vc = P^T vf / 2^dim.  Both apply the 1-D
 * operator along x, then y, then z, adding contributors in increasing index
 * order, so results are reproducible to the bit.  ncols column vectors of
 * float64 (dtype must be TGDK_F64).  Enqueue only. */
int tgdk_prolongate(tgdk_op coarse, tgdk_op fine, int dtype, const void* vc, void* vf, int ncols);
int tgdk_restrict(tgdk_op fine, tgdk_op coarse, int dtype, const void* vf, void* vc, int ncols);

/* ------------------------------------------------------ coarse GMRES-DR(m,k)
 * Phase 1 of the Sec. 3 algorithm: GMRES-DR(m,k) (Sec. 2.1) on the coarse
 * grid solves A_c x_c = b_c (or A_c^T x_c = b_c if transpose) and computes the
 * k harmonic Ritz vectors with smallest |theta|.  It stops when
 * ||b_c - A_c x_c|| <= rtol ||b_c|| and the nev smallest pairs have relative
 * eigen-residual ||A y - rho y|| / ||A||_1 <= rtolev (checked at cycle ends),
 * or after maxcyc cycles (returns TGDK_NOT_CONVERGED, outputs valid).
 * b_c, x_c: device float64, n_c elements; x_c is overwritten (start 0).
 * *coarse_space receives an orthonormal basis of the final harmonic Ritz
 * vectors (k, or k+1 when a complex pair straddles position k).
 * Requirements: 1 <= k < m <= TGDK_MAX_DEFL, nev <= k. */
typedef struct {
    int m, k, nev, maxcyc, transpose;
    double rtolev, rtol;
    /* optional right preconditioner (Sec. 5, Example 5): GMRES-DR runs on
     * A M^{-1}, x = M^{-1} u at the end, and the kept vectors are harmonic
     * Ritz vectors of A M^{-1}; NULL for none */
    tgdk_precond_fn precond;
    void* precond_user;
} tgdk_gmresdr_params;

typedef struct {
    int cycles, nconv, k_out;
    long long mvps;
    double relres;                       /* true ||b - A x|| / ||b|| at exit */
    double theta_re[TGDK_MAX_DEFL + 1];  /* kept harmonic Ritz values */
    double theta_im[TGDK_MAX_DEFL + 1];
    double eigres[TGDK_MAX_DEFL + 1];    /* relative eigen-residuals */
    double seconds;
} tgdk_gmresdr_report;

int tgdk_coarse_setup(tgdk_op coarse, const double* b_c, double* x_c,
                      const tgdk_gmresdr_params* params, tgdk_defl* coarse_space,
                      tgdk_gmresdr_report* report);

/* ------------------------------------------------------- deflation spaces
 * A deflation space holds an orthonormal V (n x k, device, stored float64 or
 * float32) and H = V^T A V with its LU factors (Sec. 2.2 projection box,
 * steps 1-2).  It belongs to one operator (and to A^T when transpose = 1).
 *
 * tgdk_defl_prolongate: V = Q of the thin QR (positive diagonal) of P W_c,
 * where W_c is the basis of a coarse space; then H.  Errors with
 * TGDK_E_SINGULAR if P W_c is rank deficient.
 * tgdk_defl_from_basis: the same from a caller basis W (device float64, n x k
 * column-major, not modified) on the operator's own grid.
 * store_dtype: TGDK_F64 or TGDK_F32 (float32 storage: V is rounded once and
 * H formed from the rounded V, so the projection stays exact for that basis).
 */
int tgdk_defl_prolongate(tgdk_defl coarse_space, tgdk_op fine, int store_dtype, tgdk_defl* fine_space);
int tgdk_defl_from_basis(tgdk_op op, const double* W, int k, int transpose, int store_dtype,
                         tgdk_defl* out);
/* MinRes projection (the variant the paper notes after the Sec. 2.2 box):
 * the same V, with H = (AV)^T (AV) and c = (AV)^T r in place of V^T A V and
 * V^T r; the update is unchanged (x += V d, r -= A V d), so the new residual
 * is the least-squares residual of r over span(AV) and never grows.
 * Builds a new space on the same operator and orientation that also stores
 * W = A V (or A^T V) in the store type of V (H is formed from the stored W).
 * Every solver accepts either kind of space.  TGDK_E_SINGULAR if AV is rank
 * deficient. */
#define TGDK_PROJ_GALERKIN 0
#define TGDK_PROJ_MINRES   1
int tgdk_defl_minres(tgdk_defl galerkin_space, tgdk_defl* minres_space);
/* Deflation with a right preconditioner M (Sec. 5, Example 5): the Galerkin
 * projection of A M^{-1} over V, i.e. c = V^T r, H = V^T A Z with
 * Z = M^{-1} V, and the update x += Z d, r -= A Z d.  Builds a new space from
 * a float64 Galerkin space (V kept, Z stored; precond called once with
 * nrhs = k).  Only the preconditioned GMRES-Proj and IDR-Proj solves accept
 * it; tgdk_defl_copy returns V. */
int tgdk_defl_precond(tgdk_defl galerkin_space, tgdk_precond_fn precond, void* precond_user,
                      tgdk_defl* precond_space);
/* Arnoldi-E(m,k) improvement of a space's vectors on its own grid (step 2
 * of the Two-grid Deflated GMRES and BiCGStab boxes, Sec. 3 and 4.1; the
 * Two-grid Arnoldi method of Sec. 2.3).  Starting from the k approximate
 * eigenvectors spanning the space, each cycle runs m - k Arnoldi steps from
 * the leading approximate eigenvector whose residual norm exceeds tol, adds
 * the k kept vectors (orthonormalised against the Krylov basis; a vector
 * that loses all but 1e-8 of its norm is dropped), and takes Rayleigh-Ritz
 * on that subspace (dimension <= m + 1), keeping the k pairs of smallest
 * |theta| (a conjugate pair whole).  Residual norms are
 * ||A y - theta y|| / ||A||_1 for unit y, formed explicitly.  Stops when the
 * nev leading pairs are below tol or after maxcyc cycles, and builds a new
 * Galerkin space (store_dtype) over an orthonormal basis of the kept span.
 * Each basis vector of a cycle is multiplied by A once. */
typedef struct {
    int m;          /* subspace dimension per cycle, k < m <= TGDK_MAX_DEFL */
    int nev;        /* leading pairs that must converge, 0 <= nev <= k */
    int maxcyc;     /* >= 0 */
    double tol;     /* > 0 */
} tgdk_arnoldie_params;

typedef struct {
    int cycles, nconv, k_out;
    long long mvps;
    double theta_re[TGDK_MAX_DEFL + 1];  /* kept Ritz values, in keeping order */
    double theta_im[TGDK_MAX_DEFL + 1];
    double eigres[TGDK_MAX_DEFL + 1];    /* their residual norms at the end */
    double eigres_start[TGDK_MAX_DEFL + 1];  /* ... before the first cycle */
    double seconds;
} tgdk_arnoldie_report;

int tgdk_defl_improve(tgdk_defl space, const tgdk_arnoldie_params* params, int store_dtype,
                      tgdk_defl* improved, tgdk_arnoldie_report* report);
/* k and the store type of a space. */
int tgdk_defl_info(tgdk_defl defl, int* k, int* store_dtype, long long* n);
/* TGDK_PROJ_GALERKIN or TGDK_PROJ_MINRES. */
int tgdk_defl_projection(tgdk_defl defl);
/* Copy V out as float64 (device, n x k) and H (host, k x k row-major; the
 * space's own H, (AV)^T AV for a MinRes space); either pointer may be NULL. */
int tgdk_defl_copy(tgdk_defl defl, double* V_out, double* H_out);
int tgdk_defl_destroy(tgdk_defl defl);

/* ------------------------------------------------------------ multigrid
 * Geometric multigrid for a constant-coefficient operator (e.g. the
 * positively shifted Laplacian -Lap(u) + kappa^2 u, which preconditions the
 * Helmholtz operator in Sec. 5, Example 5).  Levels: the operator's grid and
 * its rediscretised nested coarse grids (n -> (n-1)/2) while every side is
 * odd and >= 3.  V-cycle: damped Jacobi with the constant diagonal
 * (omega = 4/5 in 2-D, 6/7 in 3-D), nu sweeps before and after; full
 * weighting and linear interpolation; 20 sweeps on the coarsest grid.
 * tgdk_mg_apply is a tgdk_precond_fn (user = the tgdk_mg): `cycles` V-cycles
 * from zero, z_1 = V(b), z_(c+1) = z_c + V(b - A z_c) (a fixed linear
 * operator).  By default the kernel sequence is captured into a HIP graph
 * at the first apply and replayed; in and out are copied around it.  The
 * object keeps per-level work vectors: one apply at a time per object.
 * tgdk_mg_create returns TGDK_E_INVALID for an operator that is not
 * constant-coefficient, a non-positive diagonal or cycles, nu < 1, and
 * TGDK_E_NOMEM when the level vectors cannot be allocated; tgdk_mg_apply
 * returns TGDK_E_INVALID for NULL or aliasing in/out or nrhs < 1 and
 * TGDK_E_HIP if the graph capture fails. */
typedef struct tgdk_mg_s* tgdk_mg;
#define TGDK_MG_EAGER 1   /* flags: launch the kernels on every apply instead of replaying a HIP graph */
int tgdk_mg_create(tgdk_op op, int cycles, int nu, int flags, tgdk_mg* mg);
int tgdk_mg_apply(void* mg, const double* in, double* out, int nrhs);
int tgdk_mg_levels(tgdk_mg mg);
int tgdk_mg_destroy(tgdk_mg mg);

/* ------------------------------------------------------------ fine solve
 * BiCGStab(ncyc)-Proj(k) (Sec. 4.1 algorithm box, step 3 a-d) or
 * GMRES(m3)-Proj(k) (Sec. 2.2 box) on A x = b (A^T x = b if transpose).
 *  - defl may be NULL (k = 0: plain restarted BiCGStab / GMRES(m3)).
 *  - b, x: device float64, nrhs columns of n; x is the initial guess when
 *    x0_given = 1, otherwise it is zeroed first.  The nrhs systems share A,
 *    V and H and run in the same launches, each with its own state machine:
 *    its own scalars, cycle boundaries and stopping.
 *  - The overall tolerance is tau = rtol * min(||b||, ||b - A x0||) on the
 *    true residual, recomputed in float64 after every cycle.
 *  - Cycle tolerance (BiCGStab): the smaller of
 *    (tau/||r||)^(1/(ncyc-icyc+1)) and (||r0||/||r||)(tau/||r0||)^(icyc/ncyc),
 *    relative to the residual after the projection; after ncyc cycles
 *    tau/||r|| for up to max_extra_cycles more cycles, then
 *    TGDK_NOT_CONVERGED.
 *  - precision TGDK_FP32_IR: the inner BiCGStab runs in float32 on the
 *    correction system, its relative tolerance floored at fp32_floor; the
 *    projection, x and the true residual stay float64.  (BiCGStab only.)
 *  - maxit_cycle bounds the iterations of one inner cycle.
 * reports: host array of nrhs reports.  Returns the worst status over the
 * right-hand sides. */
typedef struct {
    int method;            /* TGDK_BICGSTAB_PROJ, TGDK_GMRES_PROJ or TGDK_IDRS_PROJ */
    int ncyc;              /* BiCGStab, IDR: requested cycles (>= 1) */
    int m3;                /* GMRES: cycle length m (1..TGDK_MAX_DEFL) */
    int precision;         /* TGDK_FP64 or TGDK_FP32_IR */
    int x0_given;
    int transpose;
    int maxit_cycle;
    int max_extra_cycles;  /* BiCGStab, IDR: cycles allowed past ncyc; GMRES: max cycles */
    double rtol;
    double fp32_floor;
    /* GMRES: variable restarting (Sec. 4.3, Table 4.3): cycle j (0-based)
     * has cycle_lengths[j] steps for j < n_cycle_lengths, then m3 steps;
     * every length in 1..m3.  NULL / 0: every cycle has m3 steps. */
    const int* cycle_lengths;  /* host array */
    int n_cycle_lengths;
    /* optional right preconditioner for GMRES-Proj and IDR-Proj (FP64 only;
     * BiCGStab: TGDK_E_INVALID): the inner solver works on A M^{-1} and
     * x += M^{-1} (correction); a deflation space must then come from
     * tgdk_defl_precond with the same preconditioner */
    tgdk_precond_fn precond;
    void* precond_user;
    /* Resuming a solve at a cycle boundary (Sec. 4.1 box, step 3: the
     * schedule of cycle tolerances depends on the cycle number icyc and on
     * ||r0||).  icyc0 >= 0: cycles already completed by earlier calls on
     * this system; this call's first cycle is cycle icyc0 + 1 of the
     * schedule and the cycle limit ncyc + max_extra_cycles counts them.
     * nu0 > 0: ||r0|| of the solve's original initial guess (the report's
     * nu0 of the first call); tau = rtol min(||b||, nu0).  0 takes this
     * call's starting residual.  Pass the interrupted iterate as x with
     * x0_given = 1: the resumed solve then repeats, bit for bit, what the
     * uninterrupted one computes from that cycle boundary on.
     * max_cycles_call > 0: stop after that many cycles of this call with
     * TGDK_NOT_CONVERGED (outputs valid, x is the iterate at that cycle
     * boundary); 0 for no limit. */
    int icyc0;
    int max_cycles_call;
    double nu0;
} tgdk_solve_params;

typedef struct {
    int status, cycles;
    long long iters_inner, mvp_inner, mvp_boundary;
    double relres_true;    /* ||b - A x|| / ||b|| at exit (float64) */
    double seconds;        /* host wall time of the call */
    int branch[4];         /* cycles whose tolerance came from criterion 1, 2, past-ncyc */
    int n_first;           /* recorded (rho, alpha, omega) of the first inner iterations */
    double first_rho[TGDK_NHIST], first_alpha[TGDK_NHIST], first_omega[TGDK_NHIST];
    int n_cycle_mvps;      /* min(cycles, TGDK_NCYC_REPORT) */
    int cycle_mvps[TGDK_NCYC_REPORT];  /* inner operator applications of each of the first cycles */
    int cycle_branch[TGDK_NCYC_REPORT];  /* criterion (1, 2, 3 = past ncyc) that set each cycle's
                                            tolerance; 0 for a cycle that did not start */
    double nu0;            /* ||r0|| of the schedule (pass it back as params.nu0 to resume) */
    /* Cost in the paper's terms (Sec. 3, Example 1: cost = nnz * mvps + vops).
     * mvp_setup: fine-grid operator applications spent building the
     * deflation space used (A V for H = V^T A V; paid once per space, not by
     * this call).  vops: length-n vector operations of this call (a dot
     * product, a norm or an update y += a x counts one; formed from the
     * iteration counts: BiCGStab 12 a full iteration and 7 a half step,
     * GMRES 2j^2 + 5j + 1 a cycle of j steps, IDR(s) the vector updates of
     * its rounds, 3 a true residual, 2k + 3 a projection). */
    long long mvp_setup, vops;
} tgdk_solve_report;

int tgdk_solve(tgdk_op fine, tgdk_defl defl, const double* b, double* x, int nrhs,
               const tgdk_solve_params* params, tgdk_solve_report* reports);

/* IDR(s)(ncyc)-Proj(k) on one right-hand side: the same cycles, projection
 * and cycle tolerance as BiCGStab(ncyc)-Proj(k) (Sec. 4.1 box, step 3 a-d),
 * with IDR(s) as the inner solver of step c (the paper runs s = 4 by
 * default, Sec. 4.1; s = 5 and 20 in the Helmholtz examples of Sec. 5).
 * The inner solver is the biorthogonal IDR(s) of van Gijzen and Sonneveld
 * (ACM TOMS 38(1), 2011): each cycle starts afresh (G = U = 0, M = I,
 * omega = 1) from the residual after the projection; rounds of s steps and
 * one dimension reduction, with omega the minimal-residual value enlarged
 * when the angle between r and A r is small (cos < kappa; kappa = 0.7 in
 * that paper, 0 gives the plain minimal-residual omega).
 *  - shadow: device float64, n x s column-major (s columns of n): the raw
 *    columns of the shadow space.  The library orthonormalises a copy
 *    (CholQR2); shadow is not modified.  TGDK_E_SINGULAR if rank deficient.
 *  - 1 <= s <= TGDK_IDR_SMAX, s <= n; 0 <= kappa < 1.
 *  - params.method must be TGDK_IDRS_PROJ; ncyc, max_extra_cycles,
 *    precision (TGDK_FP32_IR: G, U, P, r and e in float32), rtol,
 *    fp32_floor, x0_given, transpose as for BiCGStab; maxit_cycle bounds
 *    the operator applications of one inner cycle.
 *  - TGDK_FP32_IR is for moderately conditioned grids: on the 1023^2
 *    convection-diffusion grid the float32 IDR cycles stop reducing the
 *    true residual near 1e-6 relative and then diverge (the same happens
 *    in a plain float32 reference implementation); use TGDK_FP64 there.
 *  - report: iters_inner = mvp_inner = inner operator applications;
 *    first_rho[i] = ||r|| after the i-th update of the inner residual in the
 *    first cycle, first_alpha[i] = that update's coefficient (beta, or omega
 *    at a dimension reduction), first_omega[i] = 1 at a dimension reduction,
 *    else 0.
 * Blocking; returns the report's status. */
int tgdk_solve_idr(tgdk_op fine, tgdk_defl defl, const double* b, double* x, int s, const double* shadow,
                   double kappa, const tgdk_solve_params* params, tgdk_solve_report* report);

/* For callers that cannot allocate device memory during a solve (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * tgdk_solve for params.method = TGDK_BICGSTAB_PROJ, with the same kernels,
 * launches and results, that allocates nothing.  Its workspace (descriptors,
 * solver states, the float64 residual and inner vectors of every system,
 * partial sums) lives in one fixed device array of TGDK_NOALLOC_SCRATCH_MB
 * MiB per GPU, held by the library until the process ends; the status
 * mirror and events come from tgdk_ctx_create.  The caller passes inputs and
 * outputs as for tgdk_solve.
 *  - Capacity: about 80 n bytes per right-hand side with TGDK_FP64 inner
 *    cycles, 48 n with TGDK_FP32_IR (8 n more on 3-D grids with a deflation
 *    space), plus partial sums; at most 64 right-hand sides.  A call that
 *    needs more returns TGDK_E_INVALID (the message gives the bytes needed)
 *    without touching x.  Step-kernel timing (tgdk_ctx_time_kernel) must be
 *    off.
 *  - Every call on a GPU uses that GPU's one array, and the array keeps the
 *    last call's contents (the solve clears what must start at zero): calls
 *    that overlap on one GPU, from any context or thread, race. */
#define TGDK_NOALLOC_SCRATCH_MB 64
int tgdk_solve_noalloc(tgdk_op fine, tgdk_defl defl, const double* b, double* x, int nrhs,
                       const tgdk_solve_params* params, tgdk_solve_report* reports);

/* Several independent instances (each its own operator, deflation space or
 * NULL, right-hand side and solution, all on the context ctx -- every
 * operator must belong to it -- and of one dimension) solved together:
 * every kernel launch covers the tiles of all instances, so small and uneven
 * grids fill the device in one launch per step.  BiCGStab(ncyc)-Proj(k)
 * only.  Same parameters and reports (one per instance) as tgdk_solve;
 * TGDK_E_INVALID for an operator of another context or dimension. */
int tgdk_solve_instances(tgdk_ctx ctx, int ninst, const tgdk_op* ops, const tgdk_defl* defls,
                         const double* const* b, double* const* x,
                         const tgdk_solve_params* params, tgdk_solve_report* reports);

/* --------------------------------------------------------------- adjoint
 * Gradient of L(u) = 1/2 ||u - u*||^2 with u = A(k)^{-1} b for a DIV_K
 * operator, given u and lambda = A^{-T}(u - u*):
 *   dL/dk_c = -sum over the four sides e = (p, q) of cell c of
 *             (1/2) h^-2 (lambda_p - lambda_q)(u_p - u_q),
 * with u = lambda = 0 on boundary nodes (dL/db = lambda needs no call).
 * lambda, u: device float64 (n); grad_k: device float64 ((n_x+1)(n_y+1)).
 * TGDK_E_INVALID unless the operator is 2-D DIV_K.  Enqueue only. */
int tgdk_adjoint_grad_k(tgdk_op fine, const double* lambda, const double* u, double* grad_k);

/* ------------------------------------------------------------- autotune
 * Times the candidate tile heights of the stencil-shaped kernels for this
 * operator and element type and keeps the fastest for later launches on
 * operators of the same shape.  Results are cached in the file named by the
 * environment variable TGDK_TUNE_CACHE (if set).  Returns the chosen tile
 * height in *tile_y (may be NULL).  ctx must be the operator's context
 * (NULL: the operator's own); kernels are timed on its stream. */
int tgdk_tune(tgdk_ctx ctx, tgdk_op op, int dtype, int nrhs, int* tile_y);

#ifdef __cplusplus
}
#endif
#endif /* TGDK_H */
