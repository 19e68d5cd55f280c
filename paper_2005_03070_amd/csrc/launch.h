// Host-callable kernel launchers (defined in the .hip files).
#pragma once

#include <hip/hip_runtime.h>

#include "idr_shared.h"
#include "mg_shared.h"
#include "tgdk_shared.h"

namespace tgdk {

enum : int { K_RESIDUAL = 0, K_PROJ_DOT = 1, K_PROJ_APPLY = 2 };

// grid kernels
// gate: null, or a device word; a nonzero word makes the launch a no-op
template <class T>
void launch_apply(const DevOp& op, const T* x, T* y, int nrhs, int tile_id, hipStream_t s,
                  const int* gate = nullptr);
void launch_build_divk(int nx, int ny, const double* kc, double bx, double by, double sigma, double* coef,
                       hipStream_t s);
void launch_transpose_coef(int dim, int nx, int ny, int nz, const double* c, double* ct, hipStream_t s);
void launch_to_f32(const double* a, float* b, long long n, hipStream_t s);
void launch_to_f64(const float* a, double* b, long long n, hipStream_t s);
void launch_coarsen_kcell(int ncx, int ncy, const double* kf, double* kc, hipStream_t s);
void launch_prolong(int dim, int ncx, int ncy, int ncz, const double* vc, double* vf, int ncols, hipStream_t s);
void launch_restrict(int dim, int ncx, int ncy, int ncz, const double* vf, double* vc, int ncols, hipStream_t s);
void launch_grad_k(int nx, int ny, const double* lam, const double* u, double* g, hipStream_t s);
void launch_fill(double* a, double v, long long n, hipStream_t s);
void launch_copy(const double* a, double* b, long long n, hipStream_t s);

// tile kernels over a problem group (GMRES-Proj driver, final residual)
// flag: the residual kernel's mode (1 first call, 0 cycle end, 2 final check)
void launch_solve_kernel(int which, int dim, int inner_f32, int vtype, int tile_id, const DevProb* probs,
                         int nprob, int total_tiles, int flag, hipStream_t s);
void tile_shape(int dim, int tile_id, int* ty, int* tz);

// BiCGStab step kernel: one launch advances every running problem of the
// group by one step of its state machine.  wg_prob maps a workgroup id to its
// problem (null: every workgroup belongs to problem 0); gslot is the launch
// number within the solve; var: the operator has per-row coefficient arrays;
// single: for a group of one problem, a host copy of its descriptor (passed
// in the kernel arguments), else null.
void launch_step(int dim, int inner_f32, int var, int tile_id, const DevProb* probs, const int* wg_prob,
                 int total_wg, int gslot, hipStream_t s, const DevProb* single);
template <int DIM>
void launch_step_dim(int inner_f32, int var, int tile_id, const DevProb* probs, const int* wg_prob, int total_wg,
                     int gslot, hipStream_t s, const DevProb* single);
// Workgroups per compute unit of the 3-D step kernel (occupancy; 0 if unknown).
int step_blocks_per_cu(int inner_f32, int var, int tile_id);

// IDR(s) inner cycles (kernels_idr.hip): what = one of the IDR_* actions,
// k = the step of the round for IDR_DIR, IDR_ALPHA, IDR_ORTH, IDR_UPD.
enum : int {
    IDR_START = 0,  // f = P^T r, ||r||; the cycle's scalars reset
    IDR_DIR = 1,    // u_k from r, G, U and c
    IDR_ALPHA = 2,  // P^T g_k, alpha (k > 0)
    IDR_ORTH = 3,   // g_k, u_k orthogonalised; M_(k:,k), beta
    IDR_UPD = 4,    // r -= beta g_k, e += beta u_k; convergence; next c
    IDR_OMEGA = 5,  // omega from t = A r
    IDR_RED = 6,    // e += omega r, r -= omega t; f = P^T r; convergence; next c
    IDR_FOLD = 7,   // x += e
    IDR_DIRUPD = 8,  // the update of step k-1 fused with the direction of step k (k >= 1)
};
int idr_blocks(long long n);
void launch_idr(int what, int inner_f32, const IdrArgs& a, int k, hipStream_t s);
// 2-D grids with s <= 8: the stencil of a step fused with its products,
// y = A x and the step's partials, then the step's epilogue.  what =
// IDR_ALPHA: x = u_k (or M^-1 u_k), y = g_k, P^T g_k, then alpha (k > 0) or,
// for k = 0, M_(:,0) and beta (the orthogonalisation of step 0 has nothing
// to remove); IDR_OMEGA: x = r (or M^-1 r), y = t, t.t, t.r, r.r (r from
// a.r), then omega.  false if the fused form does not apply (3-D, s > 8).
bool launch_idr_fused(int what, int inner_f32, const IdrArgs& a, const DevOp& op, int tile_id, const void* x,
                      void* y, int k, hipStream_t s);

// tall-skinny products (column-major blocks, leading dimensions in elements)
// G (p x q, row-major, device) = A^T B, A: n x p, B: n x q; partial workspace
// of gram_partial_size(n) doubles * p*q and one counter.
int gram_blocks(long long n);
// partial workspace launch_gram needs for a p x q product (any p, q)
size_t gram_partial_bytes(long long n, int p, int q);
void launch_gram(const void* A, int atype, long long lda, int p, const void* B, int btype, long long ldb, int q,
                 long long n, double* G, double* partial, unsigned* counter, hipStream_t s);
// Out (n x q, col-major, ldo) = V (n x p, ldv) * Y (p x q, col-major, device)
void launch_vmul(const double* V, long long ldv, int p, const double* Y, int q, double* Out, long long ldo,
                 long long n, hipStream_t s);
// x += V y  (V n x p float64, y device p-vector)
void launch_vmul_add(const double* V, long long ldv, int p, const double* y, double* x, long long n,
                     hipStream_t s);

// classical Gram-Schmidt steps of the Arnoldi process (one problem)
int gs_blocks(long long n);
// hout[i] = V_i . w, i < p
void launch_gs_dot(const double* V, long long ldv, int p, const double* w, long long n, double* hout,
                   double* partial, unsigned* counter, hipStream_t s);
// w -= V h; then hout[i] = V_i . w
void launch_gs_update_dot(const double* V, long long ldv, int p, double* w, const double* h, long long n,
                          double* hout, double* partial, unsigned* counter, hipStream_t s);
// w -= V h; *nrm = ||w||; then v = w / ||w|| (zero if ||w|| = 0)
void launch_gs_update_norm(const double* V, long long ldv, int p, double* w, const double* h, long long n,
                           double* nrm, double* partial, unsigned* counter, hipStream_t s);
void launch_scale(const double* w, double* v, const double* nrm, long long n, hipStream_t s);
// a += b (n values)
void launch_add(double* a, const double* b, long long n, hipStream_t st);
// c = a - b (n values)
void launch_sub(const double* a, const double* b, double* c, long long n, hipStream_t s);

// multigrid (kernels_mg.hip): one pass over a level (mode: MG_FIRST ...
// MG_RESID, optionally | MG_ACC; zc the coarser level's z for MG_PSWEEP),
// the restricted residual of a level, and one V-cycle of the coarse tail in
// one workgroup (P: the tail description in device memory)
void launch_mg_pass(int dim, const MgLvl& L, const double* z, const double* v, const double* zc, double* out,
                    int mode, hipStream_t s);
void launch_mg_resid_restrict(int dim, const MgLvl& F, const double* z, const double* v, double* vc,
                              hipStream_t s);
void launch_mg_tail(int dim, const MgTail* P, const double* vin, double* out, int acc, hipStream_t s);
// ||w|| -> *out (deterministic)
void launch_norm2(const double* w, long long n, double* out, double* partial, unsigned* counter, hipStream_t s);

}  // namespace tgdk
