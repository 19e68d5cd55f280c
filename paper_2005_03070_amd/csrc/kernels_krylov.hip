// Tile kernels of the cycle boundary of the host-driven solvers (GMRES-Proj,
// IDR(s)-Proj) and of the final true-residual check: r = b - A x, the
// Galerkin projection c = V^T r, H d = c, and x += V d, r -= A V d (Sec. 2.2
// box).  One launch covers every tile of every problem of a group; per-tile
// partial sums are reduced in tile order by a one-workgroup-per-problem
// epilogue launch.  The BiCGStab cycles run in the step kernel
// (step_kernel.h).
#include "device_common.h"
#include "launch.h"

namespace tgdk {

__device__ __forceinline__ void mirror_out(const DevProb& P, const SolveState* st) {
    if (P.mirror) {
        P.mirror->solve_state = st->solve_state;
        P.mirror->inner_state = st->inner_state;
        P.mirror->icyc = st->icyc;
        P.mirror->iter = st->iter;
        P.mirror->target2 = st->target2;
        __threadfence_system();
    }
}

// Start of an inner cycle from a residual of norm nu: its tolerance
// (Sec. 4.1 step 3 b, cycle_tolerance) and fresh scalars.
__device__ void start_cycle(SolveState* st, double nu, double rho0) {
    double rt;
    const int branch = cycle_tolerance(nu, st->nu0, st->tau, st->icyc, st->ncyc, st->precision, st->fp32_floor, rt);
    st->rt = rt;
    st->target2 = (rt * nu) * (rt * nu);
    st->branch[branch] += 1;
    if (st->icyc >= 1 && st->icyc <= NCYCLOG) st->cyc_branch[st->icyc - 1] = branch;
    st->rho = rho0;
    st->rho_old = 1.0;
    st->alpha = 1.0;
    st->omega = 1.0;
    st->iter = 0;
    st->inner_state = IN_RUNNING;
    st->rr_last = nu * nu;
}

// ---------------------------------------------------------- true residual
// r = b - A x (float64).  first != 0 on the first call of a solve (also sums
// ||b||^2).  Without deflation vectors (k = 0) a BiCGStab cycle starts here:
// the inner residual (and BiCGStab's shadow vector) are written in the inner
// type.
template <class Cfg, int DIM, class TI>
__global__ __launch_bounds__(NT) void k_residual(const DevProb* __restrict__ probs, int nprob, int first) {
    __shared__ double L[Cfg::BOX];
    __shared__ double sh[NWAVE * 3];
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const DevProb& P = probs[find_prob(probs, nprob, t)];
    SolveState* st = P.st;
    if (first != 2 && st->solve_state != SV_RUNNING) return;
    const TilePos tp = tile_pos<Cfg>(t - P.tile_begin, P.tx, P.ty);
    const DevOp& op = P.op;
    const double* __restrict__ x = P.x;
    const double* __restrict__ b = P.b;
    long long gq[Cfg::PPT];
    int cq[Cfg::PPT];
    bool okq[Cfg::PPT];
    double bq[Cfg::PPT];
#pragma unroll
    for (int q = 0; q < Cfg::PPT; ++q) {
        int gx, gy, gz;
        point_coords<Cfg>(q, tp, gx, gy, gz, cq[q]);
        okq[q] = inside(op, gx, gy, gz);
        gq[q] = okq[q] ? gidx(op, gx, gy, gz) : 0;
        L[cq[q]] = okq[q] ? x[gq[q]] : 0.0;
        bq[q] = okq[q] ? b[gq[q]] : 0.0;
    }
    fill_halo<Cfg, DIM, double>(L, tp, op, [&](long long g) { return x[g]; });
    __syncthreads();
    const bool start = (P.k == 0) && (st->method != METHOD_GMRES) && first != 2;
    const bool shadow = st->method == METHOD_BICGSTAB;
    TI* rin = vp<TI>(P.rin);
    TI* rhat = vp<TI>(P.rhat);
    const bool sep = (void*)rin != (void*)P.r;
    double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < Cfg::PPT; ++q) {
        if (!okq[q]) continue;
        const long long g = gq[q];
        const double bv = bq[q];
        const double rv = bv - stencil_row<Cfg, DIM, double>(op, L, cq[q], g);
        P.r[g] = rv;
        acc[0] += rv * rv;
        acc[1] += bv * bv;
        if (start) {
            const TI ri = (TI)rv;
            if (sep) rin[g] = ri;
            if (shadow) rhat[g] = ri;
            acc[2] += (double)ri * (double)ri;
        }
    }
    double tot;
    block_sum<3>(acc, sh, tot);
    const int lt = t - P.tile_begin;
    if (threadIdx.x < 3) P.partial[(long long)lt * P.pstride + threadIdx.x] = tot;
}

// Epilogue of the true residual (one workgroup per problem).
__global__ __launch_bounds__(NT) void k_epi_residual(const DevProb* __restrict__ probs, int first) {
    __shared__ double sh[NWAVE * 3];
    const DevProb& P = probs[blockIdx.x];
    SolveState* st = P.st;
    if (first != 2 && st->solve_state != SV_RUNNING) return;
    const bool start = (P.k == 0) && (st->method != METHOD_GMRES) && first != 2;
    double sums[3];
    sum_partials_multi<3>(P.partial, P.ntiles, P.pstride, sums, sh);
    const double rr = sums[0], bb = sums[1], ri = sums[2];
    if (threadIdx.x != 0) return;
    if (first == 2) {
        st->nu_final = sqrt(rr);
        return;
    }
    st->mvp_boundary += 1;
    const double nu = sqrt(rr);
    st->nu = nu;
    if (first) {
        // a resumed solve keeps its first call's nu0 and tau (st->icyc
        // starts at icyc0)
        st->bnorm = sqrt(bb);
        st->nu0 = st->nu0_in > 0.0 ? st->nu0_in : nu;
        st->tau = st->rtol * fmin(st->bnorm, st->nu0);
        if (!isfinite(nu))
            st->solve_state = SV_NONFINITE;
        else if (nu <= st->tau || nu == 0.0)
            st->solve_state = SV_CONVERGED;
        else if (st->icyc > 0 && st->icyc >= st->ncyc + st->max_extra)
            st->solve_state = SV_NOT_CONVERGED;
    } else {
        if (st->icyc >= 1 && st->icyc <= NCYCLOG) {
            st->cyc_iters[st->icyc - 1] = st->iter;
            st->cyc_end[st->icyc - 1] = st->inner_state;
        }
        const bool broke = (st->inner_state == IN_BREAK_NOUPD || st->inner_state == IN_BREAK_FULL);
        if (!isfinite(nu))
            st->solve_state = SV_NONFINITE;
        else if (nu <= st->tau)
            st->solve_state = SV_CONVERGED;
        else if (broke && ((st->method == METHOD_BICGSTAB && st->iter == 0) ||
                           (st->method == METHOD_IDR && st->iter <= 1)))
            st->solve_state = SV_BREAKDOWN;
        else if (st->icyc >= st->ncyc + st->max_extra)
            st->solve_state = SV_NOT_CONVERGED;
        else if (st->maxcyc_call > 0 && st->icyc - st->icyc0 >= st->maxcyc_call)
            st->solve_state = SV_NOT_CONVERGED;
    }
    if (st->solve_state == SV_RUNNING) {
        st->icyc += 1;
        if (start) {
            start_cycle(st, nu, ri);
            if (P.mirror) {
                P.mirror->rr0 = nu * nu;
                P.mirror->rr = nu * nu;
            }
        }
    }
    mirror_out(P, st);
}

// ------------------------------------------------- projection: c = V^T r
// Partials of c over the tile, then (last workgroup) c summed in tile order
// and H d = c solved with the LU factors of H (Sec. 2.2 box, steps 2-3).
template <class Cfg, class TV>
__global__ __launch_bounds__(NT) void k_proj_dot(const DevProb* __restrict__ probs, int nprob) {
    __shared__ double sh[NWAVE * 16];
    __shared__ double y[MAXK + 1];
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const DevProb& P = probs[find_prob(probs, nprob, t)];
    SolveState* st = P.st;
    if (st->solve_state != SV_RUNNING || P.k == 0) return;
    const int lt = t - P.tile_begin;
    const TilePos tp = tile_pos<Cfg>(lt, P.tx, P.ty);
    const DevOp& op = P.op;
    const TV* V = reinterpret_cast<const TV*>(P.Vl);  // left basis of c
    const int k = P.k;
    double rv[Cfg::PPT];
    long long gq[Cfg::PPT];
#pragma unroll
    for (int q = 0; q < Cfg::PPT; ++q) {
        int gx, gy, gz, c;
        point_coords<Cfg>(q, tp, gx, gy, gz, c);
        const bool ok = inside(op, gx, gy, gz);
        gq[q] = ok ? gidx(op, gx, gy, gz) : -1;
        rv[q] = ok ? P.r[gq[q]] : 0.0;
    }
    for (int c0 = 0; c0 < k; c0 += 16) {
        double acc[16];
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) acc[jj] = 0.0;
#pragma unroll
        for (int q = 0; q < Cfg::PPT; ++q) {
            if (gq[q] < 0) continue;
#pragma unroll
            for (int jj = 0; jj < 16; ++jj)
                if (c0 + jj < k) acc[jj] += (double)V[(long long)(c0 + jj) * P.ldv + gq[q]] * rv[q];
        }
        double tot;
        block_sum<16>(acc, sh, tot);
        if (threadIdx.x < 16 && c0 + threadIdx.x < k)
            P.partial[(long long)lt * P.pstride + c0 + threadIdx.x] = tot;
    }
}

// c summed in tile order, then H d = c by the LU factors of H.
__global__ __launch_bounds__(NT) void k_epi_proj_dot(const DevProb* __restrict__ probs) {
    __shared__ double scratch[NT];
    __shared__ double y[MAXK + 1];
    const DevProb& P = probs[blockIdx.x];
    SolveState* st = P.st;
    if (st->solve_state != SV_RUNNING || P.k == 0) return;
    const int k = P.k;
    sum_partial_columns(P.partial, P.ntiles, P.pstride, k, y, scratch);
    // LU solve: row interchanges, then L (unit lower) and U (upper), row-major.
    if (threadIdx.x == 0) {
        for (int i = 0; i < k; ++i) st->cvec[i] = y[i];
        for (int i = 0; i < k; ++i) {
            const int pi = P.piv[i];
            if (pi != i) {
                const double tmp = y[i];
                y[i] = y[pi];
                y[pi] = tmp;
            }
        }
    }
    __syncthreads();
    const double* LU = P.lu;
    for (int j = 0; j < k; ++j) {
        const double yj = y[j];
        __syncthreads();
        for (int i = j + 1 + threadIdx.x; i < k; i += NT) y[i] -= LU[i * k + j] * yj;
        __syncthreads();
    }
    for (int j = k - 1; j >= 0; --j) {
        if (threadIdx.x == 0) y[j] = y[j] / LU[j * k + j];
        __syncthreads();
        const double yj = y[j];
        for (int i = threadIdx.x; i < j; i += NT) y[i] -= LU[i * k + j] * yj;
        __syncthreads();
    }
    for (int i = threadIdx.x; i < k; i += NT) st->d[i] = y[i];
}

// ---------------------------------- projection: x += V d, r -= A (V d)
// w = V d is formed on the tile halo in LDS; then x += w and r -= A w on the
// tile.  Starts the next inner cycle (inner residual, BiCGStab's shadow
// vector, the cycle tolerance).
template <class Cfg, int DIM, class TV, class TI>
__global__ __launch_bounds__(NT) void k_proj_apply(const DevProb* __restrict__ probs, int nprob) {
    __shared__ double L[Cfg::BOX];
    __shared__ double dsh[MAXK + 1];
    __shared__ double sh[NWAVE * 2];
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const DevProb& P = probs[find_prob(probs, nprob, t)];
    SolveState* st = P.st;
    if (st->solve_state != SV_RUNNING || P.k == 0) return;
    const int lt = t - P.tile_begin;
    const TilePos tp = tile_pos<Cfg>(lt, P.tx, P.ty);
    const DevOp& op = P.op;
    const TV* __restrict__ V = reinterpret_cast<const TV*>(P.V);
    const long long ldv = P.ldv;
    const int k = P.k;
    for (int i = threadIdx.x; i < k; i += NT) dsh[i] = st->d[i];
    __syncthreads();
    auto wval = [&](long long g) {
        double w = 0.0;
        for (int j = 0; j < k; ++j) w += (double)V[(long long)j * ldv + g] * dsh[j];
        return w;
    };
    long long gq[Cfg::PPT];
    int cq[Cfg::PPT];
    bool okq[Cfg::PPT];
#pragma unroll
    for (int q = 0; q < Cfg::PPT; ++q) {
        int gx, gy, gz;
        point_coords<Cfg>(q, tp, gx, gy, gz, cq[q]);
        okq[q] = inside(op, gx, gy, gz);
        gq[q] = okq[q] ? gidx(op, gx, gy, gz) : 0;
        L[cq[q]] = okq[q] ? wval(gq[q]) : 0.0;
    }
    fill_halo<Cfg, DIM, double>(L, tp, op, wval);
    __syncthreads();
    const bool start = st->method != METHOD_GMRES;
    const bool shadow = st->method == METHOD_BICGSTAB;
    TI* rin = vp<TI>(P.rin);
    TI* rhat = vp<TI>(P.rhat);
    const bool sep = (void*)rin != (void*)P.r;
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int q = 0; q < Cfg::PPT; ++q) {
        if (!okq[q]) continue;
        const long long g = gq[q];
        const int c = cq[q];
        P.x[g] += L[c];
        const double rv = P.r[g] - stencil_row<Cfg, DIM, double>(op, L, c, g);
        P.r[g] = rv;
        acc[0] += rv * rv;
        if (start) {
            const TI ri = (TI)rv;
            if (sep) rin[g] = ri;
            if (shadow) rhat[g] = ri;
            acc[1] += (double)ri * (double)ri;
        }
    }
    double tot;
    block_sum<2>(acc, sh, tot);
    if (threadIdx.x < 2) P.partial[(long long)lt * P.pstride + threadIdx.x] = tot;
}

__global__ __launch_bounds__(NT) void k_epi_proj_apply(const DevProb* __restrict__ probs) {
    __shared__ double sh[NWAVE * 2];
    const DevProb& P = probs[blockIdx.x];
    SolveState* st = P.st;
    if (st->solve_state != SV_RUNNING || P.k == 0) return;
    const bool start = st->method != METHOD_GMRES;
    double sums[2];
    sum_partials_multi<2>(P.partial, P.ntiles, P.pstride, sums, sh);
    const double rr = sums[0], ri = sums[1];
    if (threadIdx.x != 0) return;
    st->mvp_boundary += 1;
    st->nproj += 1;
    const double nu = sqrt(rr);
    st->nu = nu;
    if (!isfinite(nu))
        st->solve_state = SV_NONFINITE;
    else if (nu <= st->tau)
        st->solve_state = SV_CONVERGED;
    else if (start) {
        start_cycle(st, nu, ri);
        if (P.mirror) {
            P.mirror->rr0 = nu * nu;
            P.mirror->rr = nu * nu;
        }
    }
    mirror_out(P, st);
}

// ------------------------------------------------------------ launchers
template <class Cfg, int DIM, class TI>
static void solve_launch_cfg(int which, const DevProb* probs, int nprob, int total_tiles, int flag, int vtype,
                             hipStream_t s) {
    dim3 grid(total_tiles), block(NT);
    switch (which) {
        case K_RESIDUAL:
            hipLaunchKernelGGL((k_residual<Cfg, DIM, TI>), grid, block, 0, s, probs, nprob, flag);
            hipLaunchKernelGGL(k_epi_residual, dim3(nprob), block, 0, s, probs, flag);
            break;
        case K_PROJ_DOT:
            if (vtype == 0)
                hipLaunchKernelGGL((k_proj_dot<Cfg, double>), grid, block, 0, s, probs, nprob);
            else
                hipLaunchKernelGGL((k_proj_dot<Cfg, float>), grid, block, 0, s, probs, nprob);
            hipLaunchKernelGGL(k_epi_proj_dot, dim3(nprob), block, 0, s, probs);
            break;
        case K_PROJ_APPLY:
            if (vtype == 0)
                hipLaunchKernelGGL((k_proj_apply<Cfg, DIM, double, TI>), grid, block, 0, s, probs, nprob);
            else
                hipLaunchKernelGGL((k_proj_apply<Cfg, DIM, float, TI>), grid, block, 0, s, probs, nprob);
            hipLaunchKernelGGL(k_epi_proj_apply, dim3(nprob), block, 0, s, probs);
            break;
    }
}

template <int DIM, class TI>
static void solve_launch_dim(int which, const DevProb* probs, int nprob, int total_tiles, int flag, int vtype,
                             int tile_id, hipStream_t s) {
    with_tile<DIM>(tile_id, [&](auto cfg) {
        solve_launch_cfg<decltype(cfg), DIM, TI>(which, probs, nprob, total_tiles, flag, vtype, s);
    });
}

void launch_solve_kernel(int which, int dim, int inner_f32, int vtype, int tile_id, const DevProb* probs,
                         int nprob, int total_tiles, int flag, hipStream_t s) {
    if (total_tiles <= 0) return;
    if (dim == 2) {
        if (inner_f32)
            solve_launch_dim<2, float>(which, probs, nprob, total_tiles, flag, vtype, tile_id, s);
        else
            solve_launch_dim<2, double>(which, probs, nprob, total_tiles, flag, vtype, tile_id, s);
    } else {
        if (inner_f32)
            solve_launch_dim<3, float>(which, probs, nprob, total_tiles, flag, vtype, tile_id, s);
        else
            solve_launch_dim<3, double>(which, probs, nprob, total_tiles, flag, vtype, tile_id, s);
    }
}

void tile_shape(int dim, int tile_id, int* ty, int* tz) {
    if (dim == 2)
        with_tile<2>(tile_id, [&](auto cfg) {
            *ty = decltype(cfg)::TY;
            *tz = 1;
        });
    else
        with_tile<3>(tile_id, [&](auto cfg) {
            *ty = decltype(cfg)::TY;
            *tz = decltype(cfg)::TZ;
        });
}

}  // namespace tgdk
