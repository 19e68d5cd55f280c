// Fused kernels of the fine solve: true residual, Galerkin projection,
// restarted BiCGStab and the end-of-cycle update.  All of them take a group
// of problems (one or more right-hand sides or grid instances); one launch
// covers every tile of every problem.  The scalar recurrences run on the
// device in the epilogue of the last workgroup of each problem, so the host
// never waits inside a cycle.
//
// BiCGStab (van der Vorst; Sec. 4.1 of the paper runs it restarted) is
// evaluated in two launches per iteration:
//
//   phase A (iteration i):  r_i = s_{i-1} - w t_{i-1};  e += a p_{i-1} + w s_{i-1};
//                           p_i = r_i + beta (p_{i-1} - w v_{i-1});  v_i = A p_i;
//                           partial r^.v_i
//   epilogue:               alpha = rho_i / (r^.v_i)
//   phase B:                s_i = r_i - alpha v_i;  t_i = A s_i;
//                           partials s.s, t.s, t.t, r^.s, r^.t
//   epilogue:               omega = t.s / t.t;  ||r_{i+1}||^2 = s.s - 2 w t.s + w^2 t.t;
//                           rho_{i+1} = r^.s - w r^.t (no separate pass over r_{i+1})
//
// Each phase recomputes its stencil input (p_i or s_i) on the tile halo from
// the previous vectors, so the update and the stencil share one pass.
#include "device_common.h"
#include "launch.h"

namespace tgdk {

enum : int { SV_NONFINITE = 4 };

template <class T>
__device__ __forceinline__ T* vp(void* p) { return reinterpret_cast<T*>(p); }

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

// Sec. 4.1 step 3 b): tolerance of the cycle that starts with residual nu.
__device__ void start_cycle(SolveState* st, double nu, double rho0) {
    double rt;
    int branch;
    if (st->icyc > st->ncyc) {
        rt = st->tau / nu;
        branch = 3;
    } else {
        const double t1 = pow(st->tau / nu, 1.0 / (double)(st->ncyc - st->icyc + 1));
        const double t2 = (st->nu0 / nu) * pow(st->tau / st->nu0, (double)st->icyc / (double)st->ncyc);
        if (t1 <= t2) {
            rt = t1;
            branch = 1;
        } else {
            rt = t2;
            branch = 2;
        }
    }
    if (st->precision == 1 && rt < st->fp32_floor) rt = st->fp32_floor;
    st->rt = rt;
    st->target2 = (rt * nu) * (rt * nu);
    st->branch[branch] += 1;
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
// the inner residual and shadow vector are written in the inner type.
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
    const bool start = (P.k == 0) && (st->method == METHOD_BICGSTAB) && first != 2;
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
            rhat[g] = ri;
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
    const bool start = (P.k == 0) && (st->method == METHOD_BICGSTAB) && first != 2;
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
        st->bnorm = sqrt(bb);
        st->nu0 = nu;
        st->tau = st->rtol * fmin(st->bnorm, nu);
        if (!isfinite(nu))
            st->solve_state = SV_NONFINITE;
        else if (nu <= st->tau || nu == 0.0)
            st->solve_state = SV_CONVERGED;
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
        else if (st->method == METHOD_BICGSTAB && broke && st->iter == 0)
            st->solve_state = SV_BREAKDOWN;
        else if (st->icyc >= st->ncyc + st->max_extra)
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
    const TV* V = reinterpret_cast<const TV*>(P.V);
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
    if (P.Ccol) {
        for (int i = threadIdx.x; i < k; i += NT) y[i] = P.Ccol[i];
        __syncthreads();
    } else {
        sum_partial_columns(P.partial, P.ntiles, P.pstride, k, y, scratch);
    }
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
    for (int i = threadIdx.x; i < k; i += NT) {
        st->d[i] = y[i];
        if (P.Dcol) P.Dcol[i] = y[i];
    }
}

// ---------------------------------- projection: x += V d, r -= A (V d)
// w = V d is formed on the tile halo in LDS; then x += w and r -= A w on the
// tile.  Starts the BiCGStab cycle (inner residual, shadow vector, rticyc).
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
    const double* __restrict__ Wc = P.Wcol;
    auto wval = [&](long long g) {
        if (Wc) return Wc[g];
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
    const bool start = st->method == METHOD_BICGSTAB;
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
            rhat[g] = ri;
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
    const bool start = st->method == METHOD_BICGSTAB;
    double sums[2];
    sum_partials_multi<2>(P.partial, P.ntiles, P.pstride, sums, sh);
    const double rr = sums[0], ri = sums[1];
    if (threadIdx.x != 0) return;
    st->mvp_boundary += 1;
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

// ----------------------------------------------------- BiCGStab phase A
template <class Cfg, int DIM, class TI>
__global__ __launch_bounds__(NT) void k_bicg_a(const DevProb* __restrict__ probs, int nprob, int iter_host) {
    __shared__ TI L[Cfg::BOX];
    __shared__ double sh[NWAVE * 2];
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const DevProb& P = probs[find_prob(probs, nprob, t)];
    const int lt = t - P.tile_begin;
    const TilePos tp = tile_pos<Cfg>(lt, P.tx, P.ty);
    const DevOp& op = P.op;
    // The host enqueues iteration iter_host of the cycle; while the problem is
    // running the device's own count equals it, so the buffers and the first-
    // iteration branch are known without the solver state, and the loads of
    // this thread's tile points are issued before the state load returns.
    const bool first = iter_host == 0;
    const int cur = iter_host & 1, prv = cur ^ 1;
    TI* __restrict__ pnew = vp<TI>(P.p[cur]);
    const TI* __restrict__ pold = vp<TI>(P.p[prv]);
    TI* __restrict__ vnew = vp<TI>(P.v[cur]);
    const TI* __restrict__ vold = vp<TI>(P.v[prv]);
    TI* rin = vp<TI>(P.rin);
    const TI* __restrict__ rhat = vp<TI>(P.rhat);
    const TI* __restrict__ sv_ = vp<TI>(P.s);
    const TI* __restrict__ tv_ = vp<TI>(P.t);
    TI* __restrict__ e = vp<TI>(P.e);
    long long gq[Cfg::PPT];
    int cq[Cfg::PPT];
    bool okq[Cfg::PPT];
    TI rq[Cfg::PPT], sq[Cfg::PPT], poq[Cfg::PPT], tq[Cfg::PPT], voq[Cfg::PPT];
#pragma unroll
    for (int q = 0; q < Cfg::PPT; ++q) {
        int gx, gy, gz;
        point_coords<Cfg>(q, tp, gx, gy, gz, cq[q]);
        okq[q] = inside(op, gx, gy, gz);
        const long long g = okq[q] ? gidx(op, gx, gy, gz) : 0;
        gq[q] = g;
        rq[q] = sq[q] = poq[q] = tq[q] = voq[q] = TI(0);
        if (okq[q]) {
            if (first) {
                rq[q] = rin[g];
            } else {
                sq[q] = sv_[g];
                tq[q] = tv_[g];
                poq[q] = pold[g];
                voq[q] = vold[g];
            }
        }
    }
    SolveState* st = P.st;
    if (st->solve_state != SV_RUNNING || st->inner_state != IN_RUNNING) return;
    const TI alpha = (TI)st->alpha, omega = (TI)st->omega;
    const TI beta = first ? TI(0) : (TI)((st->rho / st->rho_old) * (st->alpha / st->omega));
    // new p on this thread's points (into LDS); r is kept for the update below
#pragma unroll
    for (int q = 0; q < Cfg::PPT; ++q) {
        TI pv = rq[q];
        if (!first) {
            rq[q] = sq[q] - omega * tq[q];
            pv = rq[q] + beta * (poq[q] - omega * voq[q]);
        }
        L[cq[q]] = okq[q] ? pv : TI(0);
    }
    fill_halo<Cfg, DIM, TI>(L, tp, op, [&](long long g) -> TI {
        if (first) return rin[g];
        const TI rv = sv_[g] - omega * tv_[g];
        return rv + beta * (pold[g] - omega * vold[g]);
    });
    __syncthreads();
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int q = 0; q < Cfg::PPT; ++q) {
        if (!okq[q]) continue;
        const long long g = gq[q];
        const TI vv = stencil_row<Cfg, DIM, TI>(op, L, cq[q], g);
        st_stream<DIM>(&pnew[g], L[cq[q]]);
        st_stream<DIM>(&vnew[g], vv);
        if (first) {
            st_stream<DIM>(&e[g], TI(0));
        } else {
            st_stream<DIM>(&rin[g], rq[q]);
            st_stream<DIM>(&e[g], e[g] + alpha * poq[q] + omega * sq[q]);
        }
        acc[0] += (double)rhat[g] * (double)vv;
        acc[1] += (double)rq[q] * (double)rq[q];
    }
    double tot;
    block_sum<2>(acc, sh, tot);
    if (threadIdx.x < 2) P.partial[(long long)lt * P.pstride + threadIdx.x] = tot;
}

// alpha = rho / (r^.v); breakdown if r^.v vanishes.
__global__ __launch_bounds__(NT) void k_epi_a(const DevProb* __restrict__ probs) {
    __shared__ double sh[NWAVE * 2];
    const DevProb& P = probs[blockIdx.x];
    SolveState* st = P.st;
    if (st->solve_state != SV_RUNNING || st->inner_state != IN_RUNNING) return;
    double sums[2];
    sum_partials_multi<2>(P.partial, P.ntiles, P.pstride, sums, sh);
    const double sig = sums[0], rr = sums[1];
    if (threadIdx.x != 0) return;
    st->mvp_inner += 1;
    st->sigma = sig;
    st->rr_last = rr;
    st->pbuf = st->iter & 1;
    if (sig == 0.0 || !isfinite(sig)) {
        st->inner_state = IN_BREAK_NOUPD;
        mirror_out(P, st);
    } else {
        st->alpha = st->rho / sig;
    }
}

// ----------------------------------------------------- BiCGStab phase B
template <class Cfg, int DIM, class TI>
__global__ __launch_bounds__(NT) void k_bicg_b(const DevProb* __restrict__ probs, int nprob, int iter_host) {
    __shared__ TI L[Cfg::BOX];
    __shared__ double sh[NWAVE * 5];
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const DevProb& P = probs[find_prob(probs, nprob, t)];
    const int lt = t - P.tile_begin;
    const TilePos tp = tile_pos<Cfg>(lt, P.tx, P.ty);
    const DevOp& op = P.op;
    const int cur = iter_host & 1;
    const TI* __restrict__ v = vp<TI>(P.v[cur]);
    const TI* __restrict__ rin = vp<TI>(P.rin);
    const TI* __restrict__ rhat = vp<TI>(P.rhat);
    TI* __restrict__ s = vp<TI>(P.s);
    TI* __restrict__ tt_ = vp<TI>(P.t);
    long long gq[Cfg::PPT];
    int cq[Cfg::PPT];
    bool okq[Cfg::PPT];
    TI rhq[Cfg::PPT], rq[Cfg::PPT], vq[Cfg::PPT];
#pragma unroll
    for (int q = 0; q < Cfg::PPT; ++q) {
        int gx, gy, gz;
        point_coords<Cfg>(q, tp, gx, gy, gz, cq[q]);
        okq[q] = inside(op, gx, gy, gz);
        const long long g = okq[q] ? gidx(op, gx, gy, gz) : 0;
        gq[q] = g;
        rq[q] = okq[q] ? rin[g] : TI(0);
        vq[q] = okq[q] ? v[g] : TI(0);
        rhq[q] = okq[q] ? rhat[g] : TI(0);
    }
    SolveState* st = P.st;
    if (st->solve_state != SV_RUNNING || st->inner_state != IN_RUNNING) return;
    const TI alpha = (TI)st->alpha;
#pragma unroll
    for (int q = 0; q < Cfg::PPT; ++q) L[cq[q]] = okq[q] ? rq[q] - alpha * vq[q] : TI(0);
    fill_halo<Cfg, DIM, TI>(L, tp, op, [&](long long g) -> TI { return rin[g] - alpha * v[g]; });
    __syncthreads();
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < Cfg::PPT; ++q) {
        if (!okq[q]) continue;
        const long long g = gq[q];
        const TI sv = L[cq[q]];
        const TI tv = stencil_row<Cfg, DIM, TI>(op, L, cq[q], g);
        st_stream<DIM>(&s[g], sv);
        st_stream<DIM>(&tt_[g], tv);
        const double rh = (double)rhq[q];
        const double sd = (double)sv, td = (double)tv;
        acc[0] += sd * sd;
        acc[1] += td * sd;
        acc[2] += td * td;
        acc[3] += rh * sd;
        acc[4] += rh * td;
    }
    double tot;
    block_sum<5>(acc, sh, tot);
    if (threadIdx.x < 5) P.partial[(long long)lt * P.pstride + threadIdx.x] = tot;
}

// omega, the next rho and the exit tests of the iteration.
__global__ __launch_bounds__(NT) void k_epi_b(const DevProb* __restrict__ probs) {
    __shared__ double sh[NWAVE * 5];
    const DevProb& P = probs[blockIdx.x];
    SolveState* st = P.st;
    if (st->solve_state != SV_RUNNING || st->inner_state != IN_RUNNING) return;
    double sums[5];
    sum_partials_multi<5>(P.partial, P.ntiles, P.pstride, sums, sh);
    if (threadIdx.x != 0) return;
    const double ss = sums[0], ts = sums[1], tt = sums[2], rs = sums[3], rt = sums[4];
    st->mvp_inner += 1;
    st->iter += 1;
    st->iters_total += 1;
    const int hi = st->nhist;
    if (ss <= st->target2) {
        if (hi < NHIST) {
            st->hist[3 * hi] = st->rho;
            st->hist[3 * hi + 1] = st->alpha;
            st->hist[3 * hi + 2] = __builtin_nan("");
            st->nhist = hi + 1;
        }
        st->inner_state = IN_HALF;
        mirror_out(P, st);
        return;
    }
    const double omega = (tt != 0.0) ? ts / tt : 0.0;
    st->omega = omega;
    if (hi < NHIST) {
        st->hist[3 * hi] = st->rho;
        st->hist[3 * hi + 1] = st->alpha;
        st->hist[3 * hi + 2] = omega;
        st->nhist = hi + 1;
    }
    if (omega == 0.0 || !isfinite(omega)) {
        st->inner_state = IN_BREAK_FULL;
    } else {
        double rr = ss - 2.0 * omega * ts + omega * omega * tt;
        if (rr < 0.0) rr = 0.0;
        const double rho_new = rs - omega * rt;
        if (rr <= st->target2)
            st->inner_state = IN_CONVERGED;
        else if (rho_new == 0.0 || !isfinite(rho_new))
            st->inner_state = IN_BREAK_FULL;
        else if (st->iter >= st->maxit)
            st->inner_state = IN_MAXIT;
        else {
            st->rho_old = st->rho;
            st->rho = rho_new;
        }
        if (P.mirror) P.mirror->rr = rr;
    }
    if (P.mirror) P.mirror->iter = st->iter;
    if (st->inner_state != IN_RUNNING) mirror_out(P, st);
}

// ------------------------------------------------ end of an inner cycle
// x += e + (pending update of the last iteration), in float64.
template <class Cfg, class TI>
__global__ __launch_bounds__(NT) void k_finalize(const DevProb* __restrict__ probs, int nprob) {
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const DevProb& P = probs[find_prob(probs, nprob, t)];
    const SolveState* st = P.st;
    if (st->solve_state != SV_RUNNING) return;
    const int lt = t - P.tile_begin;
    const TilePos tp = tile_pos<Cfg>(lt, P.tx, P.ty);
    const DevOp& op = P.op;
    const int is = st->inner_state;
    const double a = (is == IN_BREAK_NOUPD) ? 0.0 : st->alpha;
    const double w = (is == IN_CONVERGED || is == IN_BREAK_FULL || is == IN_MAXIT) ? st->omega : 0.0;
    const TI* p = vp<TI>(P.p[st->pbuf]);
    const TI* s = vp<TI>(P.s);
    const TI* e = vp<TI>(P.e);
    const bool any_iter = !(is == IN_BREAK_NOUPD && st->iter == 0);
#pragma unroll
    for (int q = 0; q < Cfg::PPT; ++q) {
        int gx, gy, gz, c;
        point_coords<Cfg>(q, tp, gx, gy, gz, c);
        if (!inside(op, gx, gy, gz)) continue;
        const long long g = gidx(op, gx, gy, gz);
        if (!any_iter) continue;
        double upd = (double)e[g];
        if (a != 0.0) upd += a * (double)p[g];
        if (w != 0.0) upd += w * (double)s[g];
        P.x[g] += upd;
    }
}

// ------------------------------------------------------------ launchers
template <class Cfg, int DIM, class TI>
static void solve_launch_cfg(int which, const DevProb* probs, int nprob, int total_tiles, int flag, int vtype,
                             hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    dim3 grid(total_tiles), block(NT);
    if (ev0) (void)hipEventRecord(ev0, s);
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
        case K_BICG_A:
            hipLaunchKernelGGL((k_bicg_a<Cfg, DIM, TI>), grid, block, 0, s, probs, nprob, flag);
            if (ev1) (void)hipEventRecord(ev1, s);
            hipLaunchKernelGGL(k_epi_a, dim3(nprob), block, 0, s, probs);
            break;
        case K_BICG_B:
            hipLaunchKernelGGL((k_bicg_b<Cfg, DIM, TI>), grid, block, 0, s, probs, nprob, flag);
            if (ev1) (void)hipEventRecord(ev1, s);
            hipLaunchKernelGGL(k_epi_b, dim3(nprob), block, 0, s, probs);
            break;
        case K_FINALIZE:
            hipLaunchKernelGGL((k_finalize<Cfg, TI>), grid, block, 0, s, probs, nprob);
            break;
    }
}

template <int DIM, class TI>
static void solve_launch_dim(int which, const DevProb* probs, int nprob, int total_tiles, int flag, int vtype,
                             int tile_id, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (DIM == 2) {
        switch (tile_id) {
            case 1: solve_launch_cfg<Tile<2, 8, 1>, 2, TI>(which, probs, nprob, total_tiles, flag, vtype, s, e0, e1); break;
            case 2: solve_launch_cfg<Tile<2, 4, 1>, 2, TI>(which, probs, nprob, total_tiles, flag, vtype, s, e0, e1); break;
            default: solve_launch_cfg<Tile<2, 16, 1>, 2, TI>(which, probs, nprob, total_tiles, flag, vtype, s, e0, e1); break;
        }
    } else {
        switch (tile_id) {
            case 1: solve_launch_cfg<Tile<3, 8, 4>, 3, TI>(which, probs, nprob, total_tiles, flag, vtype, s, e0, e1); break;
            case 2: solve_launch_cfg<Tile<3, 4, 8>, 3, TI>(which, probs, nprob, total_tiles, flag, vtype, s, e0, e1); break;
            default: solve_launch_cfg<Tile<3, 4, 4>, 3, TI>(which, probs, nprob, total_tiles, flag, vtype, s, e0, e1); break;
        }
    }
}

void launch_solve_kernel(int which, int dim, int inner_f32, int vtype, int tile_id, const DevProb* probs,
                         int nprob, int total_tiles, int flag, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (total_tiles <= 0) return;
    if (dim == 2) {
        if (inner_f32)
            solve_launch_dim<2, float>(which, probs, nprob, total_tiles, flag, vtype, tile_id, s, e0, e1);
        else
            solve_launch_dim<2, double>(which, probs, nprob, total_tiles, flag, vtype, tile_id, s, e0, e1);
    } else {
        if (inner_f32)
            solve_launch_dim<3, float>(which, probs, nprob, total_tiles, flag, vtype, tile_id, s, e0, e1);
        else
            solve_launch_dim<3, double>(which, probs, nprob, total_tiles, flag, vtype, tile_id, s, e0, e1);
    }
}

void launch_proj_shared_epilogue(const DevProb* probs, int nprob, hipStream_t s) {
    hipLaunchKernelGGL(k_epi_proj_dot, dim3(nprob), dim3(NT), 0, s, probs);
}

// The apply half of the projection for systems with Wcol set (no V reads):
// the same kernel, its V d branch never taken.
void launch_proj_apply_shared(int dim, int inner_f32, int tile_id, const DevProb* probs, int nprob,
                              int total_tiles, hipStream_t s) {
    launch_solve_kernel(K_PROJ_APPLY, dim, inner_f32, 0, tile_id, probs, nprob, total_tiles, 0, s);
}

void tile_shape(int dim, int tile_id, int* ty, int* tz) {
    if (dim == 2) {
        *tz = 1;
        *ty = tile_id == 1 ? 8 : (tile_id == 2 ? 4 : 16);
    } else {
        *ty = tile_id == 1 ? 8 : 4;
        *tz = tile_id == 2 ? 8 : 4;
    }
}

}  // namespace tgdk
