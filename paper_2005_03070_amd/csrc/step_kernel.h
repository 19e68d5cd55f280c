// BiCGStab(ncyc)-Proj(k) step kernel: the fine-grid cycle of the Sec. 2.2
// box, with the restarted BiCGStab inner solver of Sec. 4.1 (van der Vorst's
// recurrences).
//
// One launch advances every running problem of a group (right-hand sides or
// grid instances) by one step of its own state machine; the host only
// enqueues launches.  A BiCGStab iteration takes two steps:
//
//   phase A (iteration i):  r_i = s_{i-1} - w t_{i-1};  e += a p_{i-1} + w s_{i-1};
//                           p_i = r_i + beta (p_{i-1} - w v_{i-1});  v_i = A p_i;
//                           partials r^.v_i, ||r_i||^2
//   phase B:                s_i = r_i - alpha v_i;  t_i = A s_i;
//                           partials s.s, t.s, t.t, r^.s, r^.t
//
// Each phase recomputes its stencil input (p_i or s_i) on the tile halo from
// the previous vectors, so the update and the stencil share one pass.  There
// are no epilogue launches: at the start of a step every workgroup of a
// problem sums the previous step's per-workgroup partials (the same values in
// the same order, hence the same bits in every workgroup) and takes the
// scalar decisions itself -- alpha = rho / r^.v; omega = t.s / t.t;
// ||r_{i+1}||^2 = s.s - 2 w t.s + w^2 t.t; rho_{i+1} = r^.s - w r^.t; the
// inner convergence and breakdown tests.  The problem's lead workgroup stores
// the resulting state for the next launch (double-buffered by launch parity),
// the counters of the report and the host-visible status mirror.
//
// When an inner cycle ends, the same step evaluates the true residual of the
// updated iterate, r = b - A (x + e + a p + w s) in float64, with the
// partials of ||r||^2, ||b||^2 and c = V^T r.  The next step takes the
// boundary decisions (Sec. 4.1 steps 3-4) and, in the lead workgroup, sums c
// and solves H d = c with the LU factors of H.  The step after it applies
// x <- x + e + a p + w s + V d and r <- r - A V d and writes the new inner
// residual and shadow vector; the first phase A of the next cycle shares its
// launch with the test of that residual.  Problems advance independently: one
// may sit at a cycle boundary while another iterates.
//
// 2-D grids: one workgroup per 64 x TY tile (walking several tiles when a
// problem has more than 1024).  3-D grids: phases A and B march along z over
// a column chunk per workgroup (march3d.h); the rare boundary actions use box
// tiles.  Included by kernels_step2d.hip and kernels_step3d.hip, which
// instantiate the two dimensions in separate translation units.
#pragma once

#include "device_common.h"
#include "launch.h"
#include "march3d.h"

namespace tgdk {

// pending x update: x += e + a p + w s (p, and on 3-D grids r_i and v_i for
// s = r_i - a v_i, from buffer pbuf)
struct Upd {
    double a, w;
    int any, pbuf;
};

// Element i (0 or 1) of a two-buffer field of the descriptor, by a select:
// a run-time index into the descriptor that k_step1 receives by value made
// the compiler copy the whole descriptor to scratch memory.
template <class T>
__device__ __forceinline__ T pick2(const T (&a)[2], int i) {
    return i ? a[1] : a[0];
}

// Start of an inner cycle from a residual of norm nu: its tolerance
// (Sec. 4.1 step 3 b, cycle_tolerance) and fresh BiCGStab scalars; returns
// the criterion taken (1, 2 or 3).
__device__ __forceinline__ int cycle_start(StepHot& N, const SolveState* st, double nu, double rho0, double& rt) {
    const int branch = cycle_tolerance(nu, N.nu0, N.tau, N.icyc, st->ncyc, st->precision, st->fp32_floor, rt);
    N.target2 = (rt * nu) * (rt * nu);
    N.rho = rho0;
    N.rho_old = 1.0;
    N.alpha = 1.0;
    N.omega = 1.0;
    N.iter = 0;
    N.inner_state = IN_RUNNING;
    N.upd_any = 0;
    return branch;
}

// Tests on the true residual nu = ||b - A x|| at a cycle boundary (or at the
// start of the solve): Sec. 4.1 steps 1 and 4; the cycle count goes up if the
// solve continues.
__device__ __forceinline__ void boundary_tests(const StepHot& H, StepHot& N, const SolveState* st, double nu,
                                               double bb) {
    if (H.first) {
        // a resumed solve keeps the schedule of its first call: nu0 and
        // tau = rtol min(||b||, nu0) come from there, and it starts at cycle
        // icyc0 + 1 (H.icyc = icyc0)
        N.bnorm = sqrt(bb);
        N.nu0 = st->nu0_in > 0.0 ? st->nu0_in : nu;
        N.tau = st->rtol * fmin(N.bnorm, N.nu0);
        if (!isfinite(nu))
            N.solve_state = SV_NONFINITE;
        else if (nu <= N.tau || nu == 0.0)
            N.solve_state = SV_CONVERGED;
        else if (H.icyc > 0 && H.icyc >= st->ncyc + st->max_extra)
            N.solve_state = SV_NOT_CONVERGED;
    } else {
        const bool broke = H.inner_state == IN_BREAK_NOUPD || H.inner_state == IN_BREAK_FULL;
        if (!isfinite(nu))
            N.solve_state = SV_NONFINITE;
        else if (nu <= N.tau)
            N.solve_state = SV_CONVERGED;
        else if (broke && H.iter == 0)
            N.solve_state = SV_BREAKDOWN;
        else if (H.icyc >= st->ncyc + st->max_extra)
            N.solve_state = SV_NOT_CONVERGED;
        else if (st->maxcyc_call > 0 && H.icyc - st->icyc0 >= st->maxcyc_call)
            N.solve_state = SV_NOT_CONVERGED;
    }
    N.first = 0;
    if (N.solve_state == SV_RUNNING) N.icyc = H.icyc + 1;
}

// Report counters of the inner iterations, read by the scribe in one batch
// before the decision: read-modify-writes through the state pointer inside
// the decision were ordered behind the scribe's other state stores (they may
// alias), one memory round trip each, and the lead workgroup ended last.
struct ScribeCnt {
    long long mvp_inner, iters_total;
    int nhist;
};

// The scalar part of a step.  Every workgroup of the problem evaluates it on
// the same inputs; only the scribe (thread 0 of the lead workgroup) writes
// the report counters (C: their values before this launch, scribe only).
// maxit: the inner iteration cap.  Returns the action of this launch.
__device__ int step_decide(const StepHot& H, const double (&s)[5], SolveState* st, int k, int dim, bool cdot,
                           int gslot, bool scribe, int maxit, const ScribeCnt& C, StepHot& N, Upd& U,
                           double& rr_out, double& rr0_out) {
    N = H;
    U = Upd{H.upd_a, H.upd_w, H.upd_any, H.pbuf};
    const int after_res = k > 0 ? M_REDUCE : M_APPLY0;
    auto end_cycle = [&](int inner, double a, double w, int any, int pbuf) {
        N.inner_state = inner;
        U = Upd{a, w, any, pbuf};
        N.upd_a = a;
        N.upd_w = w;
        N.upd_any = any;
        N.pbuf = pbuf;
        N.mode = after_res;
        return ACT_RES;
    };
    switch (H.mode) {
        case M_RES:
            N.mode = after_res;
            return ACT_RES;
        case M_B: {  // phase A partials: r^.v, ||r_i||^2
            const double sig = s[0];
            if (scribe) {
                st->mvp_inner = C.mvp_inner + 1;
                st->sigma = sig;
                st->rr_last = s[1];
            }
            if (sig == 0.0 || !isfinite(sig)) return end_cycle(IN_BREAK_NOUPD, 0.0, 0.0, H.iter != 0, 0);
            N.alpha = H.rho / sig;
            N.mode = M_A;
            return ACT_B;
        }
        case M_A: {  // phase B partials: s.s, t.s, t.t, r^.s, r^.t
            const double ss = s[0], ts = s[1], tt = s[2], rs = s[3], rt = s[4];
            N.iter = H.iter + 1;
            const int pb = ((gslot - 2) >> 1) & 1;  // p of the iteration just finished
            const int hi = scribe ? C.nhist : NHIST;
            if (scribe) {
                st->mvp_inner = C.mvp_inner + 1;
                st->iters_total = C.iters_total + 1;
            }
            if (ss <= H.target2) {
                if (hi < NHIST) {
                    st->hist[3 * hi] = H.rho;
                    st->hist[3 * hi + 1] = H.alpha;
                    st->hist[3 * hi + 2] = __builtin_nan("");
                    st->nhist = hi + 1;
                }
                rr_out = ss;
                return end_cycle(IN_HALF, H.alpha, 0.0, 1, pb);
            }
            const double omega = (tt != 0.0) ? ts / tt : 0.0;
            N.omega = omega;
            if (hi < NHIST) {
                st->hist[3 * hi] = H.rho;
                st->hist[3 * hi + 1] = H.alpha;
                st->hist[3 * hi + 2] = omega;
                st->nhist = hi + 1;
            }
            if (omega == 0.0 || !isfinite(omega)) return end_cycle(IN_BREAK_FULL, H.alpha, omega, 1, pb);
            double rr = ss - 2.0 * omega * ts + omega * omega * tt;
            if (rr < 0.0) rr = 0.0;
            rr_out = rr;
            const double rho_new = rs - omega * rt;
            if (rr <= H.target2) return end_cycle(IN_CONVERGED, H.alpha, omega, 1, pb);
            if (rho_new == 0.0 || !isfinite(rho_new)) return end_cycle(IN_BREAK_FULL, H.alpha, omega, 1, pb);
            if (N.iter >= maxit) return end_cycle(IN_MAXIT, H.alpha, omega, 1, pb);
            N.rho_old = H.rho;
            N.rho = rho_new;
            N.mode = M_B;
            return ACT_A;
        }
        case M_REDUCE:    // true residual partials: ||r||^2, ||b||^2 (c summed by the lead)
        case M_APPLY0: {  // the same plus r^.r in the inner type (no deflation)
            const double nu = sqrt(s[0]);
            boundary_tests(H, N, st, nu, s[1]);
            if (scribe) {
                st->mvp_boundary += 1;
                st->nu = nu;
                if (!H.first && H.icyc >= 1 && H.icyc <= NCYCLOG) {
                    st->cyc_iters[H.icyc - 1] = H.iter;
                    st->cyc_end[H.icyc - 1] = H.inner_state;
                }
            }
            if (N.solve_state != SV_RUNNING) {
                N.mode = M_DONE;
                return H.upd_any ? ACT_FIN : ACT_NONE;
            }
            if (H.mode == M_REDUCE) {
                if (cdot) {  // c partials in this launch, summed in the next
                    N.mode = M_SUMC;
                    return ACT_CDOT;
                }
                N.mode = dim == 3 ? M_APPLYW : M_APPLY;
                return ACT_REDUCE;
            }
            double rt;
            const int br = cycle_start(N, st, nu, s[2], rt);
            if (scribe) {
                st->branch[br] += 1;
                if (N.icyc >= 1 && N.icyc <= NCYCLOG) st->cyc_branch[N.icyc - 1] = br;
                st->rt = rt;
            }
            rr0_out = rr_out = s[0];
            N.mode = M_B;
            return H.upd_any ? ACT_FIN_A0 : ACT_A0;
        }
        case M_SUMC:
            N.mode = M_APPLYW;
            return ACT_REDUCE;
        case M_APPLYW:
            N.mode = M_APPLY;
            N.upd_any = 0;
            return ACT_APPLYW;
        case M_APPLY:
            N.mode = M_START;
            N.upd_any = 0;
            return ACT_APPLY;
        case M_START: {  // after the projection: ||r||^2, r^.r in the inner type
            const double nu = sqrt(s[0]);
            if (scribe) {
                st->mvp_boundary += 1;
                st->nproj += 1;
                st->nu = nu;
            }
            if (!isfinite(nu))
                N.solve_state = SV_NONFINITE;
            else if (nu <= N.tau)
                N.solve_state = SV_CONVERGED;
            if (N.solve_state != SV_RUNNING) {
                N.mode = M_DONE;
                return ACT_NONE;
            }
            double rt;
            const int br = cycle_start(N, st, nu, s[1], rt);
            if (scribe) {
                st->branch[br] += 1;
                if (N.icyc >= 1 && N.icyc <= NCYCLOG) st->cyc_branch[N.icyc - 1] = br;
                st->rt = rt;
            }
            rr0_out = rr_out = s[0];
            N.mode = M_B;
            return ACT_A0;
        }
        default:
            return ACT_NONE;
    }
}

// Element i of the stored deflation basis (float64 or float32, widened).
__device__ __forceinline__ double vload(const DevProb& P, long long i) {
    return P.vtype ? (double)reinterpret_cast<const float*>(P.V)[i] : reinterpret_cast<const double*>(P.V)[i];
}

// s = r_i - alpha v_i of the iteration whose update is pending, at index g:
// phase B does not store s, so it is formed from r_i and v_i with phase B's
// own expression (a = alpha whenever w != 0), which gives the same bits.
template <int DIM, class TI>
__device__ __forceinline__ TI s_at(const DevProb& P, const Upd& U, long long g) {
    const TI a = (TI)U.a;
    const TI* r = vp<const TI>(pick2(P.r2, U.pbuf));
    const TI* v = vp<const TI>(pick2(P.v, U.pbuf));
    return r[g] - a * v[g];
}

// e + a p + w s at index g of the step kernel's own vectors (padded pitch
// on 3-D grids): the pending inner update, float64.
template <int DIM, class TI>
__device__ __forceinline__ double upd_at(const DevProb& P, const Upd& U, long long g) {
    double u = (double)vp<const TI>(P.e)[g];
    if (U.a != 0.0) u += U.a * (double)vp<const TI>(pick2(P.p, U.pbuf))[g];
    if (U.w != 0.0) u += U.w * (double)s_at<DIM, TI>(P, U, g);
    return u;
}

// Value-major partial output: value v of this workgroup.
__device__ __forceinline__ gptr<double> part_at(const DevProb& P, int slot, int v, int lw) {
    return gp<double>(P.partial) + (long long)slot * P.pslot + (long long)v * P.nwg + lw;
}

// ------------------------------------------------------------ phase A
// 2-D tiles (the 2-D actions index every vector with pitch n_x: their
// problems are not padded).  Every load of the stencil input's sources (own points and halo
// slots) is issued first, from clamped addresses (points outside the domain
// read the zero page), so all of them are in flight together; then the
// stencil input goes to LDS and the outputs are formed.  e and r^ are read
// where the outputs are formed: issuing them with the first loads costs
// registers and measured slower (phase A at 1023^2 fp64: 21.3 to 21.9 us
// against 20.7 us).
template <class Cfg, int DIM, bool VAR, bool FIRST, class TI>
__device__ __forceinline__ void phase_a(const DevProb& P, int lw, int gslot, bool fin, const StepHot& N,
                                        const Upd& U, TI* L, double* sh) {
    using HL = Halo<Cfg, DIM>;
    const DevOp& op = P.op;
    const int pb = (gslot >> 1) & 1;
    const gptr<TI> __restrict__ pnew = gp<TI>(pick2(P.p, pb));
    const gptr<const TI> __restrict__ pold = gp<const TI>(pick2(P.p, pb ^ 1));
    const gptr<TI> __restrict__ vnew = gp<TI>(pick2(P.v, pb));
    const gptr<const TI> __restrict__ vold = gp<const TI>(pick2(P.v, pb ^ 1));
    const gptr<const TI> rin = gp<const TI>(P.rin);
    const gptr<TI> __restrict__ rnew = gp<TI>(pick2(P.r2, pb));
    const gptr<const TI> __restrict__ rold = gp<const TI>(pick2(P.r2, pb ^ 1));
    const gptr<const TI> __restrict__ rhat = gp<const TI>(P.rhat);
    const gptr<const TI> __restrict__ tv_ = gp<const TI>(P.t);
    const gptr<TI> e = gp<TI>(P.e);
    const gptr<const TI> zero = gp<const TI>(op.zero);
    auto at = [&](gptr<const TI> arr, long long g) { return g >= 0 ? arr + g : zero; };
    const TI alpha = (TI)N.alpha, omega = (TI)N.omega;
    const TI beta = FIRST ? TI(0) : (TI)((N.rho / N.rho_old) * (N.alpha / N.omega));
    double acc[2] = {0.0, 0.0};
    for (int tile = lw; tile < P.ntiles; tile += P.nwg) {
        const TilePos tp = tile_pos<Cfg>(tile, P.tx, P.ty);
        long long gq[Cfg::PPT];
        int cq[Cfg::PPT];
#pragma unroll
        for (int q = 0; q < Cfg::PPT; ++q) {
            int gx, gy, gz;
            point_coords<Cfg>(q, tp, gx, gy, gz, cq[q]);
            gq[q] = inside(op, gx, gy, gz) ? gidx(op, gx, gy, gz) : -1;
        }
        int ch[HL::HK];
        long long gh[HL::HK];
        halo_slots<Cfg, DIM>(tp, op, ch, gh);
        // loads of the stencil input's sources: own points and halo slots
        TI a0[Cfg::PPT], a1[Cfg::PPT], a2[Cfg::PPT], a3[Cfg::PPT];
        TI h0[HL::HK], h1[HL::HK], h2[HL::HK], h3[HL::HK];
#pragma unroll
        for (int q = 0; q < Cfg::PPT; ++q) {
            if (FIRST) {
                a0[q] = *at(rin, gq[q]);
            } else {
                a0[q] = *at(rold, gq[q]);
                a1[q] = *at(tv_, gq[q]);
                a2[q] = *at(pold, gq[q]);
                a3[q] = *at(vold, gq[q]);
            }
        }
#pragma unroll
        for (int h = 0; h < HL::HK; ++h) {
            if (FIRST) {
                h0[h] = *at(rin, gh[h]);
            } else {
                h0[h] = *at(rold, gh[h]);
                h1[h] = *at(tv_, gh[h]);
                h2[h] = *at(pold, gh[h]);
                h3[h] = *at(vold, gh[h]);
            }
        }
        if (fin) {
#pragma unroll
            for (int q = 0; q < Cfg::PPT; ++q)
                if (gq[q] >= 0) P.x[gq[q]] += upd_at<DIM, TI>(P, U, gq[q]);
        }
        // stencil input p_i on the tile and its halo (s = r - alpha v of the
        // last phase B formed again: it is not stored)
        TI rq[Cfg::PPT];
#pragma unroll
        for (int q = 0; q < Cfg::PPT; ++q) {
            TI pv;
            if (FIRST) {
                rq[q] = a0[q];
                pv = rq[q];
            } else {
                const TI sv = a0[q] - alpha * a3[q];
                rq[q] = sv - omega * a1[q];
                pv = rq[q] + beta * (a2[q] - omega * a3[q]);
            }
            L[cq[q]] = pv;
        }
#pragma unroll
        for (int h = 0; h < HL::HK; ++h) {
            if (ch[h] < 0) continue;
            if (FIRST) {
                L[ch[h]] = h0[h];
            } else {
                const TI sv = h0[h] - alpha * h3[h];
                const TI rv = sv - omega * h1[h];
                L[ch[h]] = rv + beta * (h2[h] - omega * h3[h]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Cfg::PPT; ++q) {
            if (gq[q] < 0) continue;
            const long long g = gq[q];
            const TI vv = stencil_row_t<Cfg, DIM, VAR, TI>(op, L, cq[q], g);
            st_stream<DIM>(&pnew[g], L[cq[q]]);
            st_stream<DIM>(&vnew[g], vv);
            st_stream<DIM>(&rnew[g], rq[q]);
            if (FIRST)
                st_stream<DIM>(&e[g], TI(0));
            else
                st_stream<DIM>(&e[g], e[g] + alpha * a2[q] + omega * (a0[q] - alpha * a3[q]));
            acc[0] += (double)rhat[g] * (double)vv;
            acc[1] += (double)rq[q] * (double)rq[q];
        }
        __syncthreads();
    }
    double tot;
    block_sum<2, true>(acc, sh, tot);
    if (threadIdx.x < 2) *part_at(P, gslot & 1, threadIdx.x, lw) = tot;
}

// ------------------------------------------------------------ phase B
// 2-D tiles, loads first as in phase_a.
template <class Cfg, int DIM, bool VAR, class TI>
__device__ __forceinline__ void phase_b(const DevProb& P, int lw, int gslot, const StepHot& N, TI* L, double* sh) {
    using HL = Halo<Cfg, DIM>;
    const DevOp& op = P.op;
    const int pb = ((gslot - 1) >> 1) & 1;  // r and v of this iteration's phase A
    const gptr<const TI> __restrict__ v = gp<const TI>(pick2(P.v, pb));
    const gptr<const TI> __restrict__ rin = gp<const TI>(pick2(P.r2, pb));
    const gptr<const TI> __restrict__ rhat = gp<const TI>(P.rhat);
    const gptr<TI> __restrict__ tt_ = gp<TI>(P.t);
    const gptr<const TI> zero = gp<const TI>(op.zero);
    auto at = [&](gptr<const TI> arr, long long g) { return g >= 0 ? arr + g : zero; };
    const TI alpha = (TI)N.alpha;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int tile = lw; tile < P.ntiles; tile += P.nwg) {
        const TilePos tp = tile_pos<Cfg>(tile, P.tx, P.ty);
        long long gq[Cfg::PPT];
        int cq[Cfg::PPT];
#pragma unroll
        for (int q = 0; q < Cfg::PPT; ++q) {
            int gx, gy, gz;
            point_coords<Cfg>(q, tp, gx, gy, gz, cq[q]);
            gq[q] = inside(op, gx, gy, gz) ? gidx(op, gx, gy, gz) : -1;
        }
        int ch[HL::HK];
        long long gh[HL::HK];
        halo_slots<Cfg, DIM>(tp, op, ch, gh);
        // r^ at the own points is issued with the stencil's loads (phase B
        // at 1023^2 fp64: 14.8 us against 16.3 us when read at the outputs)
        TI rq[Cfg::PPT], vq[Cfg::PPT], hq[Cfg::PPT], hr[HL::HK], hv[HL::HK];
#pragma unroll
        for (int q = 0; q < Cfg::PPT; ++q) {
            rq[q] = *at(rin, gq[q]);
            vq[q] = *at(v, gq[q]);
            hq[q] = *at(rhat, gq[q]);
        }
#pragma unroll
        for (int h = 0; h < HL::HK; ++h) {
            hr[h] = *at(rin, gh[h]);
            hv[h] = *at(v, gh[h]);
        }
#pragma unroll
        for (int q = 0; q < Cfg::PPT; ++q) L[cq[q]] = rq[q] - alpha * vq[q];
#pragma unroll
        for (int h = 0; h < HL::HK; ++h)
            if (ch[h] >= 0) L[ch[h]] = hr[h] - alpha * hv[h];
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Cfg::PPT; ++q) {
            if (gq[q] < 0) continue;
            const long long g = gq[q];
            const TI sv = L[cq[q]];
            const TI tv = stencil_row_t<Cfg, DIM, VAR, TI>(op, L, cq[q], g);
            st_stream<DIM>(&tt_[g], tv);
            const double rh = (double)hq[q];
            const double sd = (double)sv, td = (double)tv;
            acc[0] += sd * sd;
            acc[1] += td * sd;
            acc[2] += td * td;
            acc[3] += rh * sd;
            acc[4] += rh * td;
        }
        __syncthreads();
    }
    double tot;
    block_sum<5, true>(acc, sh, tot);
    if (threadIdx.x < 5) *part_at(P, gslot & 1, threadIdx.x, lw) = tot;
}

// c partial of one tile: wave w adds V_j^T r over the tile to csum[j] for
// j = w, w + 4, ... (r of the tile in LDS in tile order).
template <class Cfg, class TV>
__device__ __forceinline__ void c_partials(const DevProb& P, const TilePos& tp, const TV* __restrict__ V,
                                           const double* __restrict__ L, double* csum) {
    const DevOp& op = P.op;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    constexpr int R = Cfg::PTS / 64;
    constexpr int RB = R < 8 ? R : 8;  // rows in flight (register budget)
    static_assert(R % RB == 0, "tile rows");
    const gptr<const TV> zero = gp<const TV>(op.zero);
    for (int j = w; j < P.k; j += NWAVE) {
        const gptr<const TV> Vj = gp<const TV>(V) + (long long)j * P.ldv;
        // RB rows of the column issued before their sum: points outside the
        // domain read the zero page (and their L entry is zero), so no load
        // is guarded (a guarded load compiles to a branch and a full wait)
        double a = 0.0;
        for (int m0 = 0; m0 < R; m0 += RB) {
            TV v[RB];
#pragma unroll
            for (int u = 0; u < RB; ++u) {
                const int l = lane + 64 * (m0 + u);
                const int gx = tp.x0 + lane, gy = tp.y0 + (l / 64) % Cfg::TY, gz = tp.z0 + l / (64 * Cfg::TY);
                v[u] = *(inside(op, gx, gy, gz) ? Vj + gidx(op, gx, gy, gz) : zero);
            }
#pragma unroll
            for (int u = 0; u < RB; ++u) a += (double)v[u] * L[lane + 64 * (m0 + u)];
        }
        a = wave_sum_dpp(a);
        if (lane == 0) csum[j] += a;
    }
}

// ------------------------------------------- true residual at a boundary
// r = b - A x' with x' = x + e + a p + w s formed on the fly (x is written in
// a later step, so neighbouring tiles still read the old x).  Partials:
// ||r||^2, ||b||^2, r^.r in the inner type (no deflation: the next cycle's
// inner residual and shadow vector are written here), and c = V^T r.
template <class Cfg, int DIM, bool VAR, class TI>
__device__ __forceinline__ void true_residual(const DevProb& P, int lw, int gslot, const Upd& U, double* L,
                                              double* sh, double* csum) {
    const DevOp& op = P.op;
    const int k = P.k;
    const bool start = k == 0;
    TI* rin = vp<TI>(P.rin);
    TI* rhat = vp<TI>(P.rhat);
    const bool sep = (void*)rin != (void*)P.r;
    const long long ldv = P.ldv;
    const double* __restrict__ x = P.x;
    const double* __restrict__ b = P.b;
    auto xval = [&](long long g) -> double { return U.any ? x[g] + upd_at<DIM, TI>(P, U, g) : x[g]; };
    for (int i = threadIdx.x; i < k; i += NT) csum[i] = 0.0;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int tile = lw; tile < P.ntiles; tile += P.nwg) {
        const TilePos tp = tile_pos<Cfg>(tile, P.tx, P.ty);
        long long gq[Cfg::PPT];
        int cq[Cfg::PPT];
        bool okq[Cfg::PPT];
        double bq[Cfg::PPT], rv[Cfg::PPT];
#pragma unroll
        for (int q = 0; q < Cfg::PPT; ++q) {
            int gx, gy, gz;
            point_coords<Cfg>(q, tp, gx, gy, gz, cq[q]);
            okq[q] = inside(op, gx, gy, gz);
            gq[q] = okq[q] ? gidx(op, gx, gy, gz) : 0;
            L[cq[q]] = okq[q] ? xval(gq[q]) : 0.0;
            bq[q] = okq[q] ? b[gq[q]] : 0.0;
        }
        fill_halo<Cfg, DIM, double>(L, tp, op, xval);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Cfg::PPT; ++q) {
            rv[q] = 0.0;
            if (!okq[q]) continue;
            const long long g = gq[q];
            const double r = bq[q] - stencil_row_t<Cfg, DIM, VAR, double>(op, L, cq[q], g);
            rv[q] = r;
            P.r[g] = r;
            acc[0] += r * r;
            acc[1] += bq[q] * bq[q];
            if (start) {
                const TI ri = (TI)r;
                if (sep) rin[g] = ri;
                rhat[g] = ri;
                acc[2] += (double)ri * (double)ri;
            }
        }
        if (k > 0) {
            // c partial: r goes to LDS in tile order; wave w forms columns
            // w, w + 4, ... with coalesced row reads of V
            __syncthreads();
#pragma unroll
            for (int q = 0; q < Cfg::PPT; ++q) L[threadIdx.x + q * NT] = rv[q];
            __syncthreads();
            if (P.vtype)
                c_partials<Cfg>(P, tp, reinterpret_cast<const float*>(P.Vl), L, csum);
            else
                c_partials<Cfg>(P, tp, reinterpret_cast<const double*>(P.Vl), L, csum);
        }
        __syncthreads();
    }
    double tot;
    block_sum<3, true>(acc, sh, tot);
    const int slot = gslot & 1;
    if (threadIdx.x < 3) *part_at(P, slot, threadIdx.x, lw) = tot;
    for (int i = threadIdx.x; i < k; i += NT) *part_at(P, slot, 3 + i, lw) = csum[i];
}

// -------------------------------------------- projection coefficients
// Lead workgroup: c = V^T r summed over the workgroups, then d = H^{-1} c
// with the inverse formed on the host from the LU factors of H (one parallel
// pass instead of 2k dependent substitution steps).
__device__ __forceinline__ void projection_coefficients(const DevProb& P, int gslot, SolveState* st, double* y,
                                                        double* sh) {
    const int k = P.k;
    const int nwg = P.nwg;
    const double* part = P.partial + (long long)((gslot & 1) ^ 1) * P.pslot + 3LL * nwg;
    // wave w sums columns w, w + 4, ...; lane l takes workgroups l, l + 64, ...
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int c = w; c < k; c += NWAVE) {
        const double* col = part + (long long)c * nwg;
        double a = 0.0;
#pragma unroll 4
        for (int t = lane; t < nwg; t += 64) a += col[t];
        a = wave_sum_dpp(a);
        if (lane == 0) y[c] = a;
    }
    __syncthreads();
    const double* __restrict__ X = P.hinv;  // column-major k x k
    for (int i = threadIdx.x; i < k; i += NT) {
        double di = 0.0;
        for (int j = 0; j < k; ++j) di += X[(long long)j * k + i] * y[j];
        st->d[i] = di;
        st->cvec[i] = y[i];
    }
}

// ----------------------------------------------- projection applied
// w = V d on the tile and its halo (LDS, float64); x <- x + upd + w and
// r <- r - A w on the tile; the new cycle's inner residual and shadow vector;
// partials ||r||^2 and r^.r in the inner type.
template <class Cfg, int DIM, bool VAR, class TI>
__device__ __forceinline__ void apply_projection(const DevProb& P, int lw, int gslot, const Upd& U,
                                                 const SolveState* st, double* L, double* sh, double* dsh) {
    const DevOp& op = P.op;
    const int k = P.k;
    const long long ldv = P.ldv;
    TI* rin = vp<TI>(P.rin);
    TI* rhat = vp<TI>(P.rhat);
    const bool sep = (void*)rin != (void*)P.r;
    for (int i = threadIdx.x; i < k; i += NT) dsh[i] = st->d[i];
    __syncthreads();
    auto wval = [&](long long g) {
        double w = 0.0;
        for (int j = 0; j < k; ++j) w += vload(P, (long long)j * ldv + g) * dsh[j];
        return w;
    };
    double acc[2] = {0.0, 0.0};
    for (int tile = lw; tile < P.ntiles; tile += P.nwg) {
        const TilePos tp = tile_pos<Cfg>(tile, P.tx, P.ty);
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
#pragma unroll
        for (int q = 0; q < Cfg::PPT; ++q) {
            if (!okq[q]) continue;
            const long long g = gq[q];
            const int c = cq[q];
            double xv = P.x[g];
            if (U.any) xv += upd_at<DIM, TI>(P, U, g);
            P.x[g] = xv + L[c];
            const double rv = P.r[g] - stencil_row_t<Cfg, DIM, VAR, double>(op, L, c, g);
            P.r[g] = rv;
            acc[0] += rv * rv;
            const TI ri = (TI)rv;
            if (sep) rin[g] = ri;
            rhat[g] = ri;
            acc[1] += (double)ri * (double)ri;
        }
        __syncthreads();
    }
    double tot;
    block_sum<2, true>(acc, sh, tot);
    if (threadIdx.x < 2) *part_at(P, gslot & 1, threadIdx.x, lw) = tot;
}

// x <- x + e + a p + w s on this workgroup's tiles (the solve stops here).
template <class Cfg, int DIM, class TI>
__device__ __forceinline__ void fold_update(const DevProb& P, int lw, const Upd& U) {
    const DevOp& op = P.op;
    for (int tile = lw; tile < P.ntiles; tile += P.nwg) {
        const TilePos tp = tile_pos<Cfg>(tile, P.tx, P.ty);
#pragma unroll
        for (int q = 0; q < Cfg::PPT; ++q) {
            int gx, gy, gz, c;
            point_coords<Cfg>(q, tp, gx, gy, gz, c);
            if (!inside(op, gx, gy, gz)) continue;
            P.x[gidx(op, gx, gy, gz)] += upd_at<DIM, TI>(P, U, pidx(op, gx, gy, gz));
        }
    }
}

// ------------------------------------------------ 3-D phases by z marching
// The same arithmetic as phase_a / phase_b (same expressions, same order),
// written as march_chunk phases: raw loads per point and plane, the stencil
// input, and the outputs at the plane being computed.  Unlike the 2-D
// phases, phase B stores t but not s: phase A forms s = r_i - alpha v_i
// again from r_i and v_i, which it reads in place of s (r_i kept in two
// buffers alternating with p and v, since phase A reads the old one on the
// ring while writing the new one).  One vector write fewer per iteration.
template <class TI>
struct MarchA {  // phase A of iteration i > 0
    const TI *ro, *t, *po, *vo, *rh, *zero;
    TI *pnew, *vnew, *rnew, *e;
    TI alpha, omega, beta;
    double acc[2] = {0.0, 0.0};
    struct Own {
        TI ro, t, po, vo, e, rh;
    };
    struct Ring {
        TI ro, t, po, vo;
    };
    __device__ __forceinline__ const TI* at(const TI* a, long long g) const { return g >= 0 ? a + g : zero; }
    __device__ __forceinline__ void load(Own& o, long long g, long long) const {
        o.ro = *at(ro, g);
        o.t = *at(t, g);
        o.po = *at(po, g);
        o.vo = *at(vo, g);
        o.e = *at(e, g);
        o.rh = *at(rh, g);
    }
    __device__ __forceinline__ void load(Ring& o, long long g, long long) const {
        o.ro = *at(ro, g);
        o.t = *at(t, g);
        o.po = *at(po, g);
        o.vo = *at(vo, g);
    }
    template <class R>
    __device__ __forceinline__ TI value(const R& o) const {
        const TI s = o.ro - alpha * o.vo;  // phase B's s
        const TI r = s - omega * o.t;
        return r + beta * (o.po - omega * o.vo);
    }
    static constexpr bool PLANE_HOOK = false;
    __device__ __forceinline__ void plane_done(const Chunk&, int) {}
    __device__ __forceinline__ void emit(int, long long g, long long, const Own& c, TI y) {
        const TI s = c.ro - alpha * c.vo;
        const TI r = s - omega * c.t;
        pnew[g] = r + beta * (c.po - omega * c.vo);
        vnew[g] = y;
        rnew[g] = r;
        e[g] = c.e + alpha * c.po + omega * s;
        acc[0] += (double)c.rh * (double)y;
        acc[1] += (double)r * (double)r;
    }
};

template <class TI>
struct MarchA0 {  // phase A of iteration 0 (r_0 copied into r2), optionally folding the last update into x
    const TI *rin, *rh, *zero;
    TI *pnew, *vnew, *rnew, *e;
    const DevProb* P;
    Upd U;
    bool fin;
    double acc[2] = {0.0, 0.0};
    struct Own {
        TI r, rh;
    };
    struct Ring {
        TI r;
    };
    __device__ __forceinline__ const TI* at(const TI* a, long long g) const { return g >= 0 ? a + g : zero; }
    __device__ __forceinline__ void load(Own& o, long long g, long long) const {
        o.r = *at(rin, g);
        o.rh = *at(rh, g);
    }
    __device__ __forceinline__ void load(Ring& o, long long g, long long) const { o.r = *at(rin, g); }
    template <class R>
    __device__ __forceinline__ TI value(const R& o) const {
        return o.r;
    }
    static constexpr bool PLANE_HOOK = false;
    __device__ __forceinline__ void plane_done(const Chunk&, int) {}
    __device__ __forceinline__ void emit(int, long long g, long long gu, const Own& c, TI y) {
        if (fin) P->x[gu] += upd_at<3, TI>(*P, U, g);
        pnew[g] = c.r;
        vnew[g] = y;
        rnew[g] = c.r;
        e[g] = TI(0);
        acc[0] += (double)c.rh * (double)y;
        acc[1] += (double)c.r * (double)c.r;
    }
};

template <class TI>
struct MarchB {  // phase B (s is not stored: phase A forms it again)
    const TI *rin, *v, *rh, *zero;
    TI* t;
    TI alpha;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    struct Own {
        TI r, v, rh;
    };
    struct Ring {
        TI r, v;
    };
    __device__ __forceinline__ const TI* at(const TI* a, long long g) const { return g >= 0 ? a + g : zero; }
    __device__ __forceinline__ void load(Own& o, long long g, long long) const {
        o.r = *at(rin, g);
        o.v = *at(v, g);
        o.rh = *at(rh, g);
    }
    __device__ __forceinline__ void load(Ring& o, long long g, long long) const {
        o.r = *at(rin, g);
        o.v = *at(v, g);
    }
    template <class R>
    __device__ __forceinline__ TI value(const R& o) const {
        return o.r - alpha * o.v;
    }
    static constexpr bool PLANE_HOOK = false;
    __device__ __forceinline__ void plane_done(const Chunk&, int) {}
    __device__ __forceinline__ void emit(int, long long g, long long, const Own& c, TI y) {
        const TI sv = c.r - alpha * c.v;
        t[g] = y;
        const double rh = (double)c.rh, sd = (double)sv, td = (double)y;
        acc[0] += sd * sd;
        acc[1] += td * sd;
        acc[2] += td * td;
        acc[3] += rh * sd;
        acc[4] += rh * td;
    }
};

// z-marching tile of the 3-D step kernel: 64 x 8 (two points per thread and
// plane, so that four planes of phase A's six raw values stay in registers)
template <class TI>
using StepMarch = March<8>;

template <bool VAR, class TI, class Ph, int NV>
__device__ __forceinline__ void march_phase(const DevProb& P, int lw, int gslot, Ph& ph, TI* L, double* sh) {
    using M = StepMarch<TI>;
    if (lw < P.nchunks) {
        const Chunk k = chunk_of<M>(lw, P.mcx, P.mcy, P.mz, P.op.nz);
        march_chunk<M, VAR, TI>(P.op, k, L, ph);
    }
    double tot;
    block_sum<NV, true>(ph.acc, sh, tot);
    if (threadIdx.x < NV) *part_at(P, gslot & 1, threadIdx.x, lw) = tot;
}

template <bool VAR, class TI>
__device__ __forceinline__ void march_a(const DevProb& P, int lw, int gslot, bool first, bool fin, const StepHot& N,
                                        const Upd& U, TI* L, double* sh) {
    const int pb = (gslot >> 1) & 1;
    const TI* zero = reinterpret_cast<const TI*>(P.op.zero);
    if (first) {
        MarchA0<TI> ph{vp<const TI>(P.rin), vp<const TI>(P.rhat), zero, vp<TI>(pick2(P.p, pb)), vp<TI>(pick2(P.v, pb)),
                       vp<TI>(pick2(P.r2, pb)), vp<TI>(P.e), &P, U, fin};
        march_phase<VAR, TI, MarchA0<TI>, 2>(P, lw, gslot, ph, L, sh);
    } else {
        const TI alpha = (TI)N.alpha, omega = (TI)N.omega;
        const TI beta = (TI)((N.rho / N.rho_old) * (N.alpha / N.omega));
        MarchA<TI> ph{vp<const TI>(pick2(P.r2, pb ^ 1)), vp<const TI>(P.t), vp<const TI>(pick2(P.p, pb ^ 1)),
                      vp<const TI>(pick2(P.v, pb ^ 1)), vp<const TI>(P.rhat), zero, vp<TI>(pick2(P.p, pb)), vp<TI>(pick2(P.v, pb)),
                      vp<TI>(pick2(P.r2, pb)), vp<TI>(P.e), alpha, omega, beta};
        march_phase<VAR, TI, MarchA<TI>, 2>(P, lw, gslot, ph, L, sh);
    }
}

template <bool VAR, class TI>
__device__ __forceinline__ void march_b(const DevProb& P, int lw, int gslot, const StepHot& N, TI* L, double* sh) {
    const int pb = ((gslot - 1) >> 1) & 1;
    MarchB<TI> ph{vp<const TI>(pick2(P.r2, pb)), vp<const TI>(pick2(P.v, pb)), vp<const TI>(P.rhat),
                  reinterpret_cast<const TI*>(P.op.zero), vp<TI>(P.t), (TI)N.alpha};
    march_phase<VAR, TI, MarchB<TI>, 5>(P, lw, gslot, ph, L, sh);
}

// --------------------------------------- 3-D cycle boundary by z marching
// True residual r = b - A x' with x' = x + e + a p + w s formed on the fly,
// with its partials.  c = V^T r: a float32 V is read in a second pass over
// the workgroup's own chunk (r read back after a workgroup barrier,
// chunk_columns); a float64 V in the next launch over contiguous ranges
// (flat_cdot).  Measured at 255^3 with 41 vectors: the chunk pass costs
// about 1.2 ms per boundary with a float64 V and 0.76 ms with a float32 V,
// the contiguous pass 1.09 ms and 1.35 ms; the float32 contiguous pass
// issues half-width loads and re-reads r once per column group.
template <class TI>
struct MarchRes {
    const double *x, *b;
    const TI *e, *p, *ri, *vi;  // pending update: e + a p + w (r_i - a v_i)
    const double* zero64;
    const TI* zeroT;
    Upd U;
    double* r;
    TI *rin, *rhat;
    bool start, sep;
    double acc[3] = {0.0, 0.0, 0.0};
    static constexpr bool PLANE_HOOK = false;
    struct Own {
        double x, b;
        TI e, p, ri, vi;
    };
    struct Ring {
        double x;
        TI e, p, ri, vi;
    };
    // x and b are caller vectors (unpadded index gu), e, p, r_i, v_i the
    // step kernel's own (padded index g)
    template <class R>
    __device__ __forceinline__ void load_upd(R& o, long long g, long long gu) const {
        o.x = *(gu >= 0 ? x + gu : zero64);
        o.e = *(U.any && g >= 0 ? e + g : zeroT);
        o.p = *(U.any && U.a != 0.0 && g >= 0 ? p + g : zeroT);
        const bool sw = U.any && U.w != 0.0 && g >= 0;
        o.ri = *(sw ? ri + g : zeroT);
        o.vi = *(sw ? vi + g : zeroT);
    }
    __device__ __forceinline__ void load(Own& o, long long g, long long gu) const {
        load_upd(o, g, gu);
        o.b = *(gu >= 0 ? b + gu : zero64);
    }
    __device__ __forceinline__ void load(Ring& o, long long g, long long gu) const { load_upd(o, g, gu); }
    template <class R>
    __device__ __forceinline__ double value(const R& o) const {
        if (!U.any) return o.x;
        double u = (double)o.e;
        if (U.a != 0.0) u += U.a * (double)o.p;
        if (U.w != 0.0) {
            const TI a = (TI)U.a;
            u += U.w * (double)(o.ri - a * o.vi);  // s, as s_at forms it
        }
        return o.x + u;
    }
    __device__ __forceinline__ void emit(int, long long g, long long, const Own& c, double y) {
        const double rr = c.b - y;
        r[g] = rr;
        acc[0] += rr * rr;
        acc[1] += c.b * c.b;
        if (start) {
            const TI ri = (TI)rr;
            if (sep) rin[g] = ri;
            rhat[g] = ri;
            acc[2] += (double)ri * (double)ri;
        }
    }
    __device__ __forceinline__ void plane_done(const Chunk&, int) {}
};

// c partial of one chunk (float32 V): the workgroup streams the chunk's
// points (thread t takes points t, t + 256, ... in x-y-z order, coalesced)
// against four columns of V at a time, reading r once per group of columns;
// per-thread sums are combined by block_sum, so the order is fixed.
template <class M>
__device__ __forceinline__ void chunk_columns(const DevProb& P, const Chunk& c, const float* __restrict__ V,
                                              double* csum, double* sh) {
    const DevOp& op = P.op;
    const long long plane = (long long)op.nx * op.ny;   // V: unpadded
    const long long pplane = (long long)op.px * op.ny;  // r: padded
    const double* __restrict__ r = P.r;
    const int k = P.k;
    const int npts = 64 * M::MY * (c.z1 - c.z0);
    for (int j0 = 0; j0 < k; j0 += 4) {
        double a[4] = {0.0, 0.0, 0.0, 0.0};
        const float* __restrict__ Vj[4];
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) Vj[jj] = V + (long long)(j0 + jj < k ? j0 + jj : j0) * P.ldv;
        // no guarded loads (a guarded load compiles to a branch and a full
        // wait): points outside the domain read the zero page for r and V
        const gptr<const double> zr = gp<const double>(op.zero);
        const gptr<const float> zv = gp<const float>(op.zero);
#pragma unroll 4
        for (int l = threadIdx.x; l < npts; l += NT) {
            const int gx = c.x0 + (l & 63), gy = c.y0 + ((l >> 6) % M::MY), z = c.z0 + l / (64 * M::MY);
            const bool in = gx < op.nx && gy < op.ny;
            const long long g = z * plane + (long long)gy * op.nx + gx;
            const long long gpad = z * pplane + (long long)gy * op.px + gx;
            const double rv = *(in ? gp<const double>(r) + gpad : zr);
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) a[jj] += (double)*(in ? gp<const float>(Vj[jj]) + g : zv) * rv;
        }
        double tot;
        block_sum<4, true>(a, sh, tot);
        if (threadIdx.x < 4 && j0 + threadIdx.x < k) csum[j0 + threadIdx.x] = tot;
    }
}

template <bool VAR, class TI>
__device__ __forceinline__ void march_res(const DevProb& P, int lw, int gslot, const Upd& U, double* Lbox,
                                          double* sh, double* csum) {
    using M = StepMarch<TI>;
    const int k = P.k;
    const bool fused_c = k > 0 && P.vtype;
    if (fused_c)
        for (int i = threadIdx.x; i < k; i += NT) csum[i] = 0.0;
    TI* rin = vp<TI>(P.rin);
    MarchRes<TI> ph{P.x, P.b, vp<const TI>(P.e), vp<const TI>(pick2(P.p, U.pbuf)),
                    vp<const TI>(pick2(P.r2, U.pbuf)), vp<const TI>(pick2(P.v, U.pbuf)),
                    reinterpret_cast<const double*>(P.op.zero), reinterpret_cast<const TI*>(P.op.zero), U, P.r,
                    rin, vp<TI>(P.rhat), k == 0, (void*)rin != (void*)P.r};
    if (lw < P.nchunks) {
        const Chunk c = chunk_of<M>(lw, P.mcx, P.mcy, P.mz, P.op.nz);
        // the 64 x 8 chunk as two 64 x 4 half columns: one point per thread
        // and plane keeps the residual's raw loads within the register
        // budget of the whole kernel
        using MH = March<M::MY / 2>;
        Chunk h = c;
        march_chunk<MH, VAR, double>(P.op, h, Lbox, ph);
        h.y0 += MH::MY;
        if (h.y0 < P.op.ny) march_chunk<MH, VAR, double>(P.op, h, Lbox, ph);
        if (fused_c) {
            __syncthreads();  // r of the chunk, written above, is read back below
            chunk_columns<M>(P, c, reinterpret_cast<const float*>(P.Vl), csum, sh);
        }
    }
    __syncthreads();
    double tot;
    block_sum<3, true>(ph.acc, sh, tot);
    const int slot = gslot & 1;
    if (threadIdx.x < 3) *part_at(P, slot, threadIdx.x, lw) = tot;
    if (fused_c)
        for (int i = threadIdx.x; i < k; i += NT) *part_at(P, slot, 3 + i, lw) = csum[i];
}

// ------------- 3-D c = V^T r over contiguous ranges (ACT_CDOT, float64 V)
// Workgroup lw takes the points [lw L, (lw + 1) L) of the unpadded index
// (L a multiple of 64), so every column load of a wave is 64 consecutive
// entries of V (512 bytes); r, stored with the padded pitch, is read at
// index g + (g / n_x)(px - n_x).  CH columns per pass over the range (r
// re-read from cache by later passes); a column past k re-reads the pass's
// first and is masked on its factor, so every load of a point is issued
// unconditionally.
__device__ __forceinline__ void flat_cdot(const DevProb& P, int lw, int gslot, double* sh) {
    using TV = double;
    constexpr int CH = 8;
    const DevOp& op = P.op;
    const long long n = op.n;
    const long long L = ((n + P.nwg - 1) / P.nwg + 63) / 64 * 64;
    const long long g0 = (long long)lw * L, g1 = g0 + L < n ? g0 + L : n;
    const gptr<const TV> V = gp<const TV>(P.Vl);
    const gptr<const double> r = gp<const double>(P.r);
    const int k = P.k;
    const double nx = (double)op.nx;
    const long long pad = op.px - op.nx;
    for (int j0 = 0; j0 < k; j0 += CH) {
        const int nc = k - j0 < CH ? k - j0 : CH;
        double a[CH];
#pragma unroll
        for (int jj = 0; jj < CH; ++jj) a[jj] = 0.0;
        gptr<const TV> Vj[CH];
#pragma unroll
        for (int jj = 0; jj < CH; ++jj) Vj[jj] = V + (long long)(j0 + (jj < nc ? jj : 0)) * P.ldv;
#pragma unroll 2
        for (long long g = g0 + threadIdx.x; g < g1; g += NT) {
            // the row (y, z) of g: a double division is exact here (g < 2^53
            // and g / n_x lies at least 1 / n_x away from the next integer)
            const long long row = (long long)((double)g / nx);
            const double rv = r[g + row * pad];
#pragma unroll
            for (int jj = 0; jj < CH; ++jj) a[jj] += (jj < nc ? (double)Vj[jj][g] : 0.0) * rv;
        }
        double tot;
        block_sum<CH, true>(a, sh, tot);
        if (threadIdx.x < nc) *part_at(P, gslot & 1, 3 + j0 + threadIdx.x, lw) = tot;
    }
}

// w = V d and x <- (x + e + a p + w s) + w over the workgroup's contiguous
// range of the unpadded index (as in flat_cdot): V and x are read at g, w and
// the update's vectors at the padded index.  All k columns of a point are
// summed in one pass, eight loads in flight.
template <class TI, class TV>
__device__ __forceinline__ void apply_w_flat(const DevProb& P, int lw, const Upd& U, const TV* __restrict__ V_,
                                             const double* __restrict__ dsh) {
    const DevOp& op = P.op;
    const long long n = op.n;
    const long long L = ((n + P.nwg - 1) / P.nwg + 63) / 64 * 64;
    const long long g0 = (long long)lw * L, g1 = g0 + L < n ? g0 + L : n;
    const gptr<const TV> V = gp<const TV>(V_);
    const double nx = (double)op.nx;
    const long long pad = op.px - op.nx;
    const int k = P.k;
    for (long long g = g0 + threadIdx.x; g < g1; g += NT) {
        const long long gpad = g + (long long)((double)g / nx) * pad;
        double w = 0.0;
#pragma unroll 8
        for (int j = 0; j < k; ++j) w += (double)V[(long long)j * P.ldv + g] * dsh[j];
        P.w[gpad] = w;
        double xv = P.x[g];
        if (U.any) xv += upd_at<3, TI>(P, U, gpad);
        P.x[g] = xv + w;
    }
}

template <class TI>
__device__ __forceinline__ void apply_w(const DevProb& P, int lw, const Upd& U, const SolveState* st, double* dsh) {
    for (int i = threadIdx.x; i < P.k; i += NT) dsh[i] = st->d[i];
    __syncthreads();
    if (P.vtype)
        apply_w_flat<TI>(P, lw, U, reinterpret_cast<const float*>(P.V), dsh);
    else
        apply_w_flat<TI>(P, lw, U, reinterpret_cast<const double*>(P.V), dsh);
}

// r <- r - A w; the new cycle's inner residual and shadow vector; partials
// ||r||^2 and r^.r in the inner type.
template <class TI>
struct MarchApply {
    const double *w, *rr_, *zero;
    double* r;
    TI *rin, *rhat;
    bool sep;
    double acc[2] = {0.0, 0.0};
    static constexpr bool PLANE_HOOK = false;
    struct Own {
        double w, r;
    };
    struct Ring {
        double w;
    };
    __device__ __forceinline__ void load(Own& o, long long g, long long) const {
        o.w = *(g >= 0 ? w + g : zero);
        o.r = *(g >= 0 ? rr_ + g : zero);
    }
    __device__ __forceinline__ void load(Ring& o, long long g, long long) const { o.w = *(g >= 0 ? w + g : zero); }
    template <class R>
    __device__ __forceinline__ double value(const R& o) const {
        return o.w;
    }
    __device__ __forceinline__ void emit(int, long long g, long long, const Own& c, double y) {
        const double rv = c.r - y;
        r[g] = rv;
        acc[0] += rv * rv;
        const TI ri = (TI)rv;
        if (sep) rin[g] = ri;
        rhat[g] = ri;
        acc[1] += (double)ri * (double)ri;
    }
    __device__ __forceinline__ void plane_done(const Chunk&, int) {}
};

template <bool VAR, class TI>
__device__ __forceinline__ void march_apply(const DevProb& P, int lw, int gslot, double* Lbox, double* sh) {
    using M = StepMarch<TI>;
    TI* rin = vp<TI>(P.rin);
    MarchApply<TI> ph{P.w, P.r, reinterpret_cast<const double*>(P.op.zero), P.r, rin, vp<TI>(P.rhat),
                      (void*)rin != (void*)P.r};
    if (lw < P.nchunks) {
        const Chunk c = chunk_of<M>(lw, P.mcx, P.mcy, P.mz, P.op.nz);
        march_chunk<M, VAR, double>(P.op, c, Lbox, ph);
    }
    double tot;
    block_sum<2, true>(ph.acc, sh, tot);
    if (threadIdx.x < 2) *part_at(P, gslot & 1, threadIdx.x, lw) = tot;
}

// ------------------------------------------------------------- kernel
template <class Cfg, int DIM, bool VAR, class TI>
__device__ __forceinline__ void step_run(const DevProb& P, int wg, int gslot, unsigned long long t_begin) {
    constexpr int NBOX = (DIM == 3 && StepMarch<TI>::PLANE > Cfg::BOX) ? StepMarch<TI>::PLANE : Cfg::BOX;
    __shared__ double Lbox[NBOX];
    __shared__ double sh[NWAVE * 16];
    __shared__ double ysh[MAXK + 1];
    const int lw = wg - P.wg_begin;
    const bool lead = lw == 0;
    const bool scribe = lead && threadIdx.x == 0;
    const int cur = gslot & 1;
    SolveState* st = P.st;
    const StepHot H = load_global(&st->hot[cur ^ 1]);
    const int maxit = P.maxit;
    double s5[5];
    sum_values<5, true>(P.partial + (long long)(cur ^ 1) * P.pslot, P.nwg, s5, sh);
    ScribeCnt C{0, 0, 0};
    if (scribe) {
        C.mvp_inner = *gp<const long long>(&st->mvp_inner);
        C.iters_total = *gp<const long long>(&st->iters_total);
        C.nhist = *gp<const int>(&st->nhist);
    }
    StepHot N;
    Upd U;
    double rr = -1.0, rr0 = -1.0;
    const int act = step_decide(H, s5, st, P.k, DIM, DIM == 3 && !P.vtype, gslot, scribe, maxit, C, N, U, rr, rr0);
    if (scribe) {
        st->hot[cur] = N;
        st->solve_state = N.solve_state;
        st->inner_state = N.inner_state;
        st->icyc = N.icyc;
        st->iter = N.iter;
        st->tau = N.tau;
        st->bnorm = N.bnorm;
        st->nu0 = N.nu0;
        if (P.actlog && gslot < NSLOTLOG) P.actlog[gslot] = (unsigned char)act;
        if (P.mirror && (act != ACT_NONE || H.mode != M_DONE)) {
            Mirror* m = P.mirror;
            m->solve_state = N.solve_state;
            m->inner_state = N.inner_state;
            m->icyc = N.icyc;
            m->iter = N.iter;
            m->mode = N.mode;
            m->slot = gslot;
            m->target2 = N.target2;
            if (rr >= 0.0) m->rr = rr;
            if (rr0 >= 0.0) m->rr0 = rr0;
        }
    }
    TI* L = reinterpret_cast<TI*>(Lbox);
    switch (act) {
        case ACT_A:
        case ACT_A0:
        case ACT_FIN_A0:
            if constexpr (DIM == 3)
                march_a<VAR, TI>(P, lw, gslot, act != ACT_A, act == ACT_FIN_A0, N, U, L, sh);
            else if (act == ACT_A)
                phase_a<Cfg, DIM, VAR, false, TI>(P, lw, gslot, false, N, U, L, sh);
            else
                phase_a<Cfg, DIM, VAR, true, TI>(P, lw, gslot, act == ACT_FIN_A0, N, U, L, sh);
            break;
        case ACT_B:
            if constexpr (DIM == 3)
                march_b<VAR, TI>(P, lw, gslot, N, L, sh);
            else
                phase_b<Cfg, DIM, VAR, TI>(P, lw, gslot, N, L, sh);
            break;
        case ACT_RES:
            if constexpr (DIM == 3)
                march_res<VAR, TI>(P, lw, gslot, U, Lbox, sh, ysh);
            else
                true_residual<Cfg, DIM, VAR, TI>(P, lw, gslot, U, Lbox, sh, ysh);
            break;
        case ACT_APPLYW:
            apply_w<TI>(P, lw, U, st, ysh);
            break;
        case ACT_CDOT:
            if constexpr (DIM == 3) flat_cdot(P, lw, gslot, sh);
            break;
        case ACT_REDUCE:
            if (lead) projection_coefficients(P, gslot, st, ysh, sh);
            break;
        case ACT_APPLY:
            if constexpr (DIM == 3)
                march_apply<VAR, TI>(P, lw, gslot, Lbox, sh);
            else
                apply_projection<Cfg, DIM, VAR, TI>(P, lw, gslot, U, st, Lbox, sh, ysh);
            break;
        case ACT_FIN:
            fold_update<Cfg, DIM, TI>(P, lw, U);
            break;
        default:
            break;
    }
    // measurement: this workgroup's start and end on the constant-rate wall
    // clock (plain stores; the host takes the first start and the last end)
    if (P.tstamp && gslot < NTSLOG) {
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long* t = P.tstamp + 2 * ((long long)gslot * P.nwg + lw);
            t[0] = t_begin;
            t[1] = (unsigned long long)wall_clock64();
        }
    }
}

// Both step kernels ask the register allocator for at least three waves per
// SIMD (168 registers): without it the 3-D float64 kernel with per-row
// coefficients came to 179 and two waves, with it 167 and no spills.

// Groups of several systems: the descriptors in device memory, wg_prob maps
// a workgroup to its system (null: all belong to system 0).
template <class Cfg, int DIM, bool VAR, class TI>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void k_step(const DevProb* __restrict__ probs, const int* __restrict__ wg_prob,
                                             int gslot) {
    const unsigned long long t_begin = (unsigned long long)wall_clock64();
    const int wg = xcd_remap(blockIdx.x, gridDim.x);
    step_run<Cfg, DIM, VAR, TI>(probs[wg_prob ? wg_prob[wg] : 0], wg, gslot, t_begin);
}

// A group of one system: its descriptor travels in the kernel arguments, so
// its fields are read from the argument segment at once instead of after a
// pointer load (one memory round trip fewer at the start of every launch).
template <class Cfg, int DIM, bool VAR, class TI>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void k_step1(const DevProb P, int gslot) {
    const unsigned long long t_begin = (unsigned long long)wall_clock64();
    step_run<Cfg, DIM, VAR, TI>(P, xcd_remap(blockIdx.x, gridDim.x), gslot, t_begin);
}

// Workgroups of the grouped step kernel that one compute unit holds at once
// (its registers and LDS decide), for the kernel the launcher would pick.
template <int DIM>
int step_blocks_per_cu_dim(int inner_f32, int var, int tile_id) {
    int nb = 0;
    with_tile<DIM>(tile_id, [&](auto cfg) {
        using Cfg = decltype(cfg);
        hipError_t e;
        if (inner_f32)
            e = var ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_step<Cfg, DIM, true, float>, NT, 0)
                    : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_step<Cfg, DIM, false, float>, NT, 0);
        else
            e = var ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_step<Cfg, DIM, true, double>, NT, 0)
                    : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_step<Cfg, DIM, false, double>, NT, 0);
        if (e != hipSuccess) nb = 0;
    });
    return nb;
}

// ------------------------------------------------------------ launcher
template <int DIM>
void launch_step_dim(int inner_f32, int var, int tile_id, const DevProb* probs, const int* wg_prob, int total_wg,
                     int gslot, hipStream_t s, const DevProb* single) {
    with_tile<DIM>(tile_id, [&](auto cfg) {
        using Cfg = decltype(cfg);
        const dim3 grid(total_wg), block(NT);
        // 2-D tiles up to 16 rows only: in the 3-D kernels and the 32-row
        // 2-D tiles with per-row coefficients the argument-segment
        // descriptor is copied to scratch (392 bytes a lane)
        bool launched = false;
        if constexpr (DIM == 2 && Cfg::TY <= 16) {
            if (single) {
                launched = true;
                const DevProb& P = *single;
                if (inner_f32) {
                    if (var)
                        hipLaunchKernelGGL((k_step1<Cfg, DIM, true, float>), grid, block, 0, s, P, gslot);
                    else
                        hipLaunchKernelGGL((k_step1<Cfg, DIM, false, float>), grid, block, 0, s, P, gslot);
                } else {
                    if (var)
                        hipLaunchKernelGGL((k_step1<Cfg, DIM, true, double>), grid, block, 0, s, P, gslot);
                    else
                        hipLaunchKernelGGL((k_step1<Cfg, DIM, false, double>), grid, block, 0, s, P, gslot);
                }
            }
        }
        if (launched) return;
        if (inner_f32) {
            if (var)
                hipLaunchKernelGGL((k_step<Cfg, DIM, true, float>), grid, block, 0, s, probs, wg_prob, gslot);
            else
                hipLaunchKernelGGL((k_step<Cfg, DIM, false, float>), grid, block, 0, s, probs, wg_prob, gslot);
        } else {
            if (var)
                hipLaunchKernelGGL((k_step<Cfg, DIM, true, double>), grid, block, 0, s, probs, wg_prob, gslot);
            else
                hipLaunchKernelGGL((k_step<Cfg, DIM, false, double>), grid, block, 0, s, probs, wg_prob, gslot);
        }
    });
}

}  // namespace tgdk
