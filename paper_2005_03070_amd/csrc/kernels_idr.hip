// IDR(s) inner cycles of IDR(s)(ncyc)-Proj(k): Sec. 4.1 box, step c), with
// the biorthogonal IDR(s) of van Gijzen and Sonneveld (ACM TOMS 38(1),
// 2011) as the inner solver in place of BiCGStab.
//
// A cycle is a sequence of rounds; a round is s steps and a dimension
// reduction, s + 1 operator applications.  Step k builds a direction
//   u_k = U_(k:) c + omega (r - G_(k:) c),   g_k = A u_k,
// makes g_k orthogonal to p_0 .. p_(k-1) (g_k -= G_(:k) alpha, u_k -= U_(:k) alpha,
// which keeps M = P^T G lower triangular), then
//   r -= beta g_k,  e += beta u_k,  beta = f_k / M_kk,  f = P^T r.
// The reduction takes t = A r, omega from t and r, e += omega r, r -= omega t.
//
// Launch structure: the host enqueues the kernels of whole rounds ahead (the
// step index k is a launch argument).  Each reduction over n is a vector
// kernel writing per-workgroup partial sums (value-major, part[v * nb + b])
// and a one-workgroup epilogue that sums them in a fixed order and takes every
// scalar decision on the device: the small triangular solves with M, beta,
// omega, convergence, breakdown and the iteration limit.  When the cycle
// ends the epilogue sets the state's gate word; every later kernel of the
// cycle (these and the gated stencil launches) then returns at once, so rounds
// enqueued past the end cost only their dispatch.
//
// The alpha of the orthogonalisation come from one product m = P^T g_k and a
// forward substitution with the leading k x k block of M (the same numbers as
// orthogonalising against p_0 .. p_(k-1) one after another); M_(k:,k) is then
// computed afresh from the orthogonalised g_k.
#include <algorithm>

#include "device_common.h"
#include "launch.h"

namespace tgdk {

constexpr int IDR_BLOCKS = 1024;  // cap on the workgroups of the vector kernels
static_assert(IDR_BLOCKS % 64 == 0, "the epilogue gives every lane IDR_BLOCKS / 64 partials");

int idr_blocks(long long n) {
    long long b = (n + 2 * NT - 1) / (2 * NT);
    return (int)std::max(1LL, std::min(b, (long long)IDR_BLOCKS));
}

// Per-workgroup sums of P_j . y (j in [0, s)) and, with SELF, y . y as value
// s, written to part.  y(i, first) returns entry i of y; first is true on
// the first pass only (where y may be formed and stored).  A pass takes CH
// columns of P (CH = s up to 8: the launcher picks 1, 2, 4 or 8); columns
// beyond CH take further passes that read y back.  Every column load of a
// pass is issued unconditionally (a column past s re-reads the pass's first
// column, a cache hit, and is masked), so a row's loads are all in flight
// together: a guarded load compiles to a branch that waits at its join.
template <class TI, bool SELF, int CH, class Y>
__device__ __forceinline__ void dots_with_P(const IdrArgs& a, Y&& y) {
    __shared__ double sh[NWAVE * (CH + 1)];
    const TI* __restrict__ P = vp<TI>(a.P);
    const long long n = a.n;
    const long long stride = (long long)gridDim.x * NT;
    const long long i0 = (long long)blockIdx.x * NT + threadIdx.x;
    for (int c0 = 0; c0 < a.s; c0 += CH) {
        const bool first = c0 == 0;
        double acc[CH + 1];
#pragma unroll
        for (int j = 0; j <= CH; ++j) acc[j] = 0.0;
        const int nc = min(CH, a.s - c0);
        const TI* Pc[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) Pc[j] = P + (long long)(c0 + (j < nc ? j : 0)) * n;
#pragma unroll 2
        for (long long i = i0; i < n; i += stride) {
            const double yv = y(i, first);
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                // the mask on the factor keeps the multiply-add fused
                const double pv = (double)Pc[j][i];
                acc[j] += (j < nc ? pv : 0.0) * yv;
            }
            if (SELF && first) acc[CH] += yv * yv;
        }
        double tot;
        block_sum<CH + 1, true>(acc, sh, tot);
        if (threadIdx.x < nc) a.part[(long long)(c0 + threadIdx.x) * a.nb + blockIdx.x] = tot;
        if (SELF && first && threadIdx.x == CH) a.part[(long long)a.s * a.nb + blockIdx.x] = tot;
    }
}

// Cycle start: f = P^T r, r . r (values 0..s-1, s).
template <class TI, int CH>
__global__ __launch_bounds__(NT) void k_idr_start(IdrArgs a) {
    if (a.ss->solve_state != SV_RUNNING) return;
    const TI* __restrict__ r = vp<TI>(a.r);
    dots_with_P<TI, true, CH>(a, [&](long long i, bool) { return (double)r[i]; });
}

// Direction of step k: u_k = U_(k:) c + omega (r - G_(k:) c); in the first
// round of a cycle G = U = 0 and omega = 1, so u_k = r.
template <class TI>
__global__ __launch_bounds__(NT) void k_idr_dir(IdrArgs a, int k) {
    __shared__ double cs[IDR_SMAX];
    const IdrState* st = a.st;
    if (st->gate) return;
    const TI* __restrict__ r = vp<TI>(a.r);
    const TI* __restrict__ G = vp<TI>(a.G);
    TI* U = vp<TI>(a.U);
    const long long n = a.n;
    TI* uk = U + (long long)k * n;
    const long long stride = (long long)gridDim.x * NT;
    const long long i0 = (long long)blockIdx.x * NT + threadIdx.x;
    if (st->round0) {
        for (long long i = i0; i < n; i += stride) uk[i] = r[i];
        return;
    }
    const int m = a.s - k;
    if (threadIdx.x < m) cs[threadIdx.x] = st->c[threadIdx.x];
    __syncthreads();
    const double om = st->om;
#pragma unroll 2
    for (long long i = i0; i < n; i += stride) {
        double gc = 0.0, uc = 0.0;
        for (int j = 0; j < m; ++j) {
            gc += (double)G[(long long)(k + j) * n + i] * cs[j];
            uc += (double)U[(long long)(k + j) * n + i] * cs[j];
        }
        const TI v = (TI)((double)r[i] - gc);
        uk[i] = (TI)(uc + om * (double)v);
    }
}

// Steps k-1 and k fused (k >= 1): the update of step k-1,
// r -= beta g_(k-1), e += beta u_(k-1) (e = beta u_(k-1) on the cycle's first
// update), with r . r into value slot s; then the direction of step k from the
// updated r.  The convergence test of that update happens in step k's alpha
// epilogue; beta's effect on f and the coefficients c of step k were formed in
// step k-1's M epilogue (they do not depend on r . r).
template <class TI>
__global__ __launch_bounds__(NT) void k_idr_dirupd(IdrArgs a, int k) {
    __shared__ double cs[IDR_SMAX];
    __shared__ double sh[NWAVE];
    const IdrState* st = a.st;
    if (st->gate) return;
    TI* r = vp<TI>(a.r);
    TI* e = vp<TI>(a.e);
    const TI* __restrict__ G = vp<TI>(a.G);
    TI* U = vp<TI>(a.U);
    const long long n = a.n;
    const TI* gp = G + (long long)(k - 1) * n;
    const TI* up = U + (long long)(k - 1) * n;
    TI* uk = U + (long long)k * n;
    const int m = a.s - k;
    const bool round0 = st->round0;
    if (!round0 && threadIdx.x < m) cs[threadIdx.x] = st->c[threadIdx.x];
    __syncthreads();
    const double beta = st->beta, om = st->om;
    const bool efirst = st->efirst;
    const long long stride = (long long)gridDim.x * NT;
    double acc = 0.0;
#pragma unroll 2
    for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += stride) {
        const TI rv = (TI)((double)r[i] - beta * (double)gp[i]);
        r[i] = rv;
        e[i] = efirst ? (TI)(beta * (double)up[i]) : (TI)((double)e[i] + beta * (double)up[i]);
        acc += (double)rv * (double)rv;
        if (round0) {
            uk[i] = rv;
        } else {
            double gc = 0.0, uc = 0.0;
            for (int j = 0; j < m; ++j) {
                gc += (double)G[(long long)(k + j) * n + i] * cs[j];
                uc += (double)U[(long long)(k + j) * n + i] * cs[j];
            }
            const TI v = (TI)((double)rv - gc);
            uk[i] = (TI)(uc + om * (double)v);
        }
    }
    const double tot = block_sum_one<true>(acc, sh);
    if (threadIdx.x == 0) a.part[(long long)a.s * a.nb + blockIdx.x] = tot;
}

// m = P^T g_k before the orthogonalisation (k > 0).
template <class TI, int CH>
__global__ __launch_bounds__(NT) void k_idr_gdot(IdrArgs a, int k) {
    if (a.st->gate) return;
    const TI* __restrict__ g = vp<TI>(a.G) + (long long)k * a.n;
    dots_with_P<TI, false, CH>(a, [&](long long i, bool) { return (double)g[i]; });
}

// g_k -= G_(:k) alpha, u_k -= U_(:k) alpha, then P^T g_k (values 0..s-1).
// The columns of G and U are taken CH at a time with unconditional loads (a
// column past k re-reads column 0 and is masked: 0 * G adds an exact zero).
template <class TI, int CH>
__global__ __launch_bounds__(NT) void k_idr_orth(IdrArgs a, int k) {
    __shared__ double al[IDR_SMAX];
    const IdrState* st = a.st;
    if (st->gate) return;
    if (threadIdx.x < k) al[threadIdx.x] = st->alpha[threadIdx.x];
    __syncthreads();
    TI* G = vp<TI>(a.G);
    TI* U = vp<TI>(a.U);
    const long long n = a.n;
    TI* g = G + (long long)k * n;
    TI* u = U + (long long)k * n;
    dots_with_P<TI, false, CH>(a, [&](long long i, bool first) {
        if (!first || k == 0) return (double)g[i];
        double gs = (double)g[i], us = (double)u[i];
        for (int j0 = 0; j0 < k; j0 += CH) {
#pragma unroll
            for (int jj = 0; jj < CH; ++jj) {
                const int j = j0 + jj;
                const int jc = j < k ? j : 0;
                const double gv = (double)G[(long long)jc * n + i], uv = (double)U[(long long)jc * n + i];
                const double aj = j < k ? al[jc] : 0.0;
                gs -= aj * gv;
                us -= aj * uv;
            }
        }
        const TI gt = (TI)gs;
        g[i] = gt;
        u[i] = (TI)us;
        return (double)gt;
    });
}

// r -= beta g_k, e += beta u_k (e = beta u_k on the cycle's first update);
// r . r (value 0).
template <class TI>
__global__ __launch_bounds__(NT) void k_idr_upd(IdrArgs a, int k) {
    __shared__ double sh[NWAVE];
    const IdrState* st = a.st;
    if (st->gate) return;
    TI* r = vp<TI>(a.r);
    TI* e = vp<TI>(a.e);
    const long long n = a.n;
    const TI* __restrict__ g = vp<TI>(a.G) + (long long)k * n;
    const TI* __restrict__ u = vp<TI>(a.U) + (long long)k * n;
    const double beta = st->beta;
    const bool efirst = st->efirst;
    const long long stride = (long long)gridDim.x * NT;
    double acc = 0.0;
#pragma unroll 4
    for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += stride) {
        const TI rv = (TI)((double)r[i] - beta * (double)g[i]);
        r[i] = rv;
        e[i] = efirst ? (TI)(beta * (double)u[i]) : (TI)((double)e[i] + beta * (double)u[i]);
        acc += (double)rv * (double)rv;
    }
    const double tot = block_sum_one<true>(acc, sh);
    if (threadIdx.x == 0) a.part[blockIdx.x] = tot;
}

// Dimension reduction, first half: t . t, t . r, r . r (values 0, 1, 2).
template <class TI>
__global__ __launch_bounds__(NT) void k_idr_tdot(IdrArgs a) {
    __shared__ double sh[NWAVE * 3];
    if (a.st->gate) return;
    const TI* __restrict__ r = vp<TI>(a.r);
    const TI* __restrict__ t = vp<TI>(a.t);
    const long long stride = (long long)gridDim.x * NT;
    double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll 4
    for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < a.n; i += stride) {
        const double tv = (double)t[i], rv = (double)r[i];
        acc[0] += tv * tv;
        acc[1] += tv * rv;
        acc[2] += rv * rv;
    }
    double tot;
    block_sum<3, true>(acc, sh, tot);
    if (threadIdx.x < 3) a.part[(long long)threadIdx.x * a.nb + blockIdx.x] = tot;
}

// Dimension reduction, second half: e += omega r, r -= omega t; then
// f = P^T r, r . r (values 0..s-1, s) for the next round.
template <class TI, int CH>
__global__ __launch_bounds__(NT) void k_idr_red(IdrArgs a) {
    const IdrState* st = a.st;
    if (st->gate) return;
    TI* r = vp<TI>(a.r);
    TI* e = vp<TI>(a.e);
    const TI* __restrict__ t = vp<TI>(a.t);
    const double om = st->om;
    const bool efirst = st->efirst;
    dots_with_P<TI, true, CH>(a, [&](long long i, bool first) {
        if (!first) return (double)r[i];
        const double rv = (double)r[i];
        e[i] = efirst ? (TI)(om * rv) : (TI)((double)e[i] + om * rv);
        const TI rn = (TI)(rv - om * (double)t[i]);
        r[i] = rn;
        return (double)rn;
    });
}

// x += e at the end of a cycle (float64; nothing if e was never written).
template <class TI>
__global__ __launch_bounds__(NT) void k_idr_fold(IdrArgs a) {
    if (a.ss->solve_state != SV_RUNNING || a.st->efirst) return;
    const TI* __restrict__ e = vp<TI>(a.e);
    const long long stride = (long long)gridDim.x * NT;
    for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < a.n; i += stride) a.x[i] += (double)e[i];
}

// ------------------------------------------- stencil fused with products
// y = A x on 2-D tiles (x staged with its halo in LDS, as k_apply), the tiles
// grid-strided over the nb workgroups of the vector kernels, with the step's
// products formed from the outputs in registers: MODE 0, P^T y (values
// 0..s-1, CH columns of P, s <= CH, unconditional loads masked on the
// factor); MODE 1, y.y, y.r, r.r (values 0, 1, 2; r read at the tile's own
// points).  Per-workgroup partials in the vector kernels' layout, so the
// epilogue reads them as it reads theirs.
template <class Cfg, class TI, int MODE, int CH>
__global__ __launch_bounds__(NT) void k_idr_apply_dots(DevOp op, IdrArgs a, const TI* __restrict__ x,
                                                       TI* __restrict__ y, int tx, int ty, int ntiles) {
    constexpr int NV = MODE == 0 ? CH : 3;
    __shared__ TI L[Cfg::BOX];
    __shared__ double sh[NWAVE * NV];
    if (a.st->gate) return;
    const TI* __restrict__ P = vp<TI>(a.P);
    const TI* __restrict__ r = vp<TI>(a.r);
    const long long n = a.n;
    const TI* Pc[MODE == 0 ? CH : 1];
    if (MODE == 0) {
#pragma unroll
        for (int j = 0; j < CH; ++j) Pc[j] = P + (long long)(j < a.s ? j : 0) * n;
    }
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    for (int tile = xcd_remap(blockIdx.x, gridDim.x); tile < ntiles; tile += gridDim.x) {
        const TilePos tp = tile_pos<Cfg>(tile, tx, ty);
        long long gq[Cfg::PPT];
        int cq[Cfg::PPT];
        bool okq[Cfg::PPT];
#pragma unroll
        for (int q = 0; q < Cfg::PPT; ++q) {
            int gx, gy, gz;
            point_coords<Cfg>(q, tp, gx, gy, gz, cq[q]);
            okq[q] = inside(op, gx, gy, gz);
            gq[q] = okq[q] ? gidx(op, gx, gy, gz) : 0;
            L[cq[q]] = okq[q] ? x[gq[q]] : TI(0);
        }
        fill_halo<Cfg, 2, TI>(L, tp, op, [&](long long g) { return x[g]; });
        __syncthreads();
#pragma unroll
        for (int q = 0; q < Cfg::PPT; ++q) {
            if (!okq[q]) continue;
            const long long g = gq[q];
            const TI yv = stencil_row<Cfg, 2, TI>(op, L, cq[q], g);
            st_stream<2>(&y[g], yv);
            const double yd = (double)yv;
            if (MODE == 0) {
#pragma unroll
                for (int j = 0; j < CH; ++j) {
                    const double pv = (double)Pc[j][g];
                    acc[j] += (j < a.s ? pv : 0.0) * yd;
                }
            } else {
                const double rv = (double)r[g];
                acc[0] += yd * yd;
                acc[1] += yd * rv;
                acc[2] += rv * rv;
            }
        }
        __syncthreads();  // L is rewritten by the next tile
    }
    double tot;
    block_sum<NV, true>(acc, sh, tot);
    const int nv = MODE == 0 ? a.s : 3;
    if (threadIdx.x < nv) a.part[(long long)threadIdx.x * a.nb + blockIdx.x] = tot;
}

// ------------------------------------------------------------ epilogues
// One workgroup: the waves sum the partials of each value in a fixed order,
// the cycle's small arrays (M, f, c, alpha) are staged in LDS, thread 0 takes
// the decisions there (no dependent global-memory round trips), and the
// workgroup writes the arrays back.
enum : int { E_START = 0, E_ALPHA = 1, E_M = 2, E_UPD = 3, E_OM = 4, E_RED = 5 };

struct EpiArrays {
    double M[IDR_SMAX * IDR_SMAX];  // row-major s x s
    double f[IDR_SMAX], c[IDR_SMAX], alpha[IDR_SMAX];
};

// c = solution of the lower-triangular system M_(k:, k:) c = f_(k:).
__device__ void idr_coeffs(EpiArrays& L, int s, int k) {
    for (int i = k; i < s; ++i) {
        double v = L.f[i];
        for (int j = k; j < i; ++j) v -= L.M[i * s + j] * L.c[j - k];
        L.c[i - k] = v / L.M[i * s + i];
    }
}

__device__ void idr_end(const IdrArgs& a, int status) {
    IdrState* st = a.st;
    SolveState* ss = a.ss;
    const int mvps = st->mvps;
    st->status = status;
    st->gate = 1;
    ss->iter = mvps;
    ss->inner_state = status;
    ss->mvp_inner += mvps;
    ss->iters_total += mvps;
    if (a.mirror) {
        a.mirror->inner_state = status;
        a.mirror->iter = mvps;
        a.mirror->rr = st->rr;
        __threadfence_system();
    }
}

// ||r|| and the coefficient of an update of r in the first cycle (the
// report's first scalars: norm, coefficient, 1 at a dimension reduction).
__device__ void idr_hist(const IdrArgs& a, double rr, double coef, int red) {
    SolveState* ss = a.ss;
    if (ss->icyc == 1 && ss->nhist < NHIST) {
        const int h = ss->nhist++;
        ss->hist[3 * h] = sqrt(rr);
        ss->hist[3 * h + 1] = coef;
        ss->hist[3 * h + 2] = (double)red;
    }
}

__device__ void idr_progress(const IdrArgs& a, double rr, int mvps) {
    if (a.mirror) {
        a.mirror->rr = rr;
        a.mirror->iter = mvps;
        __threadfence_system();
    }
}

// The decisions of epilogue `which` (thread 0, on the staged arrays).
__device__ void idr_decide(const IdrArgs& a, int which, int k, const double* v, EpiArrays& L) {
    IdrState* st = a.st;
    SolveState* ss = a.ss;
    const int s = a.s;
    switch (which) {
        case E_START: {
            for (int i = 0; i < s * s; ++i) L.M[i] = 0.0;
            for (int i = 0; i < s; ++i) {
                L.M[i * s + i] = 1.0;
                L.f[i] = v[i];
                L.c[i] = v[i];
            }
            const double rr = v[s], target2 = ss->target2;
            st->rr = rr;
            st->om = 1.0;
            st->round0 = 1;
            st->efirst = 1;
            st->mvps = 0;
            st->target2 = target2;
            st->maxit = ss->maxit;
            st->status = IN_RUNNING;
            st->gate = 0;
            if (a.mirror) {
                a.mirror->rr0 = rr;
                a.mirror->target2 = target2;
                a.mirror->inner_state = IN_RUNNING;
            }
            idr_progress(a, rr, 0);
            if (rr <= target2) idr_end(a, IN_CONVERGED);
            break;
        }
        case E_ALPHA: {
            // the update of step k-1 (fused into step k's direction): its tests
            const double rr = v[s], beta = st->beta;
            const int mvps = st->mvps;
            st->rr = rr;
            st->efirst = 0;
            idr_hist(a, rr, beta, 0);
            if (rr <= st->target2) {
                idr_end(a, IN_CONVERGED);
                break;
            }
            if (!isfinite(rr)) {
                idr_end(a, IN_BREAK_NOUPD);
                break;
            }
            if (mvps >= st->maxit) {
                idr_end(a, IN_MAXIT);
                break;
            }
            idr_progress(a, rr, mvps);
            // forward substitution with the leading k x k block of M
            for (int i = 0; i < k; ++i) {
                double x = v[i];
                for (int j = 0; j < i; ++j) x -= L.M[i * s + j] * L.alpha[j];
                L.alpha[i] = x / L.M[i * s + i];
            }
            break;
        }
        case E_M: {
            st->mvps += 1;
            for (int i = k; i < s; ++i) L.M[i * s + k] = v[i];
            const double mkk = L.M[k * s + k];
            if (mkk == 0.0 || !isfinite(mkk)) {
                idr_end(a, IN_BREAK_NOUPD);
                break;
            }
            st->beta = L.f[k] / mkk;
            // f and the next step's coefficients (the update itself and its
            // tests follow in the next step's kernels)
            if (k + 1 < s) {
                for (int i = k + 1; i < s; ++i) L.f[i] -= st->beta * L.M[i * s + k];
                idr_coeffs(L, s, k + 1);
            }
            break;
        }
        case E_UPD: {
            const double rr = v[0], beta = st->beta;
            const int mvps = st->mvps;
            st->rr = rr;
            st->efirst = 0;
            idr_hist(a, rr, beta, 0);
            if (rr <= st->target2) {
                idr_end(a, IN_CONVERGED);
                break;
            }
            if (!isfinite(rr)) {
                idr_end(a, IN_BREAK_NOUPD);
                break;
            }
            for (int i = k + 1; i < s; ++i) L.f[i] -= beta * L.M[i * s + k];
            if (mvps >= st->maxit) {
                idr_end(a, IN_MAXIT);
                break;
            }
            if (k + 1 < s) idr_coeffs(L, s, k + 1);
            idr_progress(a, rr, mvps);
            break;
        }
        case E_OM: {
            st->mvps += 1;
            const double tt = v[0], ts = v[1], rr = v[2];
            if (tt == 0.0 || ts == 0.0 || !isfinite(ts / tt)) {
                idr_end(a, IN_BREAK_NOUPD);
                break;
            }
            double om = ts / tt;
            const double rho = fabs(ts) / (sqrt(tt) * sqrt(rr));
            const double kappa = st->kappa;
            if (rho < kappa) om = om * kappa / rho;
            st->om = om;
            break;
        }
        case E_RED: {
            const double rr = v[s];
            const int mvps = st->mvps;
            st->rr = rr;
            st->efirst = 0;
            idr_hist(a, rr, st->om, 1);
            if (rr <= st->target2) {
                idr_end(a, IN_CONVERGED);
                break;
            }
            if (!isfinite(rr)) {
                idr_end(a, IN_BREAK_NOUPD);
                break;
            }
            for (int i = 0; i < s; ++i) L.f[i] = v[i];
            st->round0 = 0;
            if (mvps >= st->maxit) {
                idr_end(a, IN_MAXIT);
                break;
            }
            idr_coeffs(L, s, 0);
            idr_progress(a, rr, mvps);
            break;
        }
    }
}

__global__ __launch_bounds__(NT) void k_idr_epi(IdrArgs a, int which, int k, int nv) {
    __shared__ double v[IDR_SMAX + 4];
    __shared__ EpiArrays L;
    IdrState* st = a.st;
    if (which == E_START ? a.ss->solve_state != SV_RUNNING : st->gate != 0) return;
    const int s = a.s;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // each lane's IDR_BLOCKS / 64 partials of a value are loaded together
    // (clamped addresses, masked values), then added in a fixed order
    constexpr int PER_LANE = IDR_BLOCKS / 64;
    for (int q = w; q < nv; q += NWAVE) {
        const double* pq = a.part + (long long)q * a.nb;
        double x[PER_LANE];
#pragma unroll
        for (int i = 0; i < PER_LANE; ++i) {
            const int b = lane + 64 * i;
            x[i] = pq[b < a.nb ? b : 0];
        }
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < PER_LANE; ++i) acc += (lane + 64 * i < a.nb) ? x[i] : 0.0;
        acc = wave_sum_dpp(acc);
        if (lane == 0) v[q] = acc;
    }
    // stage what the decisions read
    const bool readM = which == E_ALPHA || which == E_M || which == E_UPD || which == E_RED;
    if (readM)
        for (int i = threadIdx.x; i < s * s; i += NT) L.M[i] = st->M[i];
    for (int i = threadIdx.x; i < s; i += NT) {
        L.f[i] = st->f[i];
        L.c[i] = st->c[i];
        L.alpha[i] = st->alpha[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) idr_decide(a, which, k, v, L);
    __syncthreads();
    // write back what the decisions may have changed
    if (which == E_START)
        for (int i = threadIdx.x; i < s * s; i += NT) st->M[i] = L.M[i];
    else if (which == E_M)
        for (int i = k + threadIdx.x; i < s; i += NT) st->M[i * s + k] = L.M[i * s + k];
    for (int i = threadIdx.x; i < s; i += NT) {
        st->f[i] = L.f[i];
        st->c[i] = L.c[i];
        st->alpha[i] = L.alpha[i];
    }
}

// ------------------------------------------------------------- launchers
template <class TI, int CH>
static void idr_launch_ch(int what, const IdrArgs& a, int k, hipStream_t s) {
    const dim3 grid(a.nb), block(NT);
    switch (what) {
        case IDR_START:
            hipLaunchKernelGGL((k_idr_start<TI, CH>), grid, block, 0, s, a);
            hipLaunchKernelGGL(k_idr_epi, dim3(1), block, 0, s, a, (int)E_START, 0, a.s + 1);
            break;
        case IDR_DIR:
            hipLaunchKernelGGL(k_idr_dir<TI>, grid, block, 0, s, a, k);
            break;
        case IDR_ALPHA:
            hipLaunchKernelGGL((k_idr_gdot<TI, CH>), grid, block, 0, s, a, k);
            hipLaunchKernelGGL(k_idr_epi, dim3(1), block, 0, s, a, (int)E_ALPHA, k, a.s + 1);
            break;
        case IDR_DIRUPD:
            hipLaunchKernelGGL(k_idr_dirupd<TI>, grid, block, 0, s, a, k);
            break;
        case IDR_ORTH:
            hipLaunchKernelGGL((k_idr_orth<TI, CH>), grid, block, 0, s, a, k);
            hipLaunchKernelGGL(k_idr_epi, dim3(1), block, 0, s, a, (int)E_M, k, a.s);
            break;
        case IDR_UPD:
            hipLaunchKernelGGL(k_idr_upd<TI>, grid, block, 0, s, a, k);
            hipLaunchKernelGGL(k_idr_epi, dim3(1), block, 0, s, a, (int)E_UPD, k, 1);
            break;
        case IDR_OMEGA:
            hipLaunchKernelGGL(k_idr_tdot<TI>, grid, block, 0, s, a);
            hipLaunchKernelGGL(k_idr_epi, dim3(1), block, 0, s, a, (int)E_OM, 0, 3);
            break;
        case IDR_RED:
            hipLaunchKernelGGL((k_idr_red<TI, CH>), grid, block, 0, s, a);
            hipLaunchKernelGGL(k_idr_epi, dim3(1), block, 0, s, a, (int)E_RED, 0, a.s + 1);
            break;
        case IDR_FOLD:
            hipLaunchKernelGGL(k_idr_fold<TI>, grid, block, 0, s, a);
            break;
    }
}

// the column chunk of the products with P: s columns up to 8 in one pass
template <class TI>
static void idr_launch_t(int what, const IdrArgs& a, int k, hipStream_t s) {
    if (a.s <= 1)
        idr_launch_ch<TI, 1>(what, a, k, s);
    else if (a.s <= 2)
        idr_launch_ch<TI, 2>(what, a, k, s);
    else if (a.s <= 4)
        idr_launch_ch<TI, 4>(what, a, k, s);
    else
        idr_launch_ch<TI, 8>(what, a, k, s);
}

template <class TI, int CH>
static void idr_fused_t(int what, const IdrArgs& a, const DevOp& op, int tile_id, const void* x, void* y, int k,
                        hipStream_t s) {
    with_tile<2>(tile_id, [&](auto cfg) {
        using Cfg = decltype(cfg);
        const int tx = (op.nx + Cfg::TX - 1) / Cfg::TX, ty = (op.ny + Cfg::TY - 1) / Cfg::TY;
        const dim3 grid(a.nb), block(NT);
        if (what == IDR_ALPHA)
            hipLaunchKernelGGL((k_idr_apply_dots<Cfg, TI, 0, CH>), grid, block, 0, s, op, a, (const TI*)x, (TI*)y,
                               tx, ty, tx * ty);
        else
            hipLaunchKernelGGL((k_idr_apply_dots<Cfg, TI, 1, 1>), grid, block, 0, s, op, a, (const TI*)x, (TI*)y,
                               tx, ty, tx * ty);
    });
    const dim3 block(NT);
    if (what == IDR_OMEGA)
        hipLaunchKernelGGL(k_idr_epi, dim3(1), block, 0, s, a, (int)E_OM, 0, 3);
    else if (k > 0)
        hipLaunchKernelGGL(k_idr_epi, dim3(1), block, 0, s, a, (int)E_ALPHA, k, a.s + 1);
    else
        hipLaunchKernelGGL(k_idr_epi, dim3(1), block, 0, s, a, (int)E_M, 0, a.s);
}

template <class TI>
static void idr_fused_s(int what, const IdrArgs& a, const DevOp& op, int tile_id, const void* x, void* y, int k,
                        hipStream_t s) {
    if (a.s <= 1)
        idr_fused_t<TI, 1>(what, a, op, tile_id, x, y, k, s);
    else if (a.s <= 2)
        idr_fused_t<TI, 2>(what, a, op, tile_id, x, y, k, s);
    else if (a.s <= 4)
        idr_fused_t<TI, 4>(what, a, op, tile_id, x, y, k, s);
    else
        idr_fused_t<TI, 8>(what, a, op, tile_id, x, y, k, s);
}

bool launch_idr_fused(int what, int inner_f32, const IdrArgs& a, const DevOp& op, int tile_id, const void* x,
                      void* y, int k, hipStream_t s) {
    if (op.dim != 2 || a.s > 8 || (what != IDR_ALPHA && what != IDR_OMEGA)) return false;
    if (inner_f32)
        idr_fused_s<float>(what, a, op, tile_id, x, y, k, s);
    else
        idr_fused_s<double>(what, a, op, tile_id, x, y, k, s);
    return true;
}

void launch_idr(int what, int inner_f32, const IdrArgs& a, int k, hipStream_t s) {
    if (inner_f32)
        idr_launch_t<float>(what, a, k, s);
    else
        idr_launch_t<double>(what, a, k, s);
}

}  // namespace tgdk
