// Fine-solve drivers: BiCGStab(ncyc)-Proj(k) over a group of problems
// (right-hand sides sharing an operator, or independent grid instances) and
// GMRES(m)-Proj(k) for one right-hand side.
//
// BiCGStab: the host only enqueues step launches; every scalar decision
// (alpha, omega, cycle tolerance, convergence, breakdown, projection) is
// taken on the device by the step kernel.  The host watches a host-mapped
// status mirror one batch behind, so the GPU queue never drains while it
// decides how many more steps to enqueue.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "dense.h"
#include "host.h"

namespace tgdk {

struct ProbSpec {
    tgdk_op op;
    tgdk_defl defl;
    const double* b;
    double* x;
};

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Workgroups of the step kernel per problem: on 2-D grids one per tile up to
// this cap (beyond it each walks several tiles; the cap bounds the partial
// sums every workgroup reads), on 3-D grids about as many z-marching chunks
// as the device holds resident at once, at most STEP_CHUNKS: the float64
// kernel (145 registers, 3 workgroups per compute unit) gets 768 chunks, so
// no fourth of them runs as a tail after the others (255^3 FP64 solve
// 272.8 -> 260.2 ms); float32 (5 per unit) keeps 1024.
constexpr int STEP_WG_CAP = 1024;
constexpr int STEP_CHUNKS = 1024;

static int status_of(const SolveState& st) {
    switch (st.solve_state) {
        case SV_CONVERGED: return TGDK_OK;
        case SV_BREAKDOWN: return TGDK_BREAKDOWN;
        case SV_NOT_CONVERGED: return TGDK_NOT_CONVERGED;
        case SV_NONFINITE: return TGDK_E_NONFINITE;
        default: return TGDK_NOT_CONVERGED;
    }
}

static int worst(int a, int b) {
    if (a < 0 || b < 0) return std::min(a, b);
    return std::max(a, b);
}

static int ensure_mirror(tgdk_ctx ctx, int n) {
    if (ctx->mirror_cap >= n) return TGDK_OK;
    if (ctx->mirror) (void)hipHostFree(ctx->mirror);
    ctx->mirror = nullptr;
    ctx->mirror_cap = 0;
    TGDK_HIP(hipHostMalloc((void**)&ctx->mirror, sizeof(Mirror) * n, hipHostMallocMapped));
    ctx->mirror_cap = n;
    return TGDK_OK;
}

static int ensure_events(tgdk_ctx ctx, int n) {
    while ((int)ctx->events.size() < n) {
        hipEvent_t e;
        TGDK_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        ctx->events.push_back(e);
    }
    return TGDK_OK;
}

struct Group {
    tgdk_ctx ctx = nullptr;
    int dim = 2, inner_f32 = 0, vtype = 0, tile_id = 0;
    int var = 0;  // some operator of the group has per-row coefficient arrays
    int nprob = 0, total_tiles = 0;
    int total_wg = 0;      // step kernel workgroups
    int gslot = 0;         // step launches enqueued so far
    DevProb* d_probs = nullptr;
    SolveState* d_states = nullptr;
    int* d_wgprob = nullptr;
    unsigned char* d_actlog = nullptr;  // action log of problem 0 (measurement only)
    unsigned long long* d_ts = nullptr;  // per-launch first start / last end (measurement only)
    std::vector<DevProb> probs;
    std::vector<SolveState> states;
    std::vector<int> wgprob;
    Mirror* mirror = nullptr;
};

static void launch(const Group& g, int which, int flag = 0) {
    launch_solve_kernel(which, g.dim, g.inner_f32, g.vtype, g.tile_id, g.d_probs, g.nprob, g.total_tiles, flag,
                        g.ctx->stream);
}

// One step launch (with measurement on, the kernel stamps its start and end,
// or a timing event follows it on the stream).
static int launch_step_timed(Group& g) {
    const int slot = g.gslot++;
    tgdk_ctx ctx = g.ctx;
    const bool ev = ctx->time_which == 2 && slot < NTSLOG;
    if (ev && slot == 0) TGDK_HIP(hipEventRecord(ctx->tevents[0], ctx->stream));
    // a group of one system passes its descriptor in the kernel arguments
    // and needs no workgroup-to-system map
    const bool one = g.nprob == 1;
    launch_step(g.dim, g.inner_f32, g.var, g.tile_id, g.d_probs, one ? nullptr : g.d_wgprob, g.total_wg, slot,
                ctx->stream, one ? &g.probs[0] : nullptr);
    if (ev) TGDK_HIP(hipEventRecord(ctx->tevents[slot + 1], ctx->stream));
    return TGDK_OK;
}

// Adds the duration of every measured step launch (last workgroup end minus
// first workgroup start, device wall clock; the group's first problem's
// workgroups) to the context's totals, per action of that problem (from the
// device's action log).
static int collect_timing(Group& g) {
    tgdk_ctx ctx = g.ctx;
    if (!g.d_actlog) return TGDK_OK;
    const int nl = std::min(g.gslot, NTSLOG);
    std::vector<unsigned char> act((size_t)nl, 0);
    TGDK_HIP(hipMemcpy(act.data(), g.d_actlog, (size_t)nl, hipMemcpyDeviceToHost));
    if (ctx->time_which == 2) {
        for (int l = 0; l < nl; ++l) {
            float ms = 0.0f;
            TGDK_HIP(hipEventElapsedTime(&ms, ctx->tevents[l], ctx->tevents[l + 1]));
            const int a = act[(size_t)l];
            ctx->act_ms[a] += (double)ms;
            ctx->act_count[a] += 1;
        }
        return TGDK_OK;
    }
    if (!g.d_ts) return TGDK_OK;
    const size_t nwg = (size_t)g.probs[0].nwg;
    std::vector<unsigned long long> ts(2 * (size_t)nl * nwg, 0);
    TGDK_HIP(hipMemcpy(ts.data(), g.d_ts, sizeof(unsigned long long) * ts.size(), hipMemcpyDeviceToHost));
    int khz = 0;
    TGDK_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device));
    if (khz <= 0) return fail(TGDK_E_HIP, "device wall clock rate unknown");
    for (int l = 0; l < nl; ++l) {
        unsigned long long t0 = ~0ull, t1 = 0;
        for (size_t w = 0; w < nwg; ++w) {
            t0 = std::min(t0, ts[2 * ((size_t)l * nwg + w)]);
            t1 = std::max(t1, ts[2 * ((size_t)l * nwg + w) + 1]);
        }
        if (t1 <= t0) continue;
        const int a = act[(size_t)l];
        ctx->act_ms[a] += (double)(t1 - t0) / (double)khz;
        ctx->act_count[a] += 1;
    }
    return TGDK_OK;
}

// Host-mapped mirror values are written by the device; read them volatile.
static Mirror read_mirror(const Group& g, int j) {
    volatile Mirror* m = g.mirror + j;
    Mirror r;
    r.solve_state = m->solve_state;
    r.inner_state = m->inner_state;
    r.icyc = m->icyc;
    r.iter = m->iter;
    r.mode = m->mode;
    r.slot = m->slot;
    r.rr = m->rr;
    r.rr0 = m->rr0;
    r.target2 = m->target2;
    return r;
}

static int wait_event(hipEvent_t e) {
    // spin on the event (low latency), yielding to the runtime
    for (;;) {
        hipError_t q = hipEventQuery(e);
        if (q == hipSuccess) return TGDK_OK;
        if (q != hipErrorNotReady) return fail(TGDK_E_HIP, std::string("kernel failed: ") + hipGetErrorString(q));
    }
}

// A caller-provided device workspace (base, capacity in bytes) used in place
// of the context's grow-only one; nothing is allocated when it is given.
struct ExtWs {
    void* base;
    size_t cap;
};

// Fills the device-side group description and workspaces (allocated in the
// context's grow-only buffer, or laid out in ext).
static int build_group(tgdk_ctx ctx, const std::vector<ProbSpec>& ps, const tgdk_solve_params* prm, Group& g,
                       const ExtWs* ext = nullptr) {
    g.ctx = ctx;
    g.nprob = (int)ps.size();
    g.dim = ps[0].op->dim;
    g.inner_f32 = prm->precision == TGDK_FP32_IR ? 1 : 0;
    g.tile_id = ps[0].op->tile_id[g.inner_f32];
    int vtype = -1;
    for (const auto& p : ps)
        if (p.defl) {
            const int t = p.defl->store == TGDK_F32 ? 1 : 0;
            if (vtype >= 0 && vtype != t) return fail(TGDK_E_INVALID, "mixed deflation storage types in one group");
            vtype = t;
        }
    g.vtype = vtype < 0 ? 0 : vtype;
    int ty, tz;
    tile_shape(g.dim, g.tile_id, &ty, &tz);
    const size_t ies = g.inner_f32 ? 4 : 8;
    int var_any = 0;
    for (const auto& p : ps) var_any |= p.op->kind != TGDK_CONST_CD;
    int chunk_target = STEP_CHUNKS;
    if (g.dim == 3) {
        const int nb = step_blocks_per_cu(g.inner_f32, var_any, g.tile_id);
        if (nb > 0) chunk_target = std::max(64, std::min(STEP_CHUNKS, nb * ctx->num_cus));
    }
    // layout
    size_t off = 0;
    const size_t off_probs = off;
    off += align256(sizeof(DevProb) * g.nprob);
    const size_t off_states = off;
    off += align256(sizeof(SolveState) * g.nprob);
    const size_t off_counters = off;
    off += align256(sizeof(unsigned) * g.nprob);
    std::vector<size_t> off_vec(g.nprob), off_part(g.nprob);
    g.probs.assign(g.nprob, DevProb());
    int tiles = 0, wgs = 0;
    // 3-D BiCGStab: the step kernel's own vectors (r, the inner vectors, w)
    // get a row pitch rounded up to 64, so that every 64-point row segment
    // the marching phases load starts on a 128-byte line (15-19 % faster
    // phases at n_x = 255); x, b and V keep the caller's pitch n_x.  The
    // other drivers' kernels and the 2-D tile paths assume pitch n_x.
    const bool padded = g.dim == 3 && prm->method == TGDK_BICGSTAB_PROJ;
    std::vector<size_t> nstore(g.nprob);  // elements per stored vector
    for (int j = 0; j < g.nprob; ++j) {
        const tgdk_op op = ps[j].op;
        DevProb& P = g.probs[j];
        memset(&P, 0, sizeof(P));
        P.op = make_devop(op, prm->transpose);
        if (padded) P.op.px = (op->n[0] + 63) / 64 * 64;
        nstore[j] = (size_t)P.op.px * op->n[1] * (g.dim == 3 ? op->n[2] : 1);
        P.tx = (op->n[0] + 63) / 64;
        P.ty = (op->n[1] + ty - 1) / ty;
        P.tz = g.dim == 3 ? (op->n[2] + tz - 1) / tz : 1;
        P.ntiles = P.tx * P.ty * P.tz;
        P.tile_begin = tiles;
        tiles += P.ntiles;
        if (g.dim == 3) {
            // z-marching chunks of the step kernel's phases (64 x MY columns,
            // about 1024 chunks in all); the boundary actions walk box tiles
            const int my = 8;
            P.mcx = (op->n[0] + 63) / 64;
            P.mcy = (op->n[1] + my - 1) / my;
            const long long cols = (long long)P.mcx * P.mcy;
            long long mz = (cols * op->n[2] + chunk_target - 1) / chunk_target;
            mz = std::max(4LL, std::min(mz, (long long)op->n[2]));
            P.mz = (int)mz;
            P.nchunks = (int)(cols * ((op->n[2] + P.mz - 1) / P.mz));
            P.nwg = P.nchunks;
        } else {
            P.nwg = std::min(P.ntiles, STEP_WG_CAP);
        }
        g.var |= P.op.var;
        P.wg_begin = wgs;
        wgs += P.nwg;
        P.k = ps[j].defl ? ps[j].defl->k : 0;
        // partial values per workgroup: at most 3 + k (true residual and c)
        P.pstride = std::max(8, 3 + P.k);
        P.pslot = (long long)P.pstride * P.nwg;
        off_vec[j] = off;
        const size_t n = nstore[j];
        off += align256(n * 8);                            // r (float64)
        off += (g.inner_f32 ? 10 : 9) * align256(n * ies);  // inner vectors
        if (g.dim == 3 && P.k > 0) off += align256(n * 8);  // w = V d (3-D boundary)
        off_part[j] = off;
        // tile kernels: ntiles rows; step kernel: two launch-parity slots
        off += align256((size_t)std::max((long long)P.ntiles * P.pstride, 2 * P.pslot) * 8);
    }
    g.total_tiles = tiles;
    g.total_wg = wgs;
    const size_t off_wgprob = off;
    off += align256(sizeof(int) * (size_t)wgs);
    const size_t off_actlog = off;
    if (ctx->time_which) off += align256(NSLOTLOG);
    const size_t off_ts = off;
    const bool stamps = ctx->time_which == 1;
    if (stamps) off += align256(sizeof(unsigned long long) * 2 * NTSLOG * (size_t)g.probs[0].nwg);
    int rc;
    char* base;
    if (ext) {
        if (off > ext->cap) {
            char msg[160];
            snprintf(msg, sizeof(msg), "the solve needs %zu bytes of workspace; the fixed scratch holds %zu", off,
                     ext->cap);
            return fail(TGDK_E_INVALID, msg);
        }
        if (ctx->mirror_cap < g.nprob || (int)ctx->events.size() < 2)
            return fail(TGDK_E_INVALID, "more systems than the context's preallocated status mirror holds");
        base = (char*)ext->base;
    } else {
        if ((rc = ctx->solve_ws.ensure(off))) return rc;
        if ((rc = ensure_mirror(ctx, g.nprob))) return rc;
        base = (char*)ctx->solve_ws.p;
    }
    g.d_probs = (DevProb*)(base + off_probs);
    g.d_states = (SolveState*)(base + off_states);
    g.d_wgprob = (int*)(base + off_wgprob);
    g.d_actlog = ctx->time_which ? (unsigned char*)(base + off_actlog) : nullptr;
    g.d_ts = stamps ? (unsigned long long*)(base + off_ts) : nullptr;
    unsigned* counters = (unsigned*)(base + off_counters);
    g.mirror = ctx->mirror;
    g.states.assign(g.nprob, SolveState());
    std::vector<int>& wgprob = g.wgprob;
    wgprob.assign((size_t)wgs, 0);
    for (int j = 0; j < g.nprob; ++j) {
        DevProb& P = g.probs[j];
        for (int w = 0; w < P.nwg; ++w) wgprob[(size_t)P.wg_begin + w] = j;
        const size_t n = nstore[j];
        char* v = base + off_vec[j];
        P.b = ps[j].b;
        P.x = ps[j].x;
        P.r = (double*)v;
        v += align256(n * 8);
        void* vecs[10];
        const int nv = g.inner_f32 ? 10 : 9;
        for (int i = 0; i < nv; ++i) {
            vecs[i] = v;
            v += align256(n * ies);
        }
        int i = 0;
        P.rin = g.inner_f32 ? vecs[i++] : (void*)P.r;
        P.rhat = vecs[i++];
        P.p[0] = vecs[i++];
        P.p[1] = vecs[i++];
        P.v[0] = vecs[i++];
        P.v[1] = vecs[i++];
        P.r2[0] = vecs[i++];  // r_i, alternating with p and v (no s is stored)
        P.r2[1] = vecs[i++];
        P.t = vecs[i++];
        P.e = vecs[i++];
        if (g.dim == 3 && P.k > 0) P.w = (double*)v;
        if (ps[j].defl) {
            P.V = ps[j].defl->V;
            P.Vl = ps[j].defl->W ? ps[j].defl->W : ps[j].defl->V;
            P.ldv = ps[j].defl->n;
            P.lu = ps[j].defl->d_lu;
            P.piv = ps[j].defl->d_piv;
            P.hinv = ps[j].defl->d_hinv;
            P.vtype = ps[j].defl->store == TGDK_F32 ? 1 : 0;
        }
        P.st = g.d_states + j;
        P.partial = (double*)(base + off_part[j]);
        P.actlog = j == 0 ? g.d_actlog : nullptr;
        P.tstamp = j == 0 ? g.d_ts : nullptr;
        P.counter = counters + j;
        P.mirror = g.mirror + j;
        SolveState& S = g.states[j];
        memset(&S, 0, sizeof(S));
        S.rtol = prm->rtol;
        S.fp32_floor = prm->fp32_floor > 0 ? prm->fp32_floor : 1e-4;
        S.method = prm->method == TGDK_GMRES_PROJ ? METHOD_GMRES
                   : prm->method == TGDK_IDRS_PROJ ? METHOD_IDR
                                                   : METHOD_BICGSTAB;
        if (S.method != METHOD_GMRES) {
            S.ncyc = prm->ncyc;
            S.max_extra = prm->max_extra_cycles >= 0 ? prm->max_extra_cycles : prm->ncyc;
        } else {
            S.ncyc = 0;
            S.max_extra = prm->max_extra_cycles > 0 ? prm->max_extra_cycles : 1000;
        }
        S.maxit = prm->maxit_cycle > 0 ? prm->maxit_cycle : 100000;
        P.maxit = S.maxit;
        S.k = P.k;
        S.precision = g.inner_f32;
        S.solve_state = SV_RUNNING;
        S.inner_state = IN_CONVERGED;
        // resuming at a cycle boundary: the cycle count continues from icyc0
        S.icyc0 = prm->icyc0;
        S.icyc = prm->icyc0;
        S.maxcyc_call = prm->max_cycles_call;
        S.nu0_in = prm->nu0;
        // the step kernel starts with the true residual of x0
        StepHot h;
        memset(&h, 0, sizeof(h));
        h.mode = M_RES;
        h.first = 1;
        h.icyc = prm->icyc0;
        h.solve_state = SV_RUNNING;
        h.inner_state = IN_CONVERGED;
        S.hot[0] = h;
        S.hot[1] = h;
        Mirror& m = g.mirror[j];
        m.solve_state = SV_RUNNING;
        m.inner_state = IN_RUNNING;
        m.icyc = 0;
        m.iter = 0;
        m.mode = M_RES;
        m.slot = -1;
        m.rr = m.rr0 = m.target2 = 0.0;
    }
    hipStream_t s = ctx->stream;
    TGDK_HIP(hipMemcpyAsync(g.d_probs, g.probs.data(), sizeof(DevProb) * g.nprob, hipMemcpyHostToDevice, s));
    TGDK_HIP(hipMemcpyAsync(g.d_states, g.states.data(), sizeof(SolveState) * g.nprob, hipMemcpyHostToDevice, s));
    TGDK_HIP(hipMemcpyAsync(g.d_wgprob, wgprob.data(), sizeof(int) * wgprob.size(), hipMemcpyHostToDevice, s));
    TGDK_HIP(hipMemsetAsync(counters, 0, sizeof(unsigned) * g.nprob, s));
    if (g.d_actlog) TGDK_HIP(hipMemsetAsync(g.d_actlog, 0, NSLOTLOG, s));
    if (g.d_ts)
        TGDK_HIP(hipMemsetAsync(g.d_ts, 0, sizeof(unsigned long long) * 2 * NTSLOG * (size_t)g.probs[0].nwg, s));
    // partial slots start finite (the first step sums them without using them)
    for (int j = 0; j < g.nprob; ++j)
        TGDK_HIP(hipMemsetAsync(g.probs[j].partial, 0, sizeof(double) * 2 * g.probs[j].pslot, s));
    if (!prm->x0_given)
        for (int j = 0; j < g.nprob; ++j)
            TGDK_HIP(hipMemsetAsync(ps[j].x, 0, sizeof(double) * ps[j].op->N, s));
    return TGDK_OK;
}

// Length-n vector operations of a solve in the paper's cost model (Sec. 3,
// Example 1: cost = nnz * mvps + vops; a dot product, a norm or an update
// y += a x counts one), from the counts of the run:
//  - BiCGStab iteration: rho, p (two updates), sigma, s, ||s||, t.s, t.t,
//    e (two updates), r, ||r||: 12; a half-step exit: rho, p, sigma, s,
//    ||s||, e: 7;
//  - GMRES cycle of j steps (CGS2): step i has two passes of i products and
//    i updates, the norm and the scaling (4i + 2), then r / ||r|| and
//    x += V y (j): 2 j^2 + 5 j + 1;
//  - IDR(s) (biorthogonal), per round of s + 1 operator applications: step k
//    forms u_k (2 (s - k) + 1), P^T g_k (s), orthogonalises g_k and u_k
//    against the earlier ones (2 k), forms M's column (s - k) and updates r,
//    e and ||r|| (3); the dimension reduction takes t.t, t.r, r.r, updates
//    e and r, forms P^T r and ||r|| (s + 6);
//  - every true residual r = b - A x with its norm and the x update: 3;
//    every projection: c = V^T r (k), V d (k), x, r and ||r|| (3).
static long long count_vops(const SolveState& S, int k, int idr_s, const std::vector<int>* cycle_steps) {
    const long long nres = S.mvp_boundary - S.nproj;
    long long v = 3 * nres + (2LL * k + 3) * S.nproj;
    if (S.method == METHOD_BICGSTAB) {
        long long half = 0;
        const int nc = std::min(S.icyc, NCYCLOG);
        for (int c = S.icyc0; c < nc; ++c) half += S.cyc_end[c] == IN_HALF ? 1 : 0;
        v += 12 * (S.iters_total - half) + 7 * half;
    } else if (S.method == METHOD_GMRES && cycle_steps) {
        for (int j : *cycle_steps) v += 2LL * j * j + 5LL * j + 1;
    } else if (S.method == METHOD_IDR && idr_s > 0) {
        const long long s = idr_s;
        long long round = s + 6;
        for (long long q = 0; q < s; ++q) round += 2 * (s - q) + 1 + s + 2 * q + (s - q) + 3;
        v += (round * S.mvp_inner) / (s + 1);
    }
    return v;
}

// cycle_steps: the GMRES driver's steps per cycle (one right-hand side);
// the other solvers' per-cycle counts come from the device's cycle log.
// idr_s: the shadow-space dimension of an IDR(s) solve (0 otherwise).
static int finish_group(Group& g, const std::vector<ProbSpec>& ps, tgdk_solve_report* reps, double secs,
                        const std::vector<long long>* extra_inner, const std::vector<int>* cycle_steps = nullptr,
                        int idr_s = 0) {
    hipStream_t s = g.ctx->stream;
    launch(g, K_RESIDUAL, 2);
    TGDK_HIP(hipGetLastError());
    TGDK_HIP(hipMemcpyAsync(g.states.data(), g.d_states, sizeof(SolveState) * g.nprob, hipMemcpyDeviceToHost, s));
    TGDK_HIP(hipStreamSynchronize(s));
    int rc = TGDK_OK;
    for (int j = 0; j < g.nprob; ++j) {
        const SolveState& S = g.states[j];
        tgdk_solve_report& R = reps[j];
        memset(&R, 0, sizeof(R));
        R.status = status_of(S);
        R.cycles = S.icyc;
        R.iters_inner = S.iters_total;
        R.mvp_inner = S.mvp_inner + (extra_inner ? (*extra_inner)[j] : 0);
        R.mvp_boundary = S.mvp_boundary;
        R.relres_true = S.bnorm > 0 ? S.nu_final / S.bnorm : S.nu_final;
        R.seconds = secs;
        for (int i = 0; i < 4; ++i) R.branch[i] = S.branch[i];
        R.n_first = S.nhist;
        for (int i = 0; i < S.nhist && i < TGDK_NHIST; ++i) {
            R.first_rho[i] = S.hist[3 * i];
            R.first_alpha[i] = S.hist[3 * i + 1];
            R.first_omega[i] = S.hist[3 * i + 2];
        }
        // inner operator applications per cycle: BiCGStab two per iteration
        // (one more when a breakdown follows phase A), IDR its count, GMRES
        // the host's step count
        const int nc = std::min(std::min(S.icyc, NCYCLOG), TGDK_NCYC_REPORT);
        for (int c = 0; c < nc; ++c) {
            int mv;
            if (S.method == METHOD_GMRES)
                mv = cycle_steps && c >= S.icyc0 && c - S.icyc0 < (int)cycle_steps->size()
                         ? (*cycle_steps)[c - S.icyc0]
                         : 0;
            else if (S.method == METHOD_IDR)
                mv = S.cyc_iters[c];
            else
                mv = 2 * S.cyc_iters[c] + (S.cyc_end[c] == IN_BREAK_NOUPD ? 1 : 0);
            R.cycle_mvps[c] = mv;
        }
        R.n_cycle_mvps = nc;
        for (int c = 0; c < nc; ++c) R.cycle_branch[c] = c >= S.icyc0 ? S.cyc_branch[c] : 0;
        R.nu0 = S.nu0;
        R.mvp_setup = ps[j].defl ? ps[j].defl->mvp_build : 0;
        R.vops = count_vops(S, g.probs[j].k, idr_s, cycle_steps);
        if (R.status == TGDK_E_NONFINITE) set_error("non-finite residual (check b, x0 and the operator)");
        rc = worst(rc, R.status);
    }
    return rc;
}

static bool all_solved(const Group& g) {
    for (int j = 0; j < g.nprob; ++j)
        if (read_mirror(g, j).solve_state == SV_RUNNING) return false;
    return true;
}

// Steps a running problem will take before it can have finished: the rest of
// its inner cycle (extrapolating the residual reduction per iteration of this
// cycle, or of the last one early in a cycle), the boundary steps, and a next
// cycle as long as this one (enqueued ahead, so the queue does not drain at a
// boundary; launches past the end of the solve return at once).
struct Predict {
    double rate = 0.0;  // residual reduction per iteration
    int len = 8;        // iterations of the current (or last) cycle
};
static int predict_steps(const Mirror& m, Predict& pr) {
    if (m.solve_state != SV_RUNNING) return 0;
    if (m.mode != M_A && m.mode != M_B) return 3 + 2 * pr.len + 3;
    if (m.iter >= 2 && m.rr > 0.0 && m.rr0 > 0.0 && m.rr < m.rr0) pr.rate = std::pow(m.rr / m.rr0, 1.0 / m.iter);
    int rem = 8;
    if (pr.rate > 0.0 && pr.rate < 0.999 && m.rr > 0.0 && m.target2 > 0.0)
        rem = m.rr <= m.target2 ? 1 : (int)std::ceil(std::log(m.target2 / m.rr) / std::log(pr.rate));
    rem = std::max(1, std::min(rem, 64));
    pr.len = std::max(2, m.iter + rem);
    return 2 * rem + 3 + 2 * pr.len + 3;
}

// BiCGStab(ncyc)-Proj(k) over a group: step launches only.  At most two
// batches are outstanding; when the older one completes, the host reads the
// status mirror and enqueues as many steps as the slowest running problem is
// predicted to need (steps past the end of a solve return at once but still
// cost a dispatch each).
static int bicgstab_group(tgdk_ctx ctx, const std::vector<ProbSpec>& ps, const tgdk_solve_params* prm,
                          tgdk_solve_report* reps, const ExtWs* ext = nullptr) {
    const auto t0 = std::chrono::steady_clock::now();
    Group g;
    int rc = build_group(ctx, ps, prm, g, ext);
    if (rc) return rc;
    if (!ext && (rc = ensure_events(ctx, 2))) return rc;
    hipStream_t s = ctx->stream;
    const int S_MAX = 24;  // largest batch of steps enqueued at once
    const long long max_cycles = prm->ncyc + (prm->max_extra_cycles >= 0 ? prm->max_extra_cycles : prm->ncyc) + 2;
    const long long maxit = prm->maxit_cycle > 0 ? prm->maxit_cycle : 100000;
    const long long slot_cap = max_cycles * (2 * maxit + 6) + 16;
    std::vector<Predict> pred(g.nprob);
    int ev_slot[2] = {0, 0};
    int head = 0, tail = 0;
    auto enqueue = [&](int cnt) -> int {
        for (int i = 0; i < cnt; ++i) {
            int r2 = launch_step_timed(g);
            if (r2) return r2;
        }
        TGDK_HIP(hipGetLastError());
        TGDK_HIP(hipEventRecord(ctx->events[tail % 2], s));
        ev_slot[tail % 2] = g.gslot;
        ++tail;
        return TGDK_OK;
    };
    if ((rc = enqueue(8))) return rc;
    for (;;) {
        if ((rc = wait_event(ctx->events[head % 2]))) return rc;
        const int completed = ev_slot[head % 2];
        ++head;
        if (all_solved(g)) break;
        if (g.gslot >= slot_cap) break;  // the device's own cycle and iteration limits end every solve first
        int want = 0;
        for (int j = 0; j < g.nprob; ++j) {
            const Mirror m = read_mirror(g, j);
            // a running problem reports every step it takes
            if (m.solve_state == SV_RUNNING && m.slot < completed - 64)
                return fail(TGDK_E_HIP, "step kernel stopped reporting progress");
            want = std::max(want, predict_steps(m, pred[j]));
        }
        want -= g.gslot - completed;
        // keep two batches queued while steps are predicted
        while (want > 0 && tail - head < 2) {
            const int cnt = std::min(want, S_MAX);
            if ((rc = enqueue(cnt))) return rc;
            want -= cnt;
        }
        if (tail == head && (rc = enqueue(2))) return rc;
    }
    // drain what is still queued (those steps find every problem finished)
    TGDK_HIP(hipStreamSynchronize(s));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    rc = finish_group(g, ps, reps, secs, nullptr);
    if (ctx->time_which) {
        int r2 = collect_timing(g);
        if (r2) return r2;
    }
    return rc;
}

// GMRES(m)-Proj(k): one right-hand side.  Arnoldi with classical
// Gram-Schmidt and one full re-orthogonalisation (CGS2), Hessenberg
// least squares on the host at the end of each cycle.
static int gmres_single(tgdk_ctx ctx, const ProbSpec& p, const tgdk_solve_params* prm, tgdk_solve_report* rep) {
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<ProbSpec> ps{p};
    Group g;
    int rc = build_group(ctx, ps, prm, g);
    if (rc) return rc;
    hipStream_t s = ctx->stream;
    const int m = prm->m3;
    const long long n = p.op->N;
    // Krylov basis, w, H columns
    double *V = nullptr, *w = nullptr, *Hd = nullptr, *dy = nullptr, *pz = nullptr;
    const size_t hsz = (size_t)(m + 1) * m;
    const bool pre = prm->precond != nullptr;
    if (hipMalloc((void**)&V, sizeof(double) * n * (m + 1)) != hipSuccess)
        return fail(TGDK_E_NOMEM, "GMRES basis allocation failed");
    if (hipMalloc((void**)&w, sizeof(double) * n * (pre ? 3 : 1)) != hipSuccess ||
        hipMalloc((void**)&Hd, sizeof(double) * (2 * hsz + m + 8)) != hipSuccess ||
        hipMalloc((void**)&dy, sizeof(double) * (m + 1)) != hipSuccess) {
        (void)hipFree(V);
        if (w) (void)hipFree(w);
        if (Hd) (void)hipFree(Hd);
        return fail(TGDK_E_NOMEM, "GMRES workspace allocation failed");
    }
    double* H1 = Hd;
    double* H2 = Hd + hsz;
    double* Nd = Hd + 2 * hsz;
    pz = pre ? w + n : nullptr;             // M^{-1} v_j; then M^{-1} (V y)
    double* pu = pre ? w + 2 * n : nullptr;  // V y
    rc = ctx->partial.ensure((size_t)gs_blocks(n) * (MAXK + 1) * sizeof(double));
    std::vector<long long> extra(1, 0);
    std::vector<int> cyc_steps;  // steps of each cycle
    const DevOp op = make_devop(p.op, prm->transpose);
    const int maxcyc = prm->max_extra_cycles > 0 ? prm->max_extra_cycles : 1000;
    std::vector<double> h1(hsz), h2(hsz), nrm(m), Hbar(hsz), rhs(m + 1), y(m), res(m + 1);
    SolveState S;
    double* d_nu = &g.d_states[0].nu;
    if (!rc) {
        launch(g, K_RESIDUAL, 1);
        TGDK_HIP(hipStreamSynchronize(s));
    }
    for (int cyc = 0; cyc < maxcyc && !rc; ++cyc) {
        if (all_solved(g)) break;
        if (p.defl) {
            launch(g, K_PROJ_DOT);
            launch(g, K_PROJ_APPLY);
            TGDK_HIP(hipStreamSynchronize(s));
            if (all_solved(g)) break;
        }
        launch_scale(g.probs[0].r, V, d_nu, n, s);
        // this cycle's length (variable restarting), at most m
        const int mc = cyc < prm->n_cycle_lengths && prm->cycle_lengths ? prm->cycle_lengths[cyc] : m;
        int steps = mc;
        for (int j = 0; j < mc; ++j) {
            if (pre) {  // right preconditioning: w = A M^{-1} v_j
                if ((rc = prm->precond(prm->precond_user, V + (size_t)j * n, pz, 1))) break;
                launch_apply<double>(op, pz, w, 1, p.op->tile_id[0], s);
            } else {
                launch_apply<double>(op, V + (size_t)j * n, w, 1, p.op->tile_id[0], s);
            }
            launch_gs_dot(V, n, j + 1, w, n, H1 + (size_t)j * (m + 1), (double*)ctx->partial.p, ctx->counters, s);
            launch_gs_update_dot(V, n, j + 1, w, H1 + (size_t)j * (m + 1), n, H2 + (size_t)j * (m + 1),
                                 (double*)ctx->partial.p, ctx->counters, s);
            launch_gs_update_norm(V, n, j + 1, w, H2 + (size_t)j * (m + 1), n, Nd + j, (double*)ctx->partial.p,
                                  ctx->counters, s);
            launch_scale(w, V + (size_t)(j + 1) * n, Nd + j, n, s);
        }
        if (rc) break;
        TGDK_HIP(hipGetLastError());
        TGDK_HIP(hipMemcpyAsync(h1.data(), H1, sizeof(double) * hsz, hipMemcpyDeviceToHost, s));
        TGDK_HIP(hipMemcpyAsync(h2.data(), H2, sizeof(double) * hsz, hipMemcpyDeviceToHost, s));
        TGDK_HIP(hipMemcpyAsync(nrm.data(), Nd, sizeof(double) * m, hipMemcpyDeviceToHost, s));
        TGDK_HIP(hipMemcpyAsync(&S, g.d_states, sizeof(SolveState), hipMemcpyDeviceToHost, s));
        TGDK_HIP(hipStreamSynchronize(s));
        // Hbar (row-major (m+1) x m); stop at an exact zero subdiagonal
        std::fill(Hbar.begin(), Hbar.end(), 0.0);
        for (int j = 0; j < mc; ++j) {
            for (int i = 0; i <= j; ++i) Hbar[(size_t)i * m + j] = h1[(size_t)j * (m + 1) + i] + h2[(size_t)j * (m + 1) + i];
            Hbar[(size_t)(j + 1) * m + j] = nrm[j];
            if (nrm[j] == 0.0) {
                steps = j + 1;
                break;
            }
        }
        std::vector<double> Hs((size_t)(steps + 1) * steps);
        for (int i = 0; i <= steps; ++i)
            for (int j = 0; j < steps; ++j) Hs[(size_t)i * steps + j] = Hbar[(size_t)i * m + j];
        std::fill(rhs.begin(), rhs.end(), 0.0);
        rhs[0] = S.nu;
        lstsq(steps + 1, steps, Hs.data(), rhs.data(), y.data(), res.data());
        TGDK_HIP(hipMemcpyAsync(dy, y.data(), sizeof(double) * steps, hipMemcpyHostToDevice, s));
        if (pre) {  // x += M^{-1} (V y)
            launch_vmul(V, n, steps, dy, 1, pu, n, n, s);
            if ((rc = prm->precond(prm->precond_user, pu, pz, 1))) break;
            launch_add(p.x, pz, n, s);
        } else {
            launch_vmul_add(V, n, steps, dy, p.x, n, s);
        }
        extra[0] += steps;
        cyc_steps.push_back(steps);
        launch(g, K_RESIDUAL, 0);
        TGDK_HIP(hipGetLastError());
        TGDK_HIP(hipStreamSynchronize(s));
    }
    (void)hipFree(V);
    (void)hipFree(w);
    (void)hipFree(Hd);
    (void)hipFree(dy);
    if (rc) return rc;
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return finish_group(g, ps, rep, secs, &extra, &cyc_steps);
}

// IDR(s)(ncyc)-Proj(k): one right-hand side.  The cycle boundary is the
// GMRES driver's (true residual, projection; the cycle tolerance is set on
// the device); the IDR rounds are enqueued ahead in batches sized from the
// residual reduction seen so far, at most two batches outstanding, and end on
// the device (kernels_idr.hip).  The host waits only at cycle ends.
static int idr_single(tgdk_ctx ctx, const ProbSpec& p, int s, const double* shadow, double kappa,
                      const tgdk_solve_params* prm, tgdk_solve_report* rep) {
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<ProbSpec> ps{p};
    Group g;
    int rc = build_group(ctx, ps, prm, g);
    if (rc) return rc;
    if ((rc = ensure_events(ctx, 2))) return rc;
    hipStream_t hs = ctx->stream;
    const long long n = p.op->N;
    const int f32 = g.inner_f32;
    const size_t ies = f32 ? 4 : 8;
    const size_t sn = (size_t)s * n;
    // G, U, P in the inner type; P64 (the orthonormalised draw); the state
    const size_t off_u = align256(sn * ies), off_p = off_u + align256(sn * ies);
    const size_t off_p64 = off_p + (f32 ? align256(sn * ies) : 0);
    const size_t off_st = off_p64 + align256(sn * 8);
    const size_t off_pz = off_st + align256(sizeof(IdrState));  // preconditioner output
    const size_t bytes = off_pz + (prm->precond ? align256((size_t)n * 8) : 0);
    char* wk = nullptr;
    if (hipMalloc((void**)&wk, bytes) != hipSuccess) return fail(TGDK_E_NOMEM, "IDR workspace allocation failed");
    double* P64 = (double*)(wk + off_p64);
    IdrState* d_st = (IdrState*)(wk + off_st);
    auto done = [&](int code) {
        (void)hipStreamSynchronize(hs);
        (void)hipFree(wk);
        return code;
    };
#define IDR_HIP(call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess) return done(fail(TGDK_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_))); \
    } while (0)
    IDR_HIP(hipMemcpyAsync(P64, shadow, sn * 8, hipMemcpyDeviceToDevice, hs));
    if ((rc = cholqr2(ctx, P64, n, s))) return done(rc == TGDK_E_SINGULAR ? fail(rc, "shadow space is rank deficient") : rc);
    if (f32) launch_to_f32(P64, (float*)(wk + off_p), (long long)sn, hs);
    IdrState h;
    memset(&h, 0, sizeof(h));
    h.gate = 1;
    h.s = s;
    h.kappa = kappa;
    h.status = IN_CONVERGED;
    IDR_HIP(hipMemcpyAsync(d_st, &h, sizeof(h), hipMemcpyHostToDevice, hs));
    IdrArgs a;
    memset(&a, 0, sizeof(a));
    DevProb& P = g.probs[0];
    a.r = P.rin;
    a.e = P.e;
    a.t = P.t;
    a.G = wk;
    a.U = wk + off_u;
    a.P = f32 ? (const void*)(wk + off_p) : (const void*)P64;
    a.x = p.x;
    a.n = n;
    a.nb = idr_blocks(n);
    a.s = s;
    a.st = d_st;
    a.ss = g.d_states;
    a.mirror = g.mirror;
    // partial sums: s + 1 values (P^T r and r . r), 3 for omega
    if ((rc = ctx->partial.ensure((size_t)a.nb * std::max(s + 1, 3) * sizeof(double)))) return done(rc);
    a.part = (double*)ctx->partial.p;
    const DevOp op = make_devop(p.op, prm->transpose);
    const int tile = p.op->tile_id[f32];
    const int* gate = &d_st->gate;
    const size_t eln = (size_t)n * ies;
    auto col = [&](void* base, int k) { return (void*)((char*)base + (size_t)k * eln); };
    const bool pre = prm->precond != nullptr;  // float64 only (checked)
    double* pz = pre ? (double*)(wk + off_pz) : nullptr;
    int prc = TGDK_OK;                          // first preconditioner failure
    auto apply = [&](const void* x, void* y) {
        if (pre) {  // right preconditioning: y = A M^{-1} x
            if (!prc) prc = prm->precond(prm->precond_user, (const double*)x, pz, 1);
            launch_apply<double>(op, pz, (double*)y, 1, tile, hs, gate);
        } else if (f32) {
            launch_apply<float>(op, (const float*)x, (float*)y, 1, tile, hs, gate);
        } else {
            launch_apply<double>(op, (const double*)x, (double*)y, 1, tile, hs, gate);
        }
    };
    // 2-D grids with s <= 8: each stencil forms its step's products too
    // (P^T g_k, or t.t, t.r, r.r), so no separate pass re-reads g_k or t, and
    // step 0 needs no orthogonalisation pass (its products are P^T g_0)
    const bool fused = op.dim == 2 && s <= 8;
    auto fused_apply = [&](int what, void* x, void* y, int k) {
        const void* in = x;
        if (pre) {  // right preconditioning: the stencil takes M^{-1} x
            if (!prc) prc = prm->precond(prm->precond_user, (const double*)x, pz, 1);
            in = pz;
        }
        launch_idr_fused(what, f32, a, op, tile, in, y, k, hs);
    };
    // a round: step 0's direction, then for k >= 1 the update of step k-1
    // fused with step k's direction, the last step's update on its own, and
    // the dimension reduction
    auto round = [&]() {
        for (int k = 0; k < s; ++k) {
            launch_idr(k == 0 ? IDR_DIR : IDR_DIRUPD, f32, a, k, hs);
            if (fused) {
                fused_apply(IDR_ALPHA, col(a.U, k), col(a.G, k), k);
                if (k > 0) launch_idr(IDR_ORTH, f32, a, k, hs);
            } else {
                apply(col(a.U, k), col(a.G, k));
                if (k > 0) launch_idr(IDR_ALPHA, f32, a, k, hs);
                launch_idr(IDR_ORTH, f32, a, k, hs);
            }
        }
        launch_idr(IDR_UPD, f32, a, s - 1, hs);
        if (fused) {
            fused_apply(IDR_OMEGA, a.r, a.t, 0);
        } else {
            apply(a.r, a.t);
            launch_idr(IDR_OMEGA, f32, a, 0, hs);
        }
        launch_idr(IDR_RED, f32, a, 0, hs);
    };
    const int maxcyc = prm->ncyc + (prm->max_extra_cycles >= 0 ? prm->max_extra_cycles : prm->ncyc) + 2;
    launch(g, K_RESIDUAL, 1);
    IDR_HIP(hipGetLastError());
    IDR_HIP(hipStreamSynchronize(hs));
    double rate = 0.0;  // squared residual reduction per operator application
    for (int cyc = 0; cyc < maxcyc; ++cyc) {
        if (all_solved(g)) break;
        if (p.defl) {
            launch(g, K_PROJ_DOT);
            launch(g, K_PROJ_APPLY);
        }
        if (pre) launch_fill((double*)a.e, 0.0, n, hs);  // the fold below reads e whatever the cycle did
        launch_idr(IDR_START, f32, a, 0, hs);
        IDR_HIP(hipGetLastError());
        // rounds until the device ends the cycle
        int ev_mvps = -1, head = 0, tail = 0, nr = 1;
        for (;;) {
            while (tail - head < 2) {
                for (int i = 0; i < nr; ++i) round();
                IDR_HIP(hipGetLastError());
                IDR_HIP(hipEventRecord(ctx->events[tail % 2], hs));
                ++tail;
            }
            if ((rc = wait_event(ctx->events[head % 2]))) return done(rc);
            ++head;
            if (prc) return done(prc);
            const Mirror m = read_mirror(g, 0);
            if (m.solve_state != SV_RUNNING || m.inner_state != IN_RUNNING) break;
            if (m.iter == ev_mvps) return done(fail(TGDK_E_HIP, "IDR cycle stopped reporting progress"));
            ev_mvps = m.iter;
            if (m.iter >= 2 && m.rr > 0.0 && m.rr0 > 0.0 && m.rr < m.rr0) rate = std::pow(m.rr / m.rr0, 1.0 / m.iter);
            int rem = s + 1;
            if (rate > 0.0 && rate < 0.9999 && m.rr > 0.0 && m.target2 > 0.0 && m.rr > m.target2)
                rem = (int)std::ceil(std::log(m.target2 / m.rr) / std::log(rate));
            nr = pre ? 1 : std::max(1, std::min(8, (rem + s) / (s + 1)));
        }
        if (pre) {  // x += M^{-1} e (e is zero if the cycle made no update)
            if ((rc = prm->precond(prm->precond_user, (const double*)a.e, pz, 1))) return done(rc);
            launch_add(p.x, pz, n, hs);
        } else {
            launch_idr(IDR_FOLD, f32, a, 0, hs);
        }
        launch(g, K_RESIDUAL, 0);
        IDR_HIP(hipGetLastError());
        IDR_HIP(hipStreamSynchronize(hs));
    }
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    rc = finish_group(g, ps, rep, secs, nullptr, nullptr, s);
    return done(rc);
#undef IDR_HIP
}

static int check_params(const tgdk_solve_params* prm) {
    if (!prm) return fail(TGDK_E_INVALID, "params is NULL");
    if (prm->method == TGDK_BICGSTAB_PROJ) {
        if (prm->ncyc < 1) return fail(TGDK_E_INVALID, "ncyc must be >= 1");
    } else if (prm->method == TGDK_IDRS_PROJ) {
        if (prm->ncyc < 1) return fail(TGDK_E_INVALID, "ncyc must be >= 1");
    } else if (prm->method == TGDK_GMRES_PROJ) {
        if (prm->m3 < 1 || prm->m3 > MAXK) return fail(TGDK_E_INVALID, "m3 out of range");
        if (prm->n_cycle_lengths < 0 || (prm->n_cycle_lengths > 0 && !prm->cycle_lengths))
            return fail(TGDK_E_INVALID, "cycle_lengths");
        for (int j = 0; j < prm->n_cycle_lengths; ++j)
            if (prm->cycle_lengths[j] < 1 || prm->cycle_lengths[j] > prm->m3)
                return fail(TGDK_E_INVALID, "cycle lengths must be in 1..m3");
        if (prm->precision != TGDK_FP64) return fail(TGDK_E_INVALID, "GMRES-Proj runs in float64 only");
    } else {
        return fail(TGDK_E_INVALID, "unknown method");
    }
    if (prm->precision != TGDK_FP64 && prm->precision != TGDK_FP32_IR) return fail(TGDK_E_INVALID, "precision");
    if (prm->precond) {
        if (prm->method == TGDK_BICGSTAB_PROJ)
            return fail(TGDK_E_INVALID, "right preconditioning is available for GMRES-Proj and IDR-Proj");
        if (prm->precision != TGDK_FP64) return fail(TGDK_E_INVALID, "preconditioned solves run in float64");
    }
    if (!(prm->rtol > 0.0)) return fail(TGDK_E_INVALID, "rtol must be > 0");
    if (prm->icyc0 < 0 || prm->max_cycles_call < 0 || !(prm->nu0 >= 0.0))
        return fail(TGDK_E_INVALID, "icyc0, max_cycles_call and nu0 must be >= 0");
    if (prm->icyc0 > 0 && !prm->x0_given) return fail(TGDK_E_INVALID, "a resumed solve (icyc0 > 0) needs x0_given");
    return TGDK_OK;
}

static int check_defl(tgdk_op op, tgdk_defl d, const tgdk_solve_params* prm) {
    if (!d) return TGDK_OK;
    if (d->n != op->N || d->op->dim != op->dim) return fail(TGDK_E_INVALID, "deflation space size does not match the operator");
    for (int a = 0; a < op->dim; ++a)
        if (d->op->n[a] != op->n[a]) return fail(TGDK_E_INVALID, "deflation space grid does not match the operator");
    if (d->transpose != (prm->transpose ? 1 : 0))
        return fail(TGDK_E_INVALID, "deflation space was built for the other orientation (A vs A^T)");
    if ((d->precond != 0) != (prm->precond != nullptr))
        return fail(TGDK_E_INVALID, "a preconditioned solve needs a space from tgdk_defl_precond, and only it");
    return TGDK_OK;
}

// BiCGStab(ncyc)-Proj(k) on nrhs systems with the workspace laid out in the
// caller's scratch (base, cap bytes): the no-allocation entry point.
int solve_bicgstab_in(tgdk_op fine, tgdk_defl defl, const double* b, double* x, int nrhs,
                      const tgdk_solve_params* prm, tgdk_solve_report* reports, void* base, size_t cap) {
    if (!fine || !b || !x || nrhs < 1 || !reports) return fail(TGDK_E_INVALID, "bad argument");
    int rc = check_params(prm);
    if (rc) return rc;
    if (prm->method != TGDK_BICGSTAB_PROJ) return fail(TGDK_E_INVALID, "the no-allocation solve is BiCGStab-Proj");
    if ((rc = check_defl(fine, defl, prm))) return rc;
    if (fine->ctx->time_which) return fail(TGDK_E_INVALID, "switch the step-kernel timing off for this call");
    TGDK_HIP(hipSetDevice(fine->ctx->device));
    std::vector<ProbSpec> ps(nrhs);
    for (int j = 0; j < nrhs; ++j) ps[j] = ProbSpec{fine, defl, b + (size_t)j * fine->N, x + (size_t)j * fine->N};
    const ExtWs ext{base, cap};
    return bicgstab_group(fine->ctx, ps, prm, reports, &ext);
}

}  // namespace tgdk

using namespace tgdk;

extern "C" {

int tgdk_solve(tgdk_op fine, tgdk_defl defl, const double* b, double* x, int nrhs, const tgdk_solve_params* prm,
               tgdk_solve_report* reports) {
    if (!fine || !b || !x || nrhs < 1 || !reports) return fail(TGDK_E_INVALID, "bad argument");
    int rc = check_params(prm);
    if (rc) return rc;
    if ((rc = check_defl(fine, defl, prm))) return rc;
    TGDK_HIP(hipSetDevice(fine->ctx->device));
    std::vector<ProbSpec> ps(nrhs);
    for (int j = 0; j < nrhs; ++j) ps[j] = ProbSpec{fine, defl, b + (size_t)j * fine->N, x + (size_t)j * fine->N};
    if (prm->method == TGDK_IDRS_PROJ) return fail(TGDK_E_INVALID, "IDR(s)-Proj is solved by tgdk_solve_idr");
    if (prm->method == TGDK_GMRES_PROJ) {
        if (nrhs != 1) return fail(TGDK_E_INVALID, "GMRES-Proj takes one right-hand side");
        return gmres_single(fine->ctx, ps[0], prm, reports);
    }
    return bicgstab_group(fine->ctx, ps, prm, reports);
}

int tgdk_solve_idr(tgdk_op fine, tgdk_defl defl, const double* b, double* x, int s, const double* shadow,
                   double kappa, const tgdk_solve_params* prm, tgdk_solve_report* report) {
    if (!fine || !b || !x || !shadow || !report) return fail(TGDK_E_INVALID, "bad argument");
    int rc = check_params(prm);
    if (rc) return rc;
    if (prm->method != TGDK_IDRS_PROJ) return fail(TGDK_E_INVALID, "params.method must be TGDK_IDRS_PROJ");
    if (s < 1 || s > IDR_SMAX) return fail(TGDK_E_INVALID, "s out of range (1..TGDK_IDR_SMAX)");
    if ((long long)s > fine->N) return fail(TGDK_E_INVALID, "s exceeds the number of unknowns");
    if (!(kappa >= 0.0 && kappa < 1.0)) return fail(TGDK_E_INVALID, "kappa must be in [0, 1)");
    if ((rc = check_defl(fine, defl, prm))) return rc;
    TGDK_HIP(hipSetDevice(fine->ctx->device));
    return idr_single(fine->ctx, ProbSpec{fine, defl, b, x}, s, shadow, kappa, prm, report);
}

int tgdk_solve_instances(tgdk_ctx ctx, int ninst, const tgdk_op* ops, const tgdk_defl* defls, const double* const* b,
                         double* const* x, const tgdk_solve_params* prm, tgdk_solve_report* reports) {
    if (!ctx || ninst < 1 || !ops || !b || !x || !reports) return fail(TGDK_E_INVALID, "bad argument");
    int rc = check_params(prm);
    if (rc) return rc;
    if (prm->method != TGDK_BICGSTAB_PROJ) return fail(TGDK_E_INVALID, "instances use BiCGStab-Proj");
    std::vector<ProbSpec> ps(ninst);
    for (int j = 0; j < ninst; ++j) {
        if (!ops[j] || !b[j] || !x[j]) return fail(TGDK_E_INVALID, "NULL instance");
        if (ops[j]->ctx != ctx || ops[j]->dim != ops[0]->dim)
            return fail(TGDK_E_INVALID, "instances must belong to the context and share a dimension");
        tgdk_defl d = defls ? defls[j] : nullptr;
        if ((rc = check_defl(ops[j], d, prm))) return rc;
        ps[j] = ProbSpec{ops[j], d, b[j], x[j]};
    }
    TGDK_HIP(hipSetDevice(ctx->device));
    return bicgstab_group(ctx, ps, prm, reports);
}

}  // extern "C"
