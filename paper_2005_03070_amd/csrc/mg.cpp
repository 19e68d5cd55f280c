// Geometric multigrid V-cycles for a constant-coefficient operator: the
// preconditioner of Sec. 5, Example 5 (solutions with the positively shifted
// Laplacian precondition the Helmholtz operator).  Levels are the operator's
// grid and its rediscretised nested coarse grids while every side is odd and
// at least 3; damped Jacobi smoothing (omega 4/5 in 2-D, 6/7 in 3-D) around a
// full-weighting / linear-interpolation coarse correction; 20 sweeps on the
// coarsest grid.  The preconditioner is a fixed number of V-cycles from zero,
// a fixed linear operator.
//
// The host walks the fine levels and enqueues one kernel per pass (the first
// two sweeps fused, the residual fused into the restriction, the coarse
// correction fused into the first post-sweep: 4 passes per level with two
// sweeps); the coarse tail of the hierarchy (the levels whose z, v and sweep
// temporary fit in the LDS budget) is one single-workgroup launch
// (kernels_mg.hip).  A 511^2 V-cycle is 17 launches.
// The kernel sequence of one application is captured once into a HIP graph on
// a private stream and replayed on the context's stream; the caller's vectors
// are copied in and out around it, so the graph only touches the object's own
// buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "host.h"

struct tgdk_mg_s {
    tgdk_ctx ctx = nullptr;
    std::vector<tgdk_op> ops;       // level 0: the caller's operator (not owned)
    std::vector<tgdk::MgLvl> lv;    // per level: sides, stencil, Jacobi factor
    std::vector<double*> z, v, t;   // per level: z and t ping-pong, v the right-hand side
    double* acc = nullptr;          // level 0: the accumulated solution
    double* bin = nullptr;          // level 0: the right-hand side, copied in
    int cycles = 2, nu = 2;
    double omega = 0.8;
    int tail = 0;                   // first level of the single-workgroup tail (ops.size(): none)
    tgdk::MgTail* tail_dev = nullptr;
    int use_graph = 1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace tgdk {

constexpr int MG_COARSEST_SWEEPS = 20;

// One V-cycle for A_l z_l = v from z = 0.  Returns the buffer holding z_l;
// with dst set (level 0) the last pass writes dst instead (added to it if
// acc).
static const double* vcycle(tgdk_mg mg, int l, const double* v, double* dst, int acc, hipStream_t s) {
    const int dim = mg->ops[0]->dim;
    if (l == mg->tail) {
        double* out = dst ? dst : mg->z[l];
        launch_mg_tail(dim, mg->tail_dev, v, out, dst ? acc : 0, s);
        return out;
    }
    const MgLvl& L = mg->lv[l];
    double *a = mg->z[l], *b = mg->t[l];
    // count sweeps, from z = 0 (start null: the first two fused) or after the
    // coarse correction (zc set: the first one fused with it), ping-ponging
    // between a and b
    auto smooth = [&](int count, const double* start, const double* zc, bool last_to_dst) {
        const double* cur = start;
        const int passes = !start && count >= 2 ? count - 1 : count;
        for (int i = 0; i < passes; ++i) {
            const bool fin = last_to_dst && dst && i == passes - 1;
            double* o = fin ? dst : (cur == a ? b : a);
            int mode = MG_SWEEP;
            if (i == 0 && !start) mode = count >= 2 ? MG_FIRST2 : MG_FIRST;
            if (i == 0 && zc) mode = MG_PSWEEP;
            if (fin && acc) mode |= MG_ACC;
            launch_mg_pass(dim, L, cur, v, i == 0 ? zc : nullptr, o, mode, s);
            cur = o;
        }
        return cur;
    };
    if (l + 1 == (int)mg->ops.size()) return smooth(MG_COARSEST_SWEEPS, nullptr, nullptr, true);
    const double* zs = smooth(mg->nu, nullptr, nullptr, false);
    launch_mg_resid_restrict(dim, L, zs, v, mg->v[l + 1], s);
    const double* zc = vcycle(mg, l + 1, mg->v[l + 1], nullptr, 0, s);
    return smooth(mg->nu, zs, zc, true);
}

// The whole preconditioner on bin -> acc: z_1 = V(b), z_(c+1) = z_c + V(b - A z_c).
static void mg_body(tgdk_mg mg, hipStream_t s) {
    vcycle(mg, 0, mg->bin, mg->acc, 0, s);
    for (int c = 1; c < mg->cycles; ++c) {
        launch_mg_pass(mg->ops[0]->dim, mg->lv[0], mg->acc, mg->bin, nullptr, mg->v[0], MG_RESID, s);
        vcycle(mg, 0, mg->v[0], mg->acc, 1, s);
    }
}

// The tail: the longest run of coarsest levels (at most MG_TAIL_MAXLEV)
// whose z, v and sweep temporary fit in MG_TAIL_LDS doubles.
static int plan_tail(tgdk_mg mg, MgTail& P) {
    const int L = (int)mg->ops.size();
    int first = L;
    long long used = 0;
    for (int l = L - 1; l >= 0 && L - l <= MG_TAIL_MAXLEV; --l) {
        used += 3 * mg->ops[l]->N;
        if (used > MG_TAIL_LDS) break;
        first = l;
    }
    P = MgTail{};
    P.dim = mg->ops[0]->dim;
    P.nlev = L - first;
    P.nu = mg->nu;
    P.coarsest_sweeps = MG_COARSEST_SWEEPS;
    P.wave_from = P.nlev;
    for (int l = L - 1; l >= first && mg->ops[l]->N <= 64; --l) P.wave_from = l - first;
    int off = 0;
    for (int l = first; l < L; ++l) {
        const int n = (int)mg->ops[l]->N;
        P.lv[l - first] = mg->lv[l];
        P.zoff[l - first] = off;
        P.voff[l - first] = off + n;
        P.toff[l - first] = off + 2 * n;
        off += 3 * n;
    }
    return first;
}

// Captures mg_body into a graph on a private stream (once per object).
static int mg_capture(tgdk_mg mg) {
    hipStream_t cs = nullptr;
    TGDK_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        mg_body(mg, cs);
        e = hipStreamEndCapture(cs, &mg->graph);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&mg->exec, mg->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        if (mg->graph) (void)hipGraphDestroy(mg->graph);
        mg->graph = nullptr;
        mg->exec = nullptr;
        return fail(TGDK_E_HIP, std::string("multigrid graph capture failed: ") + hipGetErrorString(e));
    }
    return TGDK_OK;
}

}  // namespace tgdk

using namespace tgdk;

extern "C" {

int tgdk_mg_create(tgdk_op op, int cycles, int nu, int flags, tgdk_mg* out) {
    if (!op || !out) return fail(TGDK_E_INVALID, "NULL argument");
    if (op->kind != TGDK_CONST_CD) return fail(TGDK_E_INVALID, "multigrid needs a constant-coefficient operator");
    if (cycles < 1 || nu < 1) return fail(TGDK_E_INVALID, "need cycles >= 1, nu >= 1");
    if (!(op->cc[0] > 0.0)) return fail(TGDK_E_INVALID, "multigrid needs a positive diagonal");
    TGDK_HIP(hipSetDevice(op->ctx->device));
    tgdk_mg mg = new tgdk_mg_s();
    mg->ctx = op->ctx;
    mg->cycles = cycles;
    mg->nu = nu;
    mg->omega = op->dim == 2 ? 4.0 / 5.0 : 6.0 / 7.0;
    mg->use_graph = (flags & TGDK_MG_EAGER) ? 0 : 1;
    mg->ops.push_back(op);
    int rc = TGDK_OK;
    for (;;) {
        tgdk_op f = mg->ops.back();
        bool can = true;
        for (int a = 0; a < f->dim; ++a) can = can && f->n[a] >= 3 && f->n[a] % 2 == 1;
        if (!can) break;
        tgdk_op c = nullptr;
        if ((rc = tgdk_op_coarsen(f, &c))) break;
        mg->ops.push_back(c);
    }
    for (size_t l = 0; l < mg->ops.size() && !rc; ++l) {
        const size_t n = (size_t)mg->ops[l]->N;
        double* p = nullptr;
        if (hipMalloc((void**)&p, sizeof(double) * n * (l == 0 ? 5 : 3)) != hipSuccess) {
            rc = fail(TGDK_E_NOMEM, "multigrid level allocation failed");
            break;
        }
        mg->z.push_back(p);
        mg->v.push_back(p + n);
        mg->t.push_back(p + 2 * n);
        if (l == 0) {
            mg->acc = p + 3 * n;
            mg->bin = p + 4 * n;
        }
    }
    for (size_t l = 0; l < mg->ops.size() && !rc; ++l) {
        tgdk_op o = mg->ops[l];
        if (o->N > (1LL << 30)) {
            rc = fail(TGDK_E_INVALID, "multigrid grids are limited to 2^30 points");
            break;
        }
        MgLvl L{};
        L.nx = (int)o->n[0];
        L.ny = (int)o->n[1];
        L.nz = o->dim == 3 ? (int)o->n[2] : 1;
        for (int i = 0; i < 2 * o->dim + 1; ++i) L.cc[i] = o->cc[i];
        L.sc = mg->omega / o->cc[0];
        mg->lv.push_back(L);
    }
    if (!rc) {
        MgTail P;
        mg->tail = plan_tail(mg, P);
        if (mg->tail < (int)mg->ops.size()) {
            if (hipMalloc((void**)&mg->tail_dev, sizeof(MgTail)) != hipSuccess)
                rc = fail(TGDK_E_NOMEM, "multigrid tail allocation failed");
            else if (hipMemcpy(mg->tail_dev, &P, sizeof(MgTail), hipMemcpyHostToDevice) != hipSuccess)
                rc = fail(TGDK_E_HIP, "multigrid tail upload failed");
        }
    }
    if (rc) {
        tgdk_mg_destroy(mg);
        return rc;
    }
    *out = mg;
    return TGDK_OK;
}

int tgdk_mg_apply(void* user, const double* in, double* out, int nrhs) {
    tgdk_mg mg = (tgdk_mg)user;
    if (!mg || !in || !out || nrhs < 1) return fail(TGDK_E_INVALID, "bad argument");
    if (in == out) return fail(TGDK_E_INVALID, "in and out must not alias");
    TGDK_HIP(hipSetDevice(mg->ctx->device));
    hipStream_t s = mg->ctx->stream;
    const long long n = mg->ops[0]->N;
    if (mg->use_graph && !mg->exec) {
        int rc = mg_capture(mg);
        if (rc) return rc;
    }
    for (int j = 0; j < nrhs; ++j) {
        TGDK_HIP(hipMemcpyAsync(mg->bin, in + (size_t)j * n, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        if (mg->exec)
            TGDK_HIP(hipGraphLaunch(mg->exec, s));
        else
            mg_body(mg, s);
        TGDK_HIP(hipMemcpyAsync(out + (size_t)j * n, mg->acc, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    }
    TGDK_HIP(hipGetLastError());
    return TGDK_OK;
}

int tgdk_mg_levels(tgdk_mg mg) { return mg ? (int)mg->ops.size() : TGDK_E_INVALID; }

int tgdk_mg_destroy(tgdk_mg mg) {
    if (!mg) return TGDK_OK;
    (void)hipSetDevice(mg->ctx->device);
    (void)hipStreamSynchronize(mg->ctx->stream);
    if (mg->exec) (void)hipGraphExecDestroy(mg->exec);
    if (mg->graph) (void)hipGraphDestroy(mg->graph);
    for (double* p : mg->z) (void)hipFree(p);  // one allocation per level
    if (mg->tail_dev) (void)hipFree(mg->tail_dev);
    for (size_t l = 1; l < mg->ops.size(); ++l) tgdk_op_destroy(mg->ops[l]);
    delete mg;
    return TGDK_OK;
}

}  // extern "C"
