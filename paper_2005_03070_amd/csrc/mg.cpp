// Geometric multigrid V-cycles for a constant-coefficient operator: the
// preconditioner of Sec. 5, Example 5 (solutions with the positively shifted
// Laplacian precondition the Helmholtz operator).  Levels are the operator's
// grid and its rediscretised nested coarse grids down to sides of 1; damped
// Jacobi smoothing (omega 4/5 in 2-D, 6/7 in 3-D) around a full-weighting /
// linear-interpolation coarse correction; 20 sweeps on the coarsest grid.
// The host walks the levels and enqueues the grid kernels; the
// preconditioner is a fixed number of V-cycles from zero, a fixed linear
// operator.  That kernel sequence (about 150 small launches per V-cycle on a
// 511^2 grid, latency-bound) is captured once into a HIP graph on a private
// stream and replayed on the context's stream; the caller's vectors are
// copied in and out around it, so the graph only touches the object's own
// buffers.
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "host.h"

struct tgdk_mg_s {
    tgdk_ctx ctx = nullptr;
    std::vector<tgdk_op> ops;       // level 0: the caller's operator (not owned)
    std::vector<double*> z, v, t;   // per level; t: A z, residual, prolongation scratch
    double* acc = nullptr;          // level 0: the accumulated solution
    double* bin = nullptr;          // level 0: the right-hand side, copied in
    int cycles = 2, nu = 2;
    double omega = 0.8;
    int use_graph = 1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace tgdk {

constexpr int MG_COARSEST_SWEEPS = 20;

// One V-cycle for A_l z_l = vin (vin: v_l, or the input on level 0).
static void vcycle(tgdk_mg mg, int l, const double* vin, hipStream_t s) {
    tgdk_op op = mg->ops[l];
    const DevOp d = make_devop(op, 0);
    const long long n = op->N;
    const double sc = mg->omega / op->cc[0];
    double *z = mg->z[l], *t = mg->t[l];
    const double* v = vin;
    auto sweeps = [&](int count, bool from_zero) {
        for (int i = 0; i < count; ++i) {
            if (from_zero && i == 0) {
                launch_jacobi(z, v, nullptr, sc, n, 1, s);
            } else {
                launch_apply<double>(d, z, t, 1, op->tile_id[0], s);
                launch_jacobi(z, v, t, sc, n, 0, s);
            }
        }
    };
    if (l + 1 == (int)mg->ops.size()) {
        sweeps(MG_COARSEST_SWEEPS, true);
        return;
    }
    tgdk_op c = mg->ops[l + 1];
    const int cz = op->dim == 3 ? c->n[2] : 1;
    sweeps(mg->nu, true);
    launch_apply<double>(d, z, t, 1, op->tile_id[0], s);
    launch_sub(v, t, t, n, s);
    launch_restrict(op->dim, c->n[0], c->n[1], cz, t, mg->v[l + 1], 1, s);
    vcycle(mg, l + 1, mg->v[l + 1], s);
    launch_prolong(op->dim, c->n[0], c->n[1], cz, mg->z[l + 1], t, 1, s);
    launch_add(z, t, n, s);
    sweeps(mg->nu, false);
}

// The whole preconditioner on bin -> acc: z_1 = V(b), z_(c+1) = z_c + V(b - A z_c).
static void mg_body(tgdk_mg mg, hipStream_t s) {
    tgdk_op op = mg->ops[0];
    const DevOp d = make_devop(op, 0);
    const long long n = op->N;
    vcycle(mg, 0, mg->bin, s);
    launch_copy(mg->z[0], mg->acc, n, s);
    for (int c = 1; c < mg->cycles; ++c) {
        launch_apply<double>(d, mg->acc, mg->t[0], 1, op->tile_id[0], s);
        launch_sub(mg->bin, mg->t[0], mg->v[0], n, s);
        vcycle(mg, 0, mg->v[0], s);
        launch_add(mg->acc, mg->z[0], n, s);
    }
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
    for (size_t l = 1; l < mg->ops.size(); ++l) tgdk_op_destroy(mg->ops[l]);
    delete mg;
    return TGDK_OK;
}

}  // extern "C"
