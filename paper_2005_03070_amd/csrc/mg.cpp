// Geometric multigrid V-cycles for a constant-coefficient operator: the
// preconditioner of Sec. 5, Example 5 (solutions with the positively shifted
// Laplacian precondition the Helmholtz operator).  Levels are the operator's
// grid and its rediscretised nested coarse grids down to sides of 1; damped
// Jacobi smoothing (omega 4/5 in 2-D, 6/7 in 3-D) around a full-weighting /
// linear-interpolation coarse correction; 20 sweeps on the coarsest grid.
// The host walks the levels and enqueues the grid kernels on the context's
// stream; the preconditioner is a fixed number of V-cycles from zero, a fixed
// linear operator.
#include <hip/hip_runtime.h>

#include <vector>

#include "host.h"

struct tgdk_mg_s {
    tgdk_ctx ctx = nullptr;
    std::vector<tgdk_op> ops;       // level 0: the caller's operator (not owned)
    std::vector<double*> z, v, t;   // per level; t: A z, residual, prolongation scratch
    double* acc = nullptr;          // level 0: the accumulated solution
    int cycles = 2, nu = 2;
    double omega = 0.8;
};

namespace tgdk {

constexpr int MG_COARSEST_SWEEPS = 20;

static void vcycle(tgdk_mg mg, int l) {
    tgdk_op op = mg->ops[l];
    hipStream_t s = mg->ctx->stream;
    const DevOp d = make_devop(op, 0);
    const long long n = op->N;
    const double sc = mg->omega / op->cc[0];
    double *z = mg->z[l], *v = mg->v[l], *t = mg->t[l];
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
    vcycle(mg, l + 1);
    launch_prolong(op->dim, c->n[0], c->n[1], cz, mg->z[l + 1], t, 1, s);
    launch_add(z, t, n, s);
    sweeps(mg->nu, false);
}

}  // namespace tgdk

using namespace tgdk;

extern "C" {

int tgdk_mg_create(tgdk_op op, int cycles, int nu, tgdk_mg* out) {
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
        if (hipMalloc((void**)&p, sizeof(double) * n * (l == 0 ? 4 : 3)) != hipSuccess) {
            rc = fail(TGDK_E_NOMEM, "multigrid level allocation failed");
            break;
        }
        mg->z.push_back(p);
        mg->v.push_back(p + n);
        mg->t.push_back(p + 2 * n);
        if (l == 0) mg->acc = p + 3 * n;
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
    tgdk_op op = mg->ops[0];
    const DevOp d = make_devop(op, 0);
    const long long n = op->N;
    for (int j = 0; j < nrhs; ++j) {
        const double* b = in + (size_t)j * n;
        // z_1 = V(b); z_(c+1) = z_c + V(b - A z_c)
        TGDK_HIP(hipMemcpyAsync(mg->v[0], b, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        vcycle(mg, 0);
        TGDK_HIP(hipMemcpyAsync(mg->acc, mg->z[0], sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        for (int c = 1; c < mg->cycles; ++c) {
            launch_apply<double>(d, mg->acc, mg->t[0], 1, op->tile_id[0], s);
            launch_sub(b, mg->t[0], mg->v[0], n, s);
            vcycle(mg, 0);
            launch_add(mg->acc, mg->z[0], n, s);
        }
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
    for (double* p : mg->z) (void)hipFree(p);  // one allocation per level
    for (size_t l = 1; l < mg->ops.size(); ++l) tgdk_op_destroy(mg->ops[l]);
    delete mg;
    return TGDK_OK;
}

}  // extern "C"
