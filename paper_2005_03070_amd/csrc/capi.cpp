// C-ABI entry points: contexts, operators, grid transfer, deflation spaces,
// the adjoint gradient and the tile autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "dense.h"
#include "host.h"

namespace tgdk {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }
int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int DevBuf::ensure(size_t bytes) {
    if (bytes <= cap) return TGDK_OK;
    release();
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        p = nullptr;
        cap = 0;
        return fail(TGDK_E_NOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    cap = bytes;
    return TGDK_OK;
}

void DevBuf::release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
}

DevOp make_devop(const tgdk_op_s* op, int transpose) {
    DevOp d;
    memset(&d, 0, sizeof(d));
    d.dim = op->dim;
    d.nx = op->n[0];
    d.px = op->n[0];  // unpadded; the 3-D step kernel's solve workspace widens it
    d.ny = op->n[1];
    d.nz = op->dim == 3 ? op->n[2] : 1;
    d.n = op->N;
    d.var = op->kind != TGDK_CONST_CD;
    for (int i = 0; i < 7; ++i) d.cc[i] = transpose ? op->ccT[i] : op->cc[i];
    d.coef64 = transpose ? op->coefT64 : op->coef64;
    d.coef32 = transpose ? op->coefT32 : op->coef32;
    d.zero = op->ctx->zero;
    return d;
}

template <class T>
static int dev_alloc(T** p, size_t count) {
    hipError_t e = hipMalloc((void**)p, std::max<size_t>(count, 1) * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(TGDK_E_NOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e));
    }
    return TGDK_OK;
}

// ||M||_1 with M = A (transpose 0) or A^T: the largest absolute row sum of
// M^T.  The stored transposed coefficients are zero outside the domain.
double op_norm1(tgdk_op op, int transpose) {
    const int nc = 2 * op->dim + 1;
    if (op->kind == TGDK_CONST_CD) {
        double s = 0.0;
        for (int i = 0; i < nc; ++i) s += std::fabs(op->cc[i]);
        return s;
    }
    const long long N = op->N;
    std::vector<double> c((size_t)nc * N);
    const double* src = transpose ? op->coef64 : op->coefT64;
    if (hipMemcpy(c.data(), src, c.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) return NAN;
    const int nx = op->n[0], ny = op->n[1], nz = op->dim == 3 ? op->n[2] : 1;
    double best = 0.0;
    for (long long p = 0; p < N; ++p) {
        const int i = (int)(p % nx), j = (int)((p / nx) % ny), l = (int)(p / ((long long)nx * ny));
        const bool in[7] = {true, i > 0, i < nx - 1, j > 0, j < ny - 1, l > 0, l < nz - 1};
        double s = 0.0;
        for (int o = 0; o < nc; ++o)
            if (in[o]) s += std::fabs(c[(size_t)o * N + p]);
        best = std::max(best, s);
    }
    return best;
}

int op_apply_internal(tgdk_op op, int transpose, int dtype, const void* x, void* y, int nrhs) {
    const DevOp d = make_devop(op, transpose);
    hipStream_t s = op->ctx->stream;
    if (dtype == TGDK_F64)
        launch_apply<double>(d, (const double*)x, (double*)y, nrhs, op->tile_id[0], s);
    else
        launch_apply<float>(d, (const float*)x, (float*)y, nrhs, op->tile_id[1], s);
    TGDK_HIP(hipGetLastError());
    return TGDK_OK;
}

// W (n x k) <- W R^{-1} twice, with R from the Cholesky factor of W^T W.
int cholqr2(tgdk_ctx ctx, double* W, long long n, int k) {
    if (k < 1 || k > MAXK) return fail(TGDK_E_INVALID, "deflation spaces hold 1 to 256 vectors");
    hipStream_t s = ctx->stream;
    double* tmp = nullptr;
    double* dY = nullptr;
    double* dG = nullptr;
    int rc = dev_alloc(&tmp, (size_t)n * k);
    if (rc) return rc;
    if ((rc = dev_alloc(&dY, (size_t)k * k))) {
        (void)hipFree(tmp);
        return rc;
    }
    if ((rc = dev_alloc(&dG, (size_t)k * k))) {
        (void)hipFree(tmp);
        (void)hipFree(dY);
        return rc;
    }
    std::vector<double> G((size_t)k * k), Rinv((size_t)k * k), Y((size_t)k * k);
    rc = TGDK_OK;
    for (int pass = 0; pass < 2 && rc == TGDK_OK; ++pass) {
        const size_t need = gram_partial_bytes(n, k, k);
        if ((rc = ctx->partial.ensure(need))) break;
        launch_gram(W, 0, n, k, W, 0, n, k, n, dG, (double*)ctx->partial.p, ctx->counters, s);
        if (hipMemcpyAsync(G.data(), dG, G.size() * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            rc = fail(TGDK_E_HIP, "Gram copy failed");
            break;
        }
        if (cholesky_upper(k, G.data()) != 0) {
            rc = fail(TGDK_E_SINGULAR, "deflation basis is rank deficient (Cholesky of W^T W failed)");
            break;
        }
        upper_inverse(k, G.data(), Rinv.data());
        for (int i = 0; i < k; ++i)
            for (int c = 0; c < k; ++c) Y[(size_t)c * k + i] = Rinv[(size_t)i * k + c];  // column-major
        if (hipMemcpyAsync(dY, Y.data(), Y.size() * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess) {
            rc = fail(TGDK_E_HIP, "upload failed");
            break;
        }
        launch_vmul(W, n, k, dY, k, tmp, n, n, s);
        if (hipMemcpyAsync(W, tmp, (size_t)n * k * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess) {
            rc = fail(TGDK_E_HIP, "copy failed");
            break;
        }
    }
    if (hipStreamSynchronize(s) != hipSuccess && rc == TGDK_OK) rc = fail(TGDK_E_HIP, "cholqr2 failed");
    (void)hipFree(tmp);
    (void)hipFree(dY);
    (void)hipFree(dG);
    return rc;
}

// LU factors, pivots and H^{-1} (column-major, from the LU factors) of d->H,
// uploaded to the device.  On failure nothing is left allocated.
static int defl_factor(tgdk_defl d, const char* singular_msg) {
    const int k = d->k;
    d->LU = d->H;
    d->piv.assign(k, 0);
    if (lu_factor(k, d->LU.data(), d->piv.data()) != 0) return fail(TGDK_E_SINGULAR, singular_msg);
    std::vector<double> hinv((size_t)k * k, 0.0);
    for (int j = 0; j < k; ++j) {
        double* col = hinv.data() + (size_t)j * k;
        col[j] = 1.0;
        lu_solve(k, d->LU.data(), d->piv.data(), col);
    }
    int rc;
    if ((rc = dev_alloc(&d->d_lu, (size_t)k * k)) || (rc = dev_alloc(&d->d_piv, (size_t)k)) ||
        (rc = dev_alloc(&d->d_hinv, (size_t)k * k)) ||
        hipMemcpy(d->d_lu, d->LU.data(), (size_t)k * k * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d->d_piv, d->piv.data(), (size_t)k * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(d->d_hinv, hinv.data(), (size_t)k * k * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        if (d->d_lu) (void)hipFree(d->d_lu);
        if (d->d_piv) (void)hipFree(d->d_piv);
        if (d->d_hinv) (void)hipFree(d->d_hinv);
        d->d_lu = d->d_hinv = nullptr;
        d->d_piv = nullptr;
        return rc ? rc : fail(TGDK_E_HIP, "upload of LU failed");
    }
    return TGDK_OK;
}

int defl_finish(tgdk_op op, int transpose, double* V64, int k, int store, tgdk_defl* out, int projection) {
    tgdk_ctx ctx = op->ctx;
    hipStream_t s = ctx->stream;
    const long long n = op->N;
    float* V32 = nullptr;
    double* AV = nullptr;
    int rc = TGDK_OK;
    if (store == TGDK_F32) {
        if ((rc = dev_alloc(&V32, (size_t)n * k))) return rc;
        launch_to_f32(V64, V32, (long long)n * k, s);
        launch_to_f64(V32, V64, (long long)n * k, s);  // H is formed from the rounded basis
    }
    if ((rc = dev_alloc(&AV, (size_t)n * k))) {
        if (V32) (void)hipFree(V32);
        return rc;
    }
    rc = op_apply_internal(op, transpose, TGDK_F64, V64, AV, k);
    const bool minres = projection == TGDK_PROJ_MINRES;
    float* W32 = nullptr;  // MinRes, float32 storage: the stored A V
    if (!rc && minres && store == TGDK_F32) {
        rc = dev_alloc(&W32, (size_t)n * k);
        if (!rc) {
            launch_to_f32(AV, W32, (long long)n * k, s);
            launch_to_f64(W32, AV, (long long)n * k, s);  // H is formed from the rounded W
        }
    }
    std::vector<double> H((size_t)k * k);
    double* dG = nullptr;
    if (!rc) rc = dev_alloc(&dG, (size_t)k * k);
    if (!rc) rc = ctx->partial.ensure(gram_partial_bytes(n, k, k));
    if (!rc) {
        // Galerkin H = V^T (A V); MinRes H = (A V)^T (A V)
        launch_gram(minres ? AV : V64, 0, n, k, AV, 0, n, k, n, dG, (double*)ctx->partial.p, ctx->counters, s);
        if (hipMemcpyAsync(H.data(), dG, H.size() * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            rc = fail(TGDK_E_HIP, "forming H failed");
    }
    if (dG) (void)hipFree(dG);
    void* W = nullptr;  // the stored left basis (MinRes only)
    if (minres && !rc) {
        W = store == TGDK_F32 ? (void*)W32 : (void*)AV;
        if (store == TGDK_F32) (void)hipFree(AV);
    } else {
        (void)hipFree(AV);
        if (W32) (void)hipFree(W32);
    }
    if (rc) {
        if (V32) (void)hipFree(V32);
        return rc;
    }
    tgdk_defl d = new tgdk_defl_s();
    d->ctx = ctx;
    d->op = op;
    d->transpose = transpose;
    d->k = k;
    d->n = n;
    d->store = store;
    d->projection = minres ? TGDK_PROJ_MINRES : TGDK_PROJ_GALERKIN;
    d->W = W;
    d->H = H;
    d->mvp_build = k;
    if ((rc = defl_factor(d, minres ? "projection matrix H = (AV)^T AV is singular"
                                    : "projection matrix H = V^T A V is singular"))) {
        if (V32) (void)hipFree(V32);
        if (W) (void)hipFree(W);
        delete d;
        return rc;
    }
    if (store == TGDK_F32) {
        d->V = V32;
        (void)hipFree(V64);
    } else {
        d->V = V64;
    }
    *out = d;
    return TGDK_OK;
}

}  // namespace tgdk

using namespace tgdk;

extern "C" {

const char* tgdk_last_error(void) { return tgdk::g_err.c_str(); }

int tgdk_ctx_create(tgdk_ctx* out, int device, void* hip_stream) {
    if (!out) return fail(TGDK_E_INVALID, "out is NULL");
    *out = nullptr;
    int count = 0;
    TGDK_HIP(hipGetDeviceCount(&count));
    if (device < 0 || device >= count) return fail(TGDK_E_INVALID, "no such device");
    TGDK_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    TGDK_HIP(hipGetDeviceProperties(&prop, device));
    tgdk_ctx c = new tgdk_ctx_s();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->num_cus = prop.multiProcessorCount;
    if (hipMalloc((void**)&c->counters, 64 * sizeof(unsigned)) != hipSuccess ||
        hipMemset(c->counters, 0, 64 * sizeof(unsigned)) != hipSuccess ||
        hipMalloc((void**)&c->dscal, 4096 * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&c->zero, 4096) != hipSuccess || hipMemset(c->zero, 0, 4096) != hipSuccess ||
        hipHostMalloc((void**)&c->mirror, sizeof(Mirror) * MIRROR_PREALLOC, hipHostMallocMapped) != hipSuccess) {
        (void)tgdk_ctx_destroy(c);
        return fail(TGDK_E_NOMEM, "context allocation failed");
    }
    c->mirror_cap = MIRROR_PREALLOC;
    // the solve's host-wait events and the no-allocation scratch's address,
    // set up here so that tgdk_solve_noalloc allocates nothing
    for (int i = 0; i < 2; ++i) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            (void)tgdk_ctx_destroy(c);
            return fail(TGDK_E_HIP, "context event creation failed");
        }
        c->events.push_back(e);
    }
    int rc = noalloc_init(device);
    if (rc) {
        (void)tgdk_ctx_destroy(c);
        return rc;
    }
    *out = c;
    return TGDK_OK;
}

int tgdk_ctx_destroy(tgdk_ctx c) {
    if (!c) return TGDK_OK;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->counters) (void)hipFree(c->counters);
    if (c->dscal) (void)hipFree(c->dscal);
    if (c->zero) (void)hipFree(c->zero);
    if (c->mirror) (void)hipHostFree(c->mirror);
    for (auto e : c->events) (void)hipEventDestroy(e);
    for (auto e : c->tevents) (void)hipEventDestroy(e);
    delete c;
    return TGDK_OK;
}

int tgdk_ctx_num_cus(tgdk_ctx c) { return c ? c->num_cus : 0; }

static_assert(TGDK_STEP_NONE == ACT_NONE && TGDK_STEP_A == ACT_A && TGDK_STEP_A0 == ACT_A0 && TGDK_STEP_B == ACT_B && TGDK_STEP_RES == ACT_RES &&
                  TGDK_STEP_REDUCE == ACT_REDUCE && TGDK_STEP_APPLY == ACT_APPLY && TGDK_STEP_FIN == ACT_FIN &&
                  TGDK_STEP_FIN_A0 == ACT_FIN_A0 && TGDK_STEP_APPLYW == ACT_APPLYW && TGDK_STEP_CDOT == ACT_CDOT &&
                  NACT == 11,
              "step action codes");

int tgdk_ctx_time_kernel(tgdk_ctx c, int on) {
    if (!c || on < 0 || on > 2) return fail(TGDK_E_INVALID, "bad argument");
    if (on == 2 && c->tevents.empty()) {
        TGDK_HIP(hipSetDevice(c->device));
        for (int i = 0; i <= NTSLOG; ++i) {
            hipEvent_t e;
            TGDK_HIP(hipEventCreate(&e));
            c->tevents.push_back(e);
        }
    }
    c->time_which = on;
    for (int a = 0; a < NACT; ++a) {
        c->act_ms[a] = 0.0;
        c->act_count[a] = 0;
    }
    return TGDK_OK;
}

int tgdk_ctx_kernel_time(tgdk_ctx c, int action, double* total_ms, long long* launches) {
    if (!c) return fail(TGDK_E_INVALID, "NULL context");
    if (action != TGDK_STEP_ANY && action != TGDK_STEP_ALL && (action < 0 || action >= NACT))
        return fail(TGDK_E_INVALID, "unknown action");
    double ms = 0.0;
    long long cnt = 0;
    for (int a = 0; a < NACT; ++a)
        if (action == TGDK_STEP_ALL || (action == TGDK_STEP_ANY && a > 0) || action == a) {
            ms += c->act_ms[a];
            cnt += c->act_count[a];
        }
    if (total_ms) *total_ms = ms;
    if (launches) *launches = cnt;
    return TGDK_OK;
}

int tgdk_op_create(tgdk_ctx ctx, const tgdk_op_desc* d, tgdk_op* out) {
    if (!ctx || !d || !out) return fail(TGDK_E_INVALID, "NULL argument");
    *out = nullptr;
    if (d->dim != 2 && d->dim != 3) return fail(TGDK_E_INVALID, "dim must be 2 or 3");
    for (int a = 0; a < d->dim; ++a)
        if (d->n[a] < 1) return fail(TGDK_E_INVALID, "grid sizes must be >= 1");
    if (d->kind != TGDK_CONST_CD && d->kind != TGDK_VAR_STENCIL && d->kind != TGDK_DIV_K)
        return fail(TGDK_E_INVALID, "unknown operator kind");
    if (d->kind != TGDK_CONST_CD && !d->coef) return fail(TGDK_E_INVALID, "coef is NULL");
    if (d->kind == TGDK_DIV_K && d->dim != 2) return fail(TGDK_E_INVALID, "DIV_K is 2-D only");
    TGDK_HIP(hipSetDevice(ctx->device));
    tgdk_op op = new tgdk_op_s();
    op->ctx = ctx;
    op->dim = d->dim;
    op->n[0] = d->n[0];
    op->n[1] = d->n[1];
    op->n[2] = d->dim == 3 ? d->n[2] : 1;
    op->N = (long long)op->n[0] * op->n[1] * op->n[2];
    op->kind = d->kind;
    for (int a = 0; a < 3; ++a) op->beta[a] = a < d->dim ? d->beta[a] : 0.0;
    op->sigma = d->sigma;
    const int nc = 2 * d->dim + 1;
    if (d->kind == TGDK_CONST_CD) {
        double C = d->sigma;
        for (int a = 0; a < d->dim; ++a) {
            const double h = 1.0 / (op->n[a] + 1);
            C += 2.0 / (h * h);
            op->cc[1 + 2 * a] = -1.0 / (h * h) - op->beta[a] / (2.0 * h);
            op->cc[2 + 2 * a] = -1.0 / (h * h) + op->beta[a] / (2.0 * h);
        }
        op->cc[0] = C;
        op->ccT[0] = C;
        for (int a = 0; a < d->dim; ++a) {
            op->ccT[1 + 2 * a] = op->cc[2 + 2 * a];
            op->ccT[2 + 2 * a] = op->cc[1 + 2 * a];
        }
        *out = op;
        return TGDK_OK;
    }
    hipStream_t s = ctx->stream;
    const long long N = op->N;
    int rc;
    if ((rc = dev_alloc(&op->coef64, (size_t)nc * N)) || (rc = dev_alloc(&op->coefT64, (size_t)nc * N)) ||
        (rc = dev_alloc(&op->coef32, (size_t)nc * N)) || (rc = dev_alloc(&op->coefT32, (size_t)nc * N))) {
        tgdk_op_destroy(op);
        return rc;
    }
    if (d->kind == TGDK_VAR_STENCIL) {
        if (hipMemcpyAsync(op->coef64, d->coef, (size_t)nc * N * sizeof(double), hipMemcpyDeviceToDevice, s) !=
            hipSuccess) {
            tgdk_op_destroy(op);
            return fail(TGDK_E_HIP, "copy of coefficients failed");
        }
    } else {
        const size_t ncell = (size_t)(op->n[0] + 1) * (op->n[1] + 1);
        if ((rc = dev_alloc(&op->kcell, ncell))) {
            tgdk_op_destroy(op);
            return rc;
        }
        if (hipMemcpyAsync(op->kcell, d->coef, ncell * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess) {
            tgdk_op_destroy(op);
            return fail(TGDK_E_HIP, "copy of k failed");
        }
        launch_build_divk(op->n[0], op->n[1], op->kcell, op->beta[0], op->beta[1], op->sigma, op->coef64, s);
    }
    launch_transpose_coef(op->dim, op->n[0], op->n[1], op->n[2], op->coef64, op->coefT64, s);
    launch_to_f32(op->coef64, op->coef32, (long long)nc * N, s);
    launch_to_f32(op->coefT64, op->coefT32, (long long)nc * N, s);
    if (hipStreamSynchronize(s) != hipSuccess || hipGetLastError() != hipSuccess) {
        tgdk_op_destroy(op);
        return fail(TGDK_E_HIP, "operator construction failed");
    }
    *out = op;
    return TGDK_OK;
}

int tgdk_op_coarsen(tgdk_op fine, tgdk_op* coarse) {
    if (!fine || !coarse) return fail(TGDK_E_INVALID, "NULL argument");
    if (fine->kind == TGDK_VAR_STENCIL) return fail(TGDK_E_INVALID, "VAR_STENCIL operators cannot be coarsened");
    tgdk_op_desc d;
    memset(&d, 0, sizeof(d));
    d.dim = fine->dim;
    for (int a = 0; a < fine->dim; ++a) {
        if (fine->n[a] < 3 || fine->n[a] % 2 == 0) return fail(TGDK_E_INVALID, "fine sizes must be odd and >= 3");
        d.n[a] = (fine->n[a] - 1) / 2;
        d.beta[a] = fine->beta[a];
    }
    d.kind = fine->kind;
    d.sigma = fine->sigma;
    if (fine->kind == TGDK_CONST_CD) return tgdk_op_create(fine->ctx, &d, coarse);
    double* kc = nullptr;
    const size_t ncell = (size_t)(d.n[0] + 1) * (d.n[1] + 1);
    int rc = dev_alloc(&kc, ncell);
    if (rc) return rc;
    launch_coarsen_kcell(d.n[0], d.n[1], fine->kcell, kc, fine->ctx->stream);
    d.coef = kc;
    rc = tgdk_op_create(fine->ctx, &d, coarse);
    (void)hipStreamSynchronize(fine->ctx->stream);
    (void)hipFree(kc);
    return rc;
}

int tgdk_op_apply(tgdk_op op, int transpose, int dtype, const void* x, void* y, int nrhs) {
    if (!op || !x || !y || nrhs < 1) return fail(TGDK_E_INVALID, "bad argument");
    if (dtype != TGDK_F64 && dtype != TGDK_F32) return fail(TGDK_E_INVALID, "dtype");
    TGDK_HIP(hipSetDevice(op->ctx->device));
    return op_apply_internal(op, transpose ? 1 : 0, dtype, x, y, nrhs);
}

int tgdk_op_info(tgdk_op op, int* dim, int* n_per_axis, long long* n) {
    if (!op) return fail(TGDK_E_INVALID, "NULL op");
    if (dim) *dim = op->dim;
    if (n_per_axis)
        for (int a = 0; a < 3; ++a) n_per_axis[a] = op->n[a];
    if (n) *n = op->N;
    return TGDK_OK;
}

int tgdk_op_destroy(tgdk_op op) {
    if (!op) return TGDK_OK;
    (void)hipSetDevice(op->ctx->device);
    if (op->coef64) (void)hipFree(op->coef64);
    if (op->coef32) (void)hipFree(op->coef32);
    if (op->coefT64) (void)hipFree(op->coefT64);
    if (op->coefT32) (void)hipFree(op->coefT32);
    if (op->kcell) (void)hipFree(op->kcell);
    delete op;
    return TGDK_OK;
}

static int check_nested(tgdk_op coarse, tgdk_op fine) {
    if (!coarse || !fine) return fail(TGDK_E_INVALID, "NULL operator");
    if (coarse->dim != fine->dim) return fail(TGDK_E_INVALID, "dimension mismatch");
    for (int a = 0; a < fine->dim; ++a)
        if (fine->n[a] != 2 * coarse->n[a] + 1) return fail(TGDK_E_INVALID, "grids are not nested (n_f = 2 n_c + 1)");
    return TGDK_OK;
}

int tgdk_prolongate(tgdk_op coarse, tgdk_op fine, int dtype, const void* vc, void* vf, int ncols) {
    int rc = check_nested(coarse, fine);
    if (rc) return rc;
    if (dtype != TGDK_F64 || !vc || !vf || ncols < 1) return fail(TGDK_E_INVALID, "bad argument");
    TGDK_HIP(hipSetDevice(fine->ctx->device));
    launch_prolong(fine->dim, coarse->n[0], coarse->n[1], fine->dim == 3 ? coarse->n[2] : 1, (const double*)vc,
                   (double*)vf, ncols, fine->ctx->stream);
    TGDK_HIP(hipGetLastError());
    return TGDK_OK;
}

int tgdk_restrict(tgdk_op fine, tgdk_op coarse, int dtype, const void* vf, void* vc, int ncols) {
    int rc = check_nested(coarse, fine);
    if (rc) return rc;
    if (dtype != TGDK_F64 || !vc || !vf || ncols < 1) return fail(TGDK_E_INVALID, "bad argument");
    TGDK_HIP(hipSetDevice(fine->ctx->device));
    launch_restrict(fine->dim, coarse->n[0], coarse->n[1], fine->dim == 3 ? coarse->n[2] : 1, (const double*)vf,
                    (double*)vc, ncols, fine->ctx->stream);
    TGDK_HIP(hipGetLastError());
    return TGDK_OK;
}

int tgdk_defl_prolongate(tgdk_defl cs, tgdk_op fine, int store_dtype, tgdk_defl* out) {
    if (!cs || !fine || !out) return fail(TGDK_E_INVALID, "NULL argument");
    if (store_dtype != TGDK_F64 && store_dtype != TGDK_F32) return fail(TGDK_E_INVALID, "store dtype");
    if (cs->store != TGDK_F64) return fail(TGDK_E_INVALID, "coarse space must be stored in float64");
    int rc = check_nested(cs->op, fine);
    if (rc) return rc;
    TGDK_HIP(hipSetDevice(fine->ctx->device));
    const int k = cs->k;
    double* PW = nullptr;
    if ((rc = dev_alloc(&PW, (size_t)fine->N * k))) return rc;
    tgdk_op c = cs->op;
    launch_prolong(fine->dim, c->n[0], c->n[1], fine->dim == 3 ? c->n[2] : 1, (const double*)cs->V, PW, k,
                   fine->ctx->stream);
    if ((rc = cholqr2(fine->ctx, PW, fine->N, k))) {
        (void)hipFree(PW);
        return rc;
    }
    rc = defl_finish(fine, cs->transpose, PW, k, store_dtype, out, TGDK_PROJ_GALERKIN);
    if (rc) (void)hipFree(PW);
    return rc;
}

int tgdk_defl_from_basis(tgdk_op op, const double* W, int k, int transpose, int store_dtype, tgdk_defl* out) {
    if (!op || !W || !out || k < 1) return fail(TGDK_E_INVALID, "bad argument");
    if (store_dtype != TGDK_F64 && store_dtype != TGDK_F32) return fail(TGDK_E_INVALID, "store dtype");
    TGDK_HIP(hipSetDevice(op->ctx->device));
    double* V = nullptr;
    int rc = dev_alloc(&V, (size_t)op->N * k);
    if (rc) return rc;
    TGDK_HIP(hipMemcpyAsync(V, W, (size_t)op->N * k * sizeof(double), hipMemcpyDeviceToDevice, op->ctx->stream));
    if ((rc = cholqr2(op->ctx, V, op->N, k))) {
        (void)hipFree(V);
        return rc;
    }
    rc = defl_finish(op, transpose ? 1 : 0, V, k, store_dtype, out, TGDK_PROJ_GALERKIN);
    if (rc) (void)hipFree(V);
    return rc;
}

int tgdk_defl_minres(tgdk_defl g, tgdk_defl* out) {
    if (!g || !out) return fail(TGDK_E_INVALID, "NULL argument");
    if (g->precond) return fail(TGDK_E_INVALID, "a preconditioned space has no MinRes variant");
    TGDK_HIP(hipSetDevice(g->ctx->device));
    double* V = nullptr;
    int rc = dev_alloc(&V, (size_t)g->n * g->k);
    if (rc) return rc;
    if (g->store == TGDK_F64)
        TGDK_HIP(hipMemcpyAsync(V, g->V, (size_t)g->n * g->k * sizeof(double), hipMemcpyDeviceToDevice,
                                g->ctx->stream));
    else
        launch_to_f64((const float*)g->V, V, (long long)g->n * g->k, g->ctx->stream);
    rc = defl_finish(g->op, g->transpose, V, g->k, g->store, out, TGDK_PROJ_MINRES);
    if (rc) (void)hipFree(V);
    return rc;
}

int tgdk_defl_projection(tgdk_defl d) { return d ? d->projection : TGDK_E_INVALID; }

int tgdk_defl_precond(tgdk_defl g, tgdk_precond_fn fn, void* user, tgdk_defl* out) {
    if (!g || !fn || !out) return fail(TGDK_E_INVALID, "NULL argument");
    if (g->store != TGDK_F64 || g->W || g->precond)
        return fail(TGDK_E_INVALID, "a preconditioned space is built from a float64 Galerkin space");
    tgdk_ctx ctx = g->ctx;
    TGDK_HIP(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const long long n = g->n;
    const int k = g->k;
    double *V = nullptr, *Z = nullptr, *AZ = nullptr, *dG = nullptr;
    int rc;
    auto release = [&]() {
        if (V) (void)hipFree(V);
        if (Z) (void)hipFree(Z);
        if (AZ) (void)hipFree(AZ);
        if (dG) (void)hipFree(dG);
    };
    if ((rc = dev_alloc(&V, (size_t)n * k)) || (rc = dev_alloc(&Z, (size_t)n * k)) ||
        (rc = dev_alloc(&AZ, (size_t)n * k)) || (rc = dev_alloc(&dG, (size_t)k * k))) {
        release();
        return rc;
    }
    TGDK_HIP(hipMemcpyAsync(V, g->V, sizeof(double) * n * k, hipMemcpyDeviceToDevice, s));
    // Z = M^{-1} V, then H = V^T (A Z)
    if ((rc = fn(user, V, Z, k)) || (rc = op_apply_internal(g->op, g->transpose, TGDK_F64, Z, AZ, k)) ||
        (rc = ctx->partial.ensure(gram_partial_bytes(n, k, k)))) {
        release();
        return rc < 0 ? rc : fail(TGDK_E_HIP, "preconditioner failed");
    }
    std::vector<double> H((size_t)k * k);
    launch_gram(V, 0, n, k, AZ, 0, n, k, n, dG, (double*)ctx->partial.p, ctx->counters, s);
    if (hipMemcpyAsync(H.data(), dG, H.size() * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        release();
        return fail(TGDK_E_HIP, "forming H failed");
    }
    (void)hipFree(AZ);
    (void)hipFree(dG);
    AZ = dG = nullptr;
    tgdk_defl d = new tgdk_defl_s();
    d->ctx = ctx;
    d->op = g->op;
    d->transpose = g->transpose;
    d->k = k;
    d->n = n;
    d->store = TGDK_F64;
    d->projection = TGDK_PROJ_GALERKIN;
    d->precond = 1;
    d->V = Z;  // update basis
    d->W = V;  // basis of c = V^T r
    d->H = H;
    d->mvp_build = k;  // A Z (plus k applications of the preconditioner)
    if ((rc = defl_factor(d, "projection matrix H = V^T A M^{-1} V is singular"))) {
        delete d;
        release();
        return rc;
    }
    *out = d;
    return TGDK_OK;
}

int tgdk_defl_info(tgdk_defl d, int* k, int* store, long long* n) {
    if (!d) return fail(TGDK_E_INVALID, "NULL space");
    if (k) *k = d->k;
    if (store) *store = d->store;
    if (n) *n = d->n;
    return TGDK_OK;
}

int tgdk_defl_copy(tgdk_defl d, double* V_out, double* H_out) {
    if (!d) return fail(TGDK_E_INVALID, "NULL space");
    TGDK_HIP(hipSetDevice(d->ctx->device));
    if (V_out) {
        if (d->store == TGDK_F64)
            TGDK_HIP(hipMemcpyAsync(V_out, d->precond ? d->W : d->V, (size_t)d->n * d->k * sizeof(double),
                                    hipMemcpyDeviceToDevice, d->ctx->stream));
        else
            launch_to_f64((const float*)d->V, V_out, (long long)d->n * d->k, d->ctx->stream);
        TGDK_HIP(hipStreamSynchronize(d->ctx->stream));
    }
    if (H_out) memcpy(H_out, d->H.data(), d->H.size() * sizeof(double));
    return TGDK_OK;
}

int tgdk_defl_destroy(tgdk_defl d) {
    if (!d) return TGDK_OK;
    (void)hipSetDevice(d->ctx->device);
    if (d->V) (void)hipFree(d->V);
    if (d->W) (void)hipFree(d->W);
    if (d->d_lu) (void)hipFree(d->d_lu);
    if (d->d_piv) (void)hipFree(d->d_piv);
    if (d->d_hinv) (void)hipFree(d->d_hinv);
    delete d;
    return TGDK_OK;
}

int tgdk_adjoint_grad_k(tgdk_op op, const double* lambda, const double* u, double* grad_k) {
    if (!op || !lambda || !u || !grad_k) return fail(TGDK_E_INVALID, "NULL argument");
    if (op->kind != TGDK_DIV_K || op->dim != 2) return fail(TGDK_E_INVALID, "operator must be 2-D DIV_K");
    TGDK_HIP(hipSetDevice(op->ctx->device));
    launch_grad_k(op->n[0], op->n[1], lambda, u, grad_k, op->ctx->stream);
    TGDK_HIP(hipGetLastError());
    return TGDK_OK;
}

int tgdk_tune(tgdk_ctx ctx, tgdk_op op, int dtype, int nrhs, int* tile_y) {
    if (!op || nrhs < 1 || (dtype != TGDK_F64 && dtype != TGDK_F32)) return fail(TGDK_E_INVALID, "bad argument");
    if (ctx && ctx != op->ctx) return fail(TGDK_E_INVALID, "the operator belongs to another context");
    TGDK_HIP(hipSetDevice(op->ctx->device));
    const char* cache = getenv("TGDK_TUNE_CACHE");
    char key[160];
    snprintf(key, sizeof(key), "gfx950 dim=%d n=%d,%d,%d dtype=%d nrhs=%d", op->dim, op->n[0], op->n[1], op->n[2],
             dtype, nrhs);
    if (cache) {
        FILE* f = fopen(cache, "r");
        if (f) {
            char line[256];
            while (fgets(line, sizeof(line), f)) {
                int id;
                const size_t kl = strlen(key);
                if (strncmp(line, key, kl) == 0 && sscanf(line + kl, " tile=%d", &id) == 1 && id >= 0 && id < NTILE_IDS) {
                    op->tile_id[dtype] = id;
                    fclose(f);
                    if (tile_y) {
                        int ty, tz;
                        tile_shape(op->dim, id, &ty, &tz);
                        *tile_y = ty;
                    }
                    return TGDK_OK;
                }
            }
            fclose(f);
        }
    }
    const size_t es = dtype == TGDK_F64 ? 8 : 4;
    const size_t bytes = (size_t)op->N * nrhs * es;
    void* x = nullptr;
    void* y = nullptr;
    TGDK_HIP(hipMalloc(&x, bytes));
    if (hipMalloc(&y, bytes) != hipSuccess) {
        (void)hipFree(x);
        return fail(TGDK_E_NOMEM, "tune buffers");
    }
    (void)hipMemsetAsync(x, 0, bytes, op->ctx->stream);
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    float best = 1e30f;
    int best_id = 0;
    for (int id = 0; id < NTILE_IDS; ++id) {
        op->tile_id[dtype] = id;
        for (int w = 0; w < 3; ++w) op_apply_internal(op, 0, dtype, x, y, nrhs);
        (void)hipEventRecord(e0, op->ctx->stream);
        const int reps = 20;
        for (int r = 0; r < reps; ++r) op_apply_internal(op, 0, dtype, x, y, nrhs);
        (void)hipEventRecord(e1, op->ctx->stream);
        (void)hipEventSynchronize(e1);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) {
            best = ms;
            best_id = id;
        }
    }
    op->tile_id[dtype] = best_id;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(x);
    (void)hipFree(y);
    if (cache) {
        FILE* f = fopen(cache, "a");
        if (f) {
            fprintf(f, "%s tile=%d\n", key, best_id);
            fclose(f);
        }
    }
    if (tile_y) {
        int ty, tz;
        tile_shape(op->dim, best_id, &ty, &tz);
        *tile_y = ty;
    }
    return TGDK_OK;
}

}  // extern "C"
