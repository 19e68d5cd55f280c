// Internal host-side definitions of the tgdk handles.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/tgdk.h"
#include "launch.h"
#include "tgdk_shared.h"

namespace tgdk {

void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

#define TGDK_HIP(call)                                                                       \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return ::tgdk::fail(TGDK_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Device buffer that grows on demand (contents not preserved on growth).
struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    int ensure(size_t bytes);
    void release();
    ~DevBuf() { release(); }
};

}  // namespace tgdk

struct tgdk_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    int num_cus = 0;
    // scratch for the dense and Gram-Schmidt kernels
    tgdk::DevBuf partial;      // doubles
    unsigned* counters = nullptr;  // 64 zero-initialised counters
    double* dscal = nullptr;   // small device scalar area (4096 doubles)
    void* zero = nullptr;      // 4 KiB of zeros, never written
    // solve workspace (grow-only, reused across calls)
    tgdk::DevBuf solve_ws;
    tgdk::Mirror* mirror = nullptr;  // host-mapped
    int mirror_cap = 0;
    std::vector<hipEvent_t> events;
    // step-kernel timing for measurement: 0 off, 1 device-clock stamps,
    // 2 a HIP timing event after every step launch (tevents)
    int time_which = 0;
    std::vector<hipEvent_t> tevents;
    double act_ms[tgdk::NACT] = {0};          // summed duration per action of the first problem
    long long act_count[tgdk::NACT] = {0};
};

struct tgdk_op_s {
    tgdk_ctx ctx = nullptr;
    int dim = 2;
    int n[3] = {1, 1, 1};
    long long N = 0;
    int kind = TGDK_CONST_CD;
    double beta[3] = {0, 0, 0};
    double sigma = 0;
    double cc[7] = {0}, ccT[7] = {0};
    double* coef64 = nullptr;
    float* coef32 = nullptr;
    double* coefT64 = nullptr;
    float* coefT32 = nullptr;
    double* kcell = nullptr;   // DIV_K
    int tile_id[2] = {0, 0};   // per element type (0 f64, 1 f32)
};

struct tgdk_defl_s {
    tgdk_ctx ctx = nullptr;
    tgdk_op op = nullptr;
    int transpose = 0;
    int k = 0;
    long long n = 0;
    int store = TGDK_F64;
    void* V = nullptr;         // n x k column-major (ldv = n)
    int projection = TGDK_PROJ_GALERKIN;
    void* W = nullptr;         // left basis of c when it differs from V: MinRes A V (or A^T V);
                               // preconditioned: the orthonormal basis (V then holds Z = M^{-1} V)
    int precond = 0;           // built by tgdk_defl_precond
    std::vector<double> H, LU;
    std::vector<int> piv;
    double* d_lu = nullptr;
    int* d_piv = nullptr;
    double* d_hinv = nullptr;  // H^{-1}, column-major
    long long mvp_build = 0;   // fine-grid operator applications spent building it (A V for H)
};

namespace tgdk {

DevOp make_devop(const tgdk_op_s* op, int transpose);
double op_norm1(tgdk_op op, int transpose);
// Builds H = V^T A V (Galerkin) or (AV)^T AV with W = A V kept (MinRes) from V
// (float64 device, n x k, owned by the handle on success), its LU, and the handle.
int defl_finish(tgdk_op op, int transpose, double* V64, int k, int store, tgdk_defl* out, int projection);
// Orthonormalise W (n x k, device float64) in place by CholQR2.
int cholqr2(tgdk_ctx ctx, double* W, long long n, int k);
int op_apply_internal(tgdk_op op, int transpose, int dtype, const void* x, void* y, int nrhs);
// BiCGStab(ncyc)-Proj(k) with its workspace laid out in [base, base + cap)
// (no allocation; solve.cpp).
int solve_bicgstab_in(tgdk_op fine, tgdk_defl defl, const double* b, double* x, int nrhs,
                      const tgdk_solve_params* prm, tgdk_solve_report* reports, void* base, size_t cap);
// Address of the no-allocation scratch on the current device (taken once
// per device; solve_noalloc.hip).  Called by tgdk_ctx_create.
int noalloc_init(int device);
// Systems a context's preallocated status mirror holds (the no-allocation
// solve takes at most this many right-hand sides).
constexpr int MIRROR_PREALLOC = 64;

}  // namespace tgdk
