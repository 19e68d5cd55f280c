// The no-allocation variant of the BiCGStab(ncyc)-Proj(k) fine solve.
//
// tgdk_solve keeps its workspace (group descriptors, solver states, the
// float64 residual and the inner vectors of every system, the step kernel's
// partial sums) in a grow-only device buffer of the context, allocated on
// first use.  Callers that cannot allocate device memory inside the solve
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc) call tgdk_solve_noalloc instead: the same kernels and the same
// launches, with that workspace laid out in one fixed array per device.
//
// The array is a file-scope __device__ variable.  Its name in host code is a
// host-side stand-in, not a device address, so its address is taken once per
// device with hipGetSymbolAddress (at tgdk_ctx_create, with that device
// current) and only that address is handed to the kernels and to
// hipMemsetAsync.  Everything else the solve touches is set up at context
// creation too: the host-mapped status mirror (up to MIRROR_PREALLOC systems)
// and the host-wait events.
#include <hip/hip_runtime.h>

#include <mutex>

#include "host.h"

namespace tgdk {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static_assert(NOALLOC_SCRATCH_BYTES == (size_t)TGDK_NOALLOC_SCRATCH_MB << 20, "scratch size in include/tgdk.h");
constexpr int NOALLOC_MAX_DEVICES = 64;

// the scratch: one copy per GPU the library runs on, held until the process ends
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

static void* scratch_addr[NOALLOC_MAX_DEVICES];
static std::mutex scratch_mutex;

int noalloc_init(int device) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return fail(TGDK_E_INVALID, "device index out of range");
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (scratch_addr[device]) return TGDK_OK;
    int cur = -1;
    TGDK_HIP(hipGetDevice(&cur));
    if (cur != device) return fail(TGDK_E_INVALID, "the device must be current when its scratch is set up");
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(TGDK_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    scratch_addr[device] = p;
    return TGDK_OK;
}

}  // namespace tgdk

using namespace tgdk;

extern "C" int tgdk_solve_noalloc(tgdk_op fine, tgdk_defl defl, const double* b, double* x, int nrhs,
                                  const tgdk_solve_params* params, tgdk_solve_report* reports) {
    if (!fine) return fail(TGDK_E_INVALID, "bad argument");
    const int dev = fine->ctx->device;
    void* p = nullptr;
    {
        std::lock_guard<std::mutex> lock(scratch_mutex);
        if (dev >= 0 && dev < NOALLOC_MAX_DEVICES) p = scratch_addr[dev];
    }
    if (!p) return fail(TGDK_E_INVALID, "the device's scratch was not set up (create a context on it first)");
    if (nrhs > MIRROR_PREALLOC) return fail(TGDK_E_INVALID, "at most 64 right-hand sides without allocation");
    return solve_bicgstab_in(fine, defl, b, x, nrhs, params, reports, p, NOALLOC_SCRATCH_BYTES);
}
