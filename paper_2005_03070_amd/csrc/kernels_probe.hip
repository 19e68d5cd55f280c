// Streaming ceilings for the roofline: what a plain kernel with the same
// number of read and write streams as a step-kernel phase moves per second,
// in two access orders.  Measurement only; not a step of the method.
//
//  contiguous: each stream is one array walked grid-strided, one float64 a
//              lane, four rows of the workgroup in flight (the order of a
//              copy kernel);
//  march:      the arrays are 3-D grids n_x x n_y x n_z with row pitch px and
//              each workgroup walks a chunk of 64 x 8 columns plane by plane,
//              two points a thread, as the 3-D step kernel's z-marching
//              phases do (no LDS and no stencil: the access order alone).
//
// Every stream holds float64 values; a point's reads are summed and the sum
// times (w + 1) is written to write stream w, so no load is dead.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "device_common.h"
#include "host.h"

namespace tgdk {

namespace {

constexpr int PROBE_MAX_STREAMS = 12;

struct ProbeArgs {
    const double* in[PROBE_MAX_STREAMS];
    double* out[PROBE_MAX_STREAMS];
};

template <int NR, int NW>
__global__ __launch_bounds__(NT) void k_probe_contiguous(ProbeArgs a, long long n) {
    constexpr int U = 4;
    const long long stride = (long long)gridDim.x * NT * U;
    for (long long i0 = (long long)blockIdx.x * NT * U + threadIdx.x; i0 < n; i0 += stride) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = 0.0;
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const long long i = i0 + u * NT;
                if (i < n) v[u] += a.in[r][i];
            }
#pragma unroll
        for (int w = 0; w < NW; ++w)
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const long long i = i0 + u * NT;
                if (i < n) a.out[w][i] = v[u] * (double)(w + 1);
            }
    }
}

template <int NR, int NW>
__global__ __launch_bounds__(NT) void k_probe_march(ProbeArgs a, int nx, int ny, int nz, int px, int mz) {
    constexpr int TX = 64, TY = 8, PPT = TX * TY / NT;
    const int cx = (nx + TX - 1) / TX, cy = (ny + TY - 1) / TY;
    const int c = blockIdx.x;
    const int x0 = (c % cx) * TX, y0 = ((c / cx) % cy) * TY, z0 = (c / (cx * cy)) * mz;
    const int z1 = min(z0 + mz, nz);
    const long long pplane = (long long)px * ny;
    long long off[PPT];
    bool ok[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int l = threadIdx.x + q * NT;
        const int gx = x0 + l % TX, gy = y0 + l / TX;
        ok[q] = gx < nx && gy < ny;
        off[q] = (long long)gy * px + gx;
    }
#pragma unroll 4
    for (int z = z0; z < z1; ++z) {
#pragma unroll
        for (int q = 0; q < PPT; ++q) {
            if (!ok[q]) continue;
            const long long g = z * pplane + off[q];
            double v = 0.0;
#pragma unroll
            for (int r = 0; r < NR; ++r) v += a.in[r][g];
#pragma unroll
            for (int w = 0; w < NW; ++w) a.out[w][g] = v * (double)(w + 1);
        }
    }
}

template <int NR, int NW>
void launch_probe(int pattern, const ProbeArgs& a, const int* dims, int px, long long n, int blocks, int mz,
                  hipStream_t s) {
    if (pattern == 0)
        hipLaunchKernelGGL((k_probe_contiguous<NR, NW>), dim3(blocks), dim3(NT), 0, s, a, n);
    else
        hipLaunchKernelGGL((k_probe_march<NR, NW>), dim3(blocks), dim3(NT), 0, s, a, dims[0], dims[1], dims[2],
                           px, mz);
}

}  // namespace

}  // namespace tgdk

using namespace tgdk;

extern "C" int tgdk_stream_probe(tgdk_ctx ctx, int pattern, int nreads, int nwrites, const int* dims, int blocks,
                                 int reps, double* ms_per_launch) {
    if (!ctx || !dims || !ms_per_launch || reps < 1 || (pattern != 0 && pattern != 1))
        return fail(TGDK_E_INVALID, "bad argument");
    if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1) return fail(TGDK_E_INVALID, "grid dimensions must be >= 1");
    const bool known = (nreads == 1 && nwrites == 1) || (nreads == 3 && nwrites == 1) || (nreads == 6 && nwrites == 4);
    if (!known) return fail(TGDK_E_INVALID, "stream mixes: 1+1, 3+1 and 6+4 (reads + writes)");
    const int px = (dims[0] + 63) / 64 * 64;
    const long long n = (long long)px * dims[1] * dims[2];
    int mz = 0;
    if (pattern == 1) {  // one workgroup per 64 x 8 x mz chunk, about `blocks` chunks
        const long long cols = (long long)((dims[0] + 63) / 64) * ((dims[1] + 7) / 8);
        long long d = (cols * dims[2] + blocks - 1) / std::max(blocks, 1);
        mz = (int)std::max(4LL, std::min(d, (long long)dims[2]));
        blocks = (int)(cols * ((dims[2] + mz - 1) / mz));
    } else if (blocks < 1) {
        return fail(TGDK_E_INVALID, "blocks must be >= 1");
    }
    const int ns = nreads + nwrites;
    std::vector<double*> bufs(ns, nullptr);
    auto release = [&]() {
        for (double* p : bufs)
            if (p) (void)hipFree(p);
    };
    TGDK_HIP(hipSetDevice(ctx->device));
    for (int i = 0; i < ns; ++i) {
        if (hipMalloc((void**)&bufs[i], (size_t)n * 8) != hipSuccess) {
            release();
            return fail(TGDK_E_NOMEM, "probe buffers");
        }
        if (hipMemsetAsync(bufs[i], 0, (size_t)n * 8, ctx->stream) != hipSuccess) {
            release();
            return fail(TGDK_E_HIP, "probe buffers");
        }
    }
    ProbeArgs a;
    memset(&a, 0, sizeof(a));
    for (int i = 0; i < nreads; ++i) a.in[i] = bufs[i];
    for (int i = 0; i < nwrites; ++i) a.out[i] = bufs[nreads + i];
    auto launch = [&]() {
        if (nreads == 1 && nwrites == 1) launch_probe<1, 1>(pattern, a, dims, px, n, blocks, mz, ctx->stream);
        if (nreads == 3 && nwrites == 1) launch_probe<3, 1>(pattern, a, dims, px, n, blocks, mz, ctx->stream);
        if (nreads == 6 && nwrites == 4) launch_probe<6, 4>(pattern, a, dims, px, n, blocks, mz, ctx->stream);
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = TGDK_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        rc = fail(TGDK_E_HIP, "probe events");
    } else {
        launch();  // warm-up
        (void)hipEventRecord(e0, ctx->stream);
        for (int i = 0; i < reps; ++i) launch();
        (void)hipEventRecord(e1, ctx->stream);
        float ms = 0.0f;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
            hipGetLastError() != hipSuccess)
            rc = fail(TGDK_E_HIP, "probe launch");
        else
            *ms_per_launch = ms / reps;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    release();
    return rc;
}
