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
//              phases do (no LDS and no stencil: the access order alone);
//  tiled:      the same walk over arrays stored chunk by chunk: the 64 x 8
//              points of a chunk's plane are one contiguous 4 KB block
//              (layout [z][chunk][y mod 8][x mod 64]), padding points not
//              read or written;
//  march, D planes in flight: the march order again, with the loads of
//              plane z + D - 1 issued before plane z is summed and stored
//              (D = 2, 3), as the step kernel keeps loads of later planes in
//              flight while it computes a plane.
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

template <int NR, int NW, bool TILED>
__global__ __launch_bounds__(NT) void k_probe_march(ProbeArgs a, int nx, int ny, int nz, int px, int mz) {
    constexpr int TX = 64, TY = 8, PPT = TX * TY / NT;
    const int cx = (nx + TX - 1) / TX, cy = (ny + TY - 1) / TY;
    const int c = blockIdx.x;
    const int x0 = (c % cx) * TX, y0 = ((c / cx) % cy) * TY, z0 = (c / (cx * cy)) * mz;
    const int z1 = min(z0 + mz, nz);
    const long long pplane = TILED ? (long long)cx * cy * TX * TY : (long long)px * ny;
    long long off[PPT];
    bool ok[PPT];
#pragma unroll
    for (int q = 0; q < PPT; ++q) {
        const int l = threadIdx.x + q * NT;
        const int gx = x0 + l % TX, gy = y0 + l / TX;
        ok[q] = gx < nx && gy < ny;
        off[q] = TILED ? (long long)(c % (cx * cy)) * TX * TY + l : (long long)gy * px + gx;
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

// Loads of D planes in flight: register set d % D holds plane z0 + d; the z
// loop is unrolled by D so that every set is indexed statically.  A load
// past the chunk reads its last plane again (in bounds, not stored).
template <int NR, int NW, int D>
__global__ __launch_bounds__(NT) void k_probe_march_pf(ProbeArgs a, int nx, int ny, int nz, int px, int mz) {
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
        off[q] = ok[q] ? (long long)gy * px + gx : 0;
    }
    const double* __restrict__ in[NR];
    double* __restrict__ out[NW];
#pragma unroll
    for (int r = 0; r < NR; ++r) in[r] = a.in[r];
#pragma unroll
    for (int w = 0; w < NW; ++w) out[w] = a.out[w];
    double buf[D][PPT][NR];
    auto load = [&](double (&b)[PPT][NR], int z) {
        const long long zp = (long long)(z < z1 ? z : z1 - 1) * pplane;
#pragma unroll
        for (int q = 0; q < PPT; ++q)
#pragma unroll
            for (int r = 0; r < NR; ++r) b[q][r] = in[r][zp + off[q]];
    };
#pragma unroll
    for (int d = 0; d < D - 1; ++d) load(buf[d], z0 + d);
    for (int z = z0; z < z1; z += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            if (z + d >= z1) break;
            load(buf[(d + D - 1) % D], z + d + D - 1);
#pragma unroll
            for (int q = 0; q < PPT; ++q) {
                if (!ok[q]) continue;
                double v = 0.0;
#pragma unroll
                for (int r = 0; r < NR; ++r) v += buf[d][q][r];
                const long long g = (long long)(z + d) * pplane + off[q];
#pragma unroll
                for (int w = 0; w < NW; ++w) out[w][g] = v * (double)(w + 1);
            }
        }
    }
}

template <int NR, int NW>
void launch_probe(int pattern, const ProbeArgs& a, const int* dims, int px, long long n, int blocks, int mz,
                  hipStream_t s) {
    if (pattern == 0)
        hipLaunchKernelGGL((k_probe_contiguous<NR, NW>), dim3(blocks), dim3(NT), 0, s, a, n);
    else if (pattern == 1)
        hipLaunchKernelGGL((k_probe_march<NR, NW, false>), dim3(blocks), dim3(NT), 0, s, a, dims[0], dims[1],
                           dims[2], px, mz);
    else if (pattern == 2)
        hipLaunchKernelGGL((k_probe_march<NR, NW, true>), dim3(blocks), dim3(NT), 0, s, a, dims[0], dims[1],
                           dims[2], px, mz);
    else if (pattern == 3)
        hipLaunchKernelGGL((k_probe_march_pf<NR, NW, 2>), dim3(blocks), dim3(NT), 0, s, a, dims[0], dims[1],
                           dims[2], px, mz);
    else
        hipLaunchKernelGGL((k_probe_march_pf<NR, NW, 3>), dim3(blocks), dim3(NT), 0, s, a, dims[0], dims[1],
                           dims[2], px, mz);
}

}  // namespace

}  // namespace tgdk

using namespace tgdk;

extern "C" int tgdk_stream_probe(tgdk_ctx ctx, int pattern, int nreads, int nwrites, const int* dims, int blocks,
                                 int reps, double* ms_per_launch) {
    if (!ctx || !dims || !ms_per_launch || reps < 1 || pattern < 0 || pattern > 4)
        return fail(TGDK_E_INVALID, "bad argument");
    if (dims[0] < 1 || dims[1] < 1 || dims[2] < 1) return fail(TGDK_E_INVALID, "grid dimensions must be >= 1");
    const bool known = (nreads == 1 && nwrites == 1) || (nreads == 3 && nwrites == 1) || (nreads == 6 && nwrites == 4);
    if (!known) return fail(TGDK_E_INVALID, "stream mixes: 1+1, 3+1 and 6+4 (reads + writes)");
    const int px = (dims[0] + 63) / 64 * 64;
    // pattern 2 pads y to a multiple of 8 as well (whole 64 x 8 chunks)
    const long long n = (long long)px * (pattern == 2 ? (dims[1] + 7) / 8 * 8 : dims[1]) * dims[2];
    int mz = 0;
    if (pattern != 0) {  // one workgroup per 64 x 8 x mz chunk, about `blocks` chunks
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
