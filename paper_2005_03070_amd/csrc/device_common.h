// Device-side building blocks shared by the tgdk kernels (gfx950, wave64).
//
// * Tile geometry: every grid-shaped kernel gives one 256-thread workgroup a
//   64 (x) by TY (y) by TZ (z) tile.  x rows of 64 elements keep global
//   accesses coalesced; stencil kernels stage the tile plus a one-point halo
//   in LDS.
// * XCD-aware tile order: consecutive workgroup ids are dispatched round-robin
//   over the 8 XCDs, each with its own L2.  xcd_remap() gives every XCD a
//   contiguous range of tiles so the halo rows a tile shares with its
//   neighbours are read through the same L2.
// * Deterministic reductions: wave butterflies and a fixed LDS combine give a
//   per-workgroup partial; the next launch sums the partials in a fixed order
//   (a one-workgroup epilogue, or every workgroup of the step kernel
//   redundantly).  No atomics and no device-scope fences (on a multi-XCD part
//   an agent-scope release writes back the L2, which would serialise
//   thousands of workgroups); the kernel boundary makes the partials visible.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tgdk_shared.h"

namespace tgdk {

// Global-memory pointers.  The vectors reach the kernels inside descriptors
// read from memory, so the compiler cannot tell their address space and
// emits flat accesses, which count against the LDS counter as well as the
// memory counter: every LDS wait (each barrier, each LDS read of a
// reduction) then also waits for the loads and stores in flight.  gptr<T>
// is a pointer the compiler knows to be global; gp() converts a descriptor
// pointer (device memory from hipMalloc) to one.
template <class T>
using gptr = __attribute__((address_space(1))) T*;
template <class T>
__device__ __forceinline__ gptr<T> gp(const void* p) {
    return (gptr<T>)const_cast<void*>(p);
}
// A copy of a struct in global memory, read as 8-byte words through a
// global pointer (a struct copy through a generic pointer compiles to flat
// loads).
template <class T>
__device__ __forceinline__ T load_global(const T* p) {
    static_assert(sizeof(T) % 8 == 0, "8-byte words");
    T v;
    const gptr<const unsigned long long> s = gp<const unsigned long long>(p);
    unsigned long long* d = reinterpret_cast<unsigned long long*>(&v);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 8); ++i) d[i] = s[i];
    return v;
}

constexpr int NT = 256;         // threads per workgroup of the tile kernels
constexpr int NWAVE = NT / 64;
constexpr int NXCD = 8;         // XCDs on MI355X

template <int DIM, int TY_, int TZ_>
struct Tile {
    static constexpr int TX = 64, TY = TY_, TZ = TZ_;
    static constexpr int HZ = (DIM == 3) ? 1 : 0;
    static constexpr int BX = TX + 2, BY = TY + 2, BZ = TZ + 2 * HZ;
    static constexpr int BOX = BX * BY * BZ;
    static constexpr int PTS = TX * TY * TZ;
    static constexpr int PPT = PTS / NT;
    static_assert(PTS % NT == 0, "tile must be a multiple of the workgroup");
};

// The tile shapes a launch can use, by id (picked per operator by the tuner):
//   2-D: 0 = 64x16, 1 = 64x8, 2 = 64x4, 3 = 64x32
//   3-D: 0 = 64x4x4, 1 = 64x8x4, 2 = 64x4x8, 3 = 64x2x8
// with_tile<DIM>(id, f) calls f(Tile<...>{}) for that shape (host side).
template <int DIM, class F>
inline void with_tile(int tile_id, F&& f) {
    if constexpr (DIM == 2) {
        switch (tile_id) {
            case 1: f(Tile<2, 8, 1>{}); break;
            case 2: f(Tile<2, 4, 1>{}); break;
            case 3: f(Tile<2, 32, 1>{}); break;
            default: f(Tile<2, 16, 1>{}); break;
        }
    } else {
        switch (tile_id) {
            case 1: f(Tile<3, 8, 4>{}); break;
            case 2: f(Tile<3, 4, 8>{}); break;
            case 3: f(Tile<3, 2, 8>{}); break;
            default: f(Tile<3, 4, 4>{}); break;
        }
    }
}

__device__ __forceinline__ int xcd_remap(int b, int G) {
    const int q = G / NXCD, rem = G % NXCD;
    const int xcd = b % NXCD, local = b / NXCD;
    return xcd * q + (xcd < rem ? xcd : rem) + local;
}

// Position of a tile inside its problem.
struct TilePos {
    int x0, y0, z0;
};

template <class Cfg>
__device__ __forceinline__ TilePos tile_pos(int t, int tx, int ty) {
    TilePos p;
    const int ix = t % tx;
    const int rest = t / tx;
    p.x0 = ix * Cfg::TX;
    p.y0 = (rest % ty) * Cfg::TY;
    p.z0 = (rest / ty) * Cfg::TZ;
    return p;
}

template <class T>
__device__ __forceinline__ const T* coef_ptr(const DevOp& op);
template <>
__device__ __forceinline__ const double* coef_ptr<double>(const DevOp& op) { return op.coef64; }
template <>
__device__ __forceinline__ const float* coef_ptr<float>(const DevOp& op) { return op.coef32; }

// Stencil row at global point g whose value sits at LDS index c of a halo box
// with x stride 1, y stride BX and z stride BX*BY.  Terms are added in the
// fixed order C, W, E, S, N, D, U.
template <class Cfg, int DIM, class T>
__device__ __forceinline__ T stencil_row(const DevOp& op, const T* __restrict__ L, int c, long long g) {
    T cC, cW, cE, cS, cN, cD = 0, cU = 0;
    if (op.var) {
        const T* cf = coef_ptr<T>(op);
        const long long n = op.n;
        cC = cf[g];
        cW = cf[n + g];
        cE = cf[2 * n + g];
        cS = cf[3 * n + g];
        cN = cf[4 * n + g];
        if (DIM == 3) {
            cD = cf[5 * n + g];
            cU = cf[6 * n + g];
        }
    } else {
        cC = (T)op.cc[0];
        cW = (T)op.cc[1];
        cE = (T)op.cc[2];
        cS = (T)op.cc[3];
        cN = (T)op.cc[4];
        if (DIM == 3) {
            cD = (T)op.cc[5];
            cU = (T)op.cc[6];
        }
    }
    T y = cC * L[c];
    y += cW * L[c - 1];
    y += cE * L[c + 1];
    y += cS * L[c - Cfg::BX];
    y += cN * L[c + Cfg::BX];
    if (DIM == 3) {
        y += cD * L[c - Cfg::BX * Cfg::BY];
        y += cU * L[c + Cfg::BX * Cfg::BY];
    }
    return y;
}

// stencil_row with the coefficient kind narrowed at compile time: VAR = false
// takes the constants only, so the constant-coefficient kernels carry no
// branch and no wait for coefficient loads in their inner loops (VAR = true
// decides per operator at run time); same terms, same order.
template <class Cfg, int DIM, bool VAR, class T>
__device__ __forceinline__ T stencil_row_t(const DevOp& op, const T* __restrict__ L, int c, long long g) {
    T cC, cW, cE, cS, cN, cD = 0, cU = 0;
    if (VAR && op.var) {
        const T* cf = coef_ptr<T>(op);
        const long long n = op.n;
        cC = cf[g];
        cW = cf[n + g];
        cE = cf[2 * n + g];
        cS = cf[3 * n + g];
        cN = cf[4 * n + g];
        if (DIM == 3) {
            cD = cf[5 * n + g];
            cU = cf[6 * n + g];
        }
    } else {
        cC = (T)op.cc[0];
        cW = (T)op.cc[1];
        cE = (T)op.cc[2];
        cS = (T)op.cc[3];
        cN = (T)op.cc[4];
        if (DIM == 3) {
            cD = (T)op.cc[5];
            cU = (T)op.cc[6];
        }
    }
    T y = cC * L[c];
    y += cW * L[c - 1];
    y += cE * L[c + 1];
    y += cS * L[c - Cfg::BX];
    y += cN * L[c + Cfg::BX];
    if (DIM == 3) {
        y += cD * L[c - Cfg::BX * Cfg::BY];
        y += cU * L[c + Cfg::BX * Cfg::BY];
    }
    return y;
}

// Halo-box index h -> global coordinates.
template <class Cfg>
__device__ __forceinline__ void box_coords(int h, const TilePos& tp, int& gx, int& gy, int& gz) {
    const int hx = h % Cfg::BX;
    const int hy = (h / Cfg::BX) % Cfg::BY;
    const int hz = h / (Cfg::BX * Cfg::BY);
    gx = tp.x0 + hx - 1;
    gy = tp.y0 + hy - 1;
    gz = tp.z0 + hz - Cfg::HZ;
}

// Interior point q of this thread -> global coordinates and LDS centre index.
template <class Cfg>
__device__ __forceinline__ void point_coords(int q, const TilePos& tp, int& gx, int& gy, int& gz, int& c) {
    const int l = threadIdx.x + q * NT;
    const int lx = l % Cfg::TX;
    const int ly = (l / Cfg::TX) % Cfg::TY;
    const int lz = l / (Cfg::TX * Cfg::TY);
    gx = tp.x0 + lx;
    gy = tp.y0 + ly;
    gz = tp.z0 + lz;
    c = ((lz + Cfg::HZ) * Cfg::BY + (ly + 1)) * Cfg::BX + (lx + 1);
}

// Store of a vector element that the next launch reads (from any XCD).  On
// 2-D grids (working sets that live in the 256 MB MALL, launches dominated by
// latency) a streaming store keeps the line from sitting dirty in this XCD's
// L2 until the end-of-kernel write-back; on the large 3-D grids a plain store
// measured slightly faster.
template <int DIM, class T>
__device__ __forceinline__ void st_stream(T* p, T v) {
    if (DIM == 2)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <int DIM, class T>
__device__ __forceinline__ void st_stream(gptr<T> p, T v) {
    if (DIM == 2)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Sec. 4.1, step 3 b): the relative tolerance rt of inner cycle icyc
// (1-based, of ncyc requested) that starts from a residual of norm nu, given
// the initial residual norm nu0 and the overall tolerance tau (rtol ||r0||
// in the paper).  Criterion 1 shares the remaining orders of magnitude
// equally over the cycles left; criterion 2 asks the cycle to reach at
// least the geometric schedule's value for icyc; the smaller one is taken
// (ties count as criterion 1).  Past ncyc the cycle aims straight at tau.
// float32 inner cycles are floored at fp32_floor.  Returns the criterion
// (1, 2, or 3 past ncyc).  The one definition for every solver driver.
__device__ __forceinline__ int cycle_tolerance(double nu, double nu0, double tau, int icyc, int ncyc, int fp32,
                                               double fp32_floor, double& rt) {
    int branch;
    if (icyc > ncyc) {
        rt = tau / nu;
        branch = 3;
    } else {
        const double t1 = pow(tau / nu, 1.0 / (double)(ncyc - icyc + 1));
        const double t2 = (nu0 / nu) * pow(tau / nu0, (double)icyc / (double)ncyc);
        if (t1 <= t2) {
            rt = t1;
            branch = 1;
        } else {
            rt = t2;
            branch = 2;
        }
    }
    if (fp32 == 1 && rt < fp32_floor) rt = fp32_floor;
    return branch;
}

__device__ __forceinline__ bool inside(const DevOp& op, int gx, int gy, int gz) {
    return gx >= 0 && gx < op.nx && gy >= 0 && gy < op.ny && gz >= 0 && gz < op.nz;
}

__device__ __forceinline__ long long gidx(const DevOp& op, int gx, int gy, int gz) {
    return ((long long)gz * op.ny + gy) * op.nx + gx;
}

// Index of point (gx, gy, gz) in a vector stored with the padded row pitch
// op.px (the step kernel's residual and inner vectors on 3-D grids).
__device__ __forceinline__ long long pidx(const DevOp& op, int gx, int gy, int gz) {
    return ((long long)gz * op.ny + gy) * op.px + gx;
}

// Fills the halo of an LDS box (everything except the tile interior, which
// the caller writes from its own points): the rows above/below the tile (and
// the planes in front/behind it in 3-D), 64 wide and coalesced, then the two
// halo columns of every box row.  val(g) gives the value at an in-domain
// global index; out-of-domain points get zero.  Fixed trip counts, so the
// loads of all iterations are in flight together.
template <class Cfg, int DIM, class T, class F>
__device__ __forceinline__ void fill_halo(T* L, const TilePos& tp, const DevOp& op, F&& val) {
    constexpr int BX = Cfg::BX, BY = Cfg::BY, BZ = Cfg::BZ, TY = Cfg::TY, TZ = Cfg::TZ, HZ = Cfg::HZ;
    constexpr int HR = (DIM == 3) ? (2 * TZ + 2 * BY) : 2;
    constexpr int NHR = HR * 64;
#pragma unroll
    for (int k = 0; k < (NHR + NT - 1) / NT; ++k) {
        const int e = threadIdx.x + k * NT;
        if (e < NHR) {
            const int hr = e >> 6, lane = e & 63;
            int hy, hz;
            if (hr < 2 * TZ) {
                hz = (hr >> 1) + HZ;
                hy = (hr & 1) ? TY + 1 : 0;
            } else {
                const int i2 = hr - 2 * TZ;
                hz = (i2 >= BY) ? BZ - 1 : 0;
                hy = i2 % BY;
            }
            const int gx = tp.x0 + lane, gy = tp.y0 + hy - 1, gz = tp.z0 + hz - HZ;
            L[(hz * BY + hy) * BX + lane + 1] =
                (gx < op.nx && gy >= 0 && gy < op.ny && gz >= 0 && gz < op.nz) ? val(gidx(op, gx, gy, gz)) : T(0);
        }
    }
    constexpr int NHC = BY * BZ * 2;
#pragma unroll
    for (int k = 0; k < (NHC + NT - 1) / NT; ++k) {
        const int e = threadIdx.x + k * NT;
        if (e < NHC) {
            const int br = e >> 1, side = e & 1;
            const int hz = br / BY, hy = br % BY, hx = side ? BX - 1 : 0;
            const int gx = tp.x0 + hx - 1, gy = tp.y0 + hy - 1, gz = tp.z0 + hz - HZ;
            L[(hz * BY + hy) * BX + hx] = inside(op, gx, gy, gz) ? val(gidx(op, gx, gy, gz)) : T(0);
        }
    }
}

// The halo of a tile as fixed per-thread slots (the same enumeration as
// fill_halo): HK slots per thread; slot h of this thread has LDS index ch[h]
// (-1: unused slot) and global index gh[h] (-1: outside the domain).  Lets a
// kernel issue every halo load before any arithmetic or LDS store.
template <class Cfg, int DIM>
struct Halo {
    static constexpr int HR = (DIM == 3) ? (2 * Cfg::TZ + 2 * Cfg::BY) : 2;
    static constexpr int NHR = HR * 64;
    static constexpr int NHC = Cfg::BY * Cfg::BZ * 2;
    static constexpr int KR = (NHR + NT - 1) / NT, KC = (NHC + NT - 1) / NT;
    static constexpr int HK = KR + KC;
};

template <class Cfg, int DIM>
__device__ __forceinline__ void halo_slots(const TilePos& tp, const DevOp& op, int (&ch)[Halo<Cfg, DIM>::HK],
                                           long long (&gh)[Halo<Cfg, DIM>::HK]) {
    using H = Halo<Cfg, DIM>;
    constexpr int BX = Cfg::BX, BY = Cfg::BY, BZ = Cfg::BZ, TY = Cfg::TY, TZ = Cfg::TZ, HZ = Cfg::HZ;
#pragma unroll
    for (int k = 0; k < H::KR; ++k) {
        const int e = threadIdx.x + k * NT;
        ch[k] = -1;
        gh[k] = -1;
        if (e < H::NHR) {
            const int hr = e >> 6, lane = e & 63;
            int hy, hz;
            if (hr < 2 * TZ) {
                hz = (hr >> 1) + HZ;
                hy = (hr & 1) ? TY + 1 : 0;
            } else {
                const int i2 = hr - 2 * TZ;
                hz = (i2 >= BY) ? BZ - 1 : 0;
                hy = i2 % BY;
            }
            const int gx = tp.x0 + lane, gy = tp.y0 + hy - 1, gz = tp.z0 + hz - HZ;
            ch[k] = (hz * BY + hy) * BX + lane + 1;
            if (gx < op.nx && gy >= 0 && gy < op.ny && gz >= 0 && gz < op.nz) gh[k] = gidx(op, gx, gy, gz);
        }
    }
#pragma unroll
    for (int k = 0; k < H::KC; ++k) {
        const int e = threadIdx.x + k * NT;
        ch[H::KR + k] = -1;
        gh[H::KR + k] = -1;
        if (e < H::NHC) {
            const int br = e >> 1, side = e & 1;
            const int hz = br / BY, hy = br % BY, hx = side ? BX - 1 : 0;
            const int gx = tp.x0 + hx - 1, gy = tp.y0 + hy - 1, gz = tp.z0 + hz - HZ;
            ch[H::KR + k] = (hz * BY + hy) * BX + hx;
            if (inside(op, gx, gy, gz)) gh[H::KR + k] = gidx(op, gx, gy, gz);
        }
    }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One data-parallel-primitive move of a double (two 32-bit halves): lane i
// receives the source lane that CTRL selects; lanes of rows outside ROWMASK
// receive 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_move(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROWMASK, 0xf, false);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROWMASK, 0xf, false);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Sum over the 64 lanes of a wave through lane moves instead of LDS
// permutes: pairs, quads (quad permutations), eight and sixteen lanes (half-
// row and row mirrors), then the rows combined by the row broadcasts of
// lanes 15 and 31 into row 3; lane 63's total is returned to every lane.
// A fixed order: every wave that sums the same values gets the same bits.
__device__ __forceinline__ double wave_sum_dpp(double v) {
    v += dpp_move<0xB1, 0xf>(v);   // quad_perm [1,0,3,2]
    v += dpp_move<0x4E, 0xf>(v);   // quad_perm [2,3,0,1]
    v += dpp_move<0x141, 0xf>(v);  // row_half_mirror
    v += dpp_move<0x140, 0xf>(v);  // row_mirror
    v += dpp_move<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_move<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 63);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

template <bool DPP>
__device__ __forceinline__ double wave_sum_t(double v) {
    if constexpr (DPP)
        return wave_sum_dpp(v);
    else
        return wave_sum(v);
}

// Sums a[0..NR) over the workgroup; the totals land in out[0..NR) of thread
// i < NR (other threads' out is undefined).  sh needs NWAVE*NR doubles.
template <int NR, bool DPP = false>
__device__ __forceinline__ void block_sum(const double (&a)[NR], double* sh, double& out) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NR; ++i) {
        const double s = wave_sum_t<DPP>(a[i]);
        if (lane == 0) sh[w * NR + i] = s;
    }
    __syncthreads();
    out = 0.0;
    if (threadIdx.x < NR) {
        double s = sh[threadIdx.x];
        for (int w2 = 1; w2 < NWAVE; ++w2) s += sh[w2 * NR + threadIdx.x];
        out = s;
    }
    __syncthreads();
}

// Runtime-width variant: a[i] for i < nr held in shared memory rows; used
// by the projection kernels.  vals[t * stride + i] contains thread t's value i.
template <bool DPP = false>
__device__ __forceinline__ double block_sum_one(double v, double* sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v = wave_sum_t<DPP>(v);
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = sh[0];
    for (int w2 = 1; w2 < NWAVE; ++w2) s += sh[w2];
    __syncthreads();
    return s;
}

// Sums column i of partial[t * stride + i] over t = 0..ntiles-1 in a fixed
// order (one workgroup); the result is valid in every thread.
__device__ __forceinline__ double sum_partials(const double* partial, int ntiles, int stride, int i, double* sh) {
    double s = 0.0;
    for (int t = threadIdx.x; t < ntiles; t += NT) s += partial[(long long)t * stride + i];
    return block_sum_one(s, sh);
}

// Sums columns 0..NV-1 of partial[t * stride + v] over t = 0..ntiles-1 in a
// fixed order, all columns in one pass (independent loads in flight); every
// thread receives the totals.  sh needs NWAVE*NV doubles.
template <int NV>
__device__ __forceinline__ void sum_partials_multi(const double* __restrict__ partial, int ntiles, int stride,
                                                   double (&out)[NV], double* sh) {
    double a[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) a[v] = 0.0;
#pragma unroll 4
    for (int t = threadIdx.x; t < ntiles; t += NT) {
        const double* row = partial + (long long)t * stride;
#pragma unroll
        for (int v = 0; v < NV; ++v) a[v] += row[v];
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const double s = wave_sum(a[v]);
        if (lane == 0) sh[w * NV + v] = s;
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double s = sh[v];
        for (int w2 = 1; w2 < NWAVE; ++w2) s += sh[w2 * NV + v];
        out[v] = s;
    }
    __syncthreads();
}

// Sums ncols columns (ncols <= NT/4) of partial[t * stride + c] over
// t = 0..ntiles-1 into out[c] (LDS or global), in a fixed order: thread
// (part, c) sums tiles part, part + nparts, ...; then the parts are added in
// order.  scratch needs NT doubles.
__device__ __forceinline__ void sum_partial_columns(const double* __restrict__ partial, int ntiles, int stride,
                                                    int ncols, double* out, double* scratch) {
    const int nparts = NT / ncols;
    const int c = threadIdx.x % ncols, part = threadIdx.x / ncols;
    double a = 0.0;
    if (part < nparts)
        for (int t = part; t < ntiles; t += nparts) a += partial[(long long)t * stride + c];
    scratch[threadIdx.x] = a;
    __syncthreads();
    if (threadIdx.x < ncols) {
        double s = 0.0;
        for (int q = 0; q < nparts; ++q) s += scratch[q * ncols + threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

// Sums values 0..NV-1 of a value-major partial array (value v of workgroup t
// at part[v * nwg + t]) over t = 0..nwg-1 in a fixed order; every thread
// receives the totals, and every workgroup that calls this on the same array
// gets the same bits.  sh needs NWAVE*NV doubles.
template <int NV, bool DPP = false>
__device__ __forceinline__ void sum_values(const double* __restrict__ part_in, int nwg, double (&out)[NV], double* sh) {
    const gptr<const double> part = gp<const double>(part_in);
    double a[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) a[v] = 0.0;
    // the first four rounds with every load issued before the adds (clamped
    // addresses, masked values); more workgroups than 4 * NT in a tail loop
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int t = threadIdx.x + r * NT;
        const int tc = t < nwg ? t : 0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double x = part[(long long)v * nwg + tc];
            a[v] += t < nwg ? x : 0.0;
        }
    }
    for (int t = threadIdx.x + 4 * NT; t < nwg; t += NT) {
#pragma unroll
        for (int v = 0; v < NV; ++v) a[v] += part[(long long)v * nwg + t];
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const double s = wave_sum_t<DPP>(a[v]);
        if (lane == 0) sh[w * NV + v] = s;
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double s = sh[v];
        for (int w2 = 1; w2 < NWAVE; ++w2) s += sh[w2 * NV + v];
        out[v] = s;
    }
    __syncthreads();
}

template <class T>
__device__ __forceinline__ T* vp(void* p) {
    return reinterpret_cast<T*>(p);
}

template <class T>
__device__ __forceinline__ const T* vp(const void* p) {
    return reinterpret_cast<const T*>(p);
}

// Problem lookup for grouped launches (linear scan; groups are small).
__device__ __forceinline__ int find_prob(const DevProb* probs, int nprob, int tile) {
    int j = 0;
    while (j + 1 < nprob && tile >= probs[j + 1].tile_begin) ++j;
    return j;
}

}  // namespace tgdk
