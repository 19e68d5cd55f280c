// 2.5-D blocking for the 3-D grid kernels (gfx950, wave64).
//
// A box tile of 64 x 4 x 4 points needs a 66 x 6 x 6 halo box, so every point
// of the grid is read about 2.3 times.  The marching kernels instead give a
// workgroup a column chunk of 64 (x) x MY (y) x MZ (z) points and walk it one
// z plane at a time: the plane's own points of z-1, z and z+1 stay in
// registers (the stencil's D and U terms), only plane z with its one-point
// ring in x and y goes through LDS (the W, E, S, N terms), and the loads of
// the plane after next are issued before the current plane is computed, so
// one plane of loads is always in flight behind the arithmetic.  Each point is
// read once, plus the ring (2 (64 + MY + 2) of 64 MY points per plane) and two
// extra planes per chunk.
#pragma once

#include "device_common.h"

namespace tgdk {

template <int MY_>
struct March {
    static constexpr int MY = MY_;
    static constexpr int BX = 66, BY = MY + 2;
    static constexpr int PLANE = BX * BY;           // LDS values per plane
    static constexpr int PPT = 64 * MY / NT;        // own points per thread per plane
    static constexpr int NRING = 2 * 64 + 2 * BY;   // ring points per plane
    static constexpr int RPT = (NRING + NT - 1) / NT;
    static_assert((64 * MY) % NT == 0, "plane must be a multiple of the workgroup");
};

// Chunk c of a grid with cx x cy columns: its first point and z range.
struct Chunk {
    int x0, y0, z0, z1;
};

template <class M>
__device__ __forceinline__ Chunk chunk_of(int c, int cx, int cy, int mz, int nz) {
    Chunk k;
    k.x0 = (c % cx) * 64;
    k.y0 = ((c / cx) % cy) * M::MY;
    k.z0 = (c / (cx * cy)) * mz;
    k.z1 = min(k.z0 + mz, nz);
    return k;
}

// Own point q of this thread in a plane: x, y offsets and LDS index.
template <class M>
__device__ __forceinline__ void own_point(int q, int& lx, int& ly, int& c) {
    const int l = threadIdx.x + q * NT;
    lx = l & 63;
    ly = l >> 6;
    c = (ly + 1) * M::BX + lx + 1;
}

// Ring point r of a plane: x, y offsets (-1 .. 64, -1 .. MY) and LDS index.
template <class M>
__device__ __forceinline__ void ring_point(int r, int& lx, int& ly, int& c) {
    if (r < 128) {
        lx = r & 63;
        ly = r < 64 ? -1 : M::MY;
    } else {
        const int i = r - 128;
        ly = (i >> 1) - 1;
        lx = (i & 1) ? 64 : -1;
    }
    c = (ly + 1) * M::BX + lx + 1;
}

// Plane stencil at LDS index c with the z neighbours from registers; terms in
// the order C, W, E, S, N, D, U (the same as stencil_row, so both give the
// same bits).  VAR = false takes the constant coefficients only, so the
// constant-coefficient kernels carry no branch (and no wait for coefficient
// loads) in their inner loop; VAR = true decides per operator at run time.
template <class M, bool VAR, class T>
__device__ __forceinline__ T stencil_march(const DevOp& op, const T* __restrict__ L, int c, long long g, T um,
                                           T up) {
    T cC, cW, cE, cS, cN, cD, cU;
    if (VAR && op.var) {
        const T* cf = coef_ptr<T>(op);
        const long long n = op.n;
        cC = cf[g];
        cW = cf[n + g];
        cE = cf[2 * n + g];
        cS = cf[3 * n + g];
        cN = cf[4 * n + g];
        cD = cf[5 * n + g];
        cU = cf[6 * n + g];
    } else {
        cC = (T)op.cc[0];
        cW = (T)op.cc[1];
        cE = (T)op.cc[2];
        cS = (T)op.cc[3];
        cN = (T)op.cc[4];
        cD = (T)op.cc[5];
        cU = (T)op.cc[6];
    }
    T y = cC * L[c];
    y += cW * L[c - 1];
    y += cE * L[c + 1];
    y += cS * L[c - M::BX];
    y += cN * L[c + M::BX];
    y += cD * um;
    y += cU * up;
    return y;
}

// Chunks per z column for a grid of cx x cy columns: the z depth of a chunk
// is chosen so that the grid has about `target` chunks, at least 4 planes.
inline int march_depth(int nz, int cx, int cy, int target) {
    const long long cols = (long long)cx * cy;
    long long mz = (cols * nz + target - 1) / target;
    if (mz < 4) mz = 4;
    if (mz > nz) mz = nz;
    return (int)mz;
}

}  // namespace tgdk

namespace tgdk {

// The marching loop over one chunk, shared by the 3-D kernels.  Ph (the
// kernel's phase) provides
//   struct Own, struct Ring        raw loads of an own / ring point of a plane
//   void load(Own&, long long g, long long gu)   g < 0: a point outside the domain (reads zeros)
//   void load(Ring&, long long g, long long gu)
//   T value(const Own&), T value(const Ring&)     the stencil input u
//   void emit(int q, long long g, long long gu, const Own& c, T y)
//                                                 outputs at own point q of plane z, y = (A u) there
//   void plane_done(const Chunk&, int z)          after every thread's emits of plane z
//                                                 (between two workgroup barriers)
// Every point comes with two indices: g in vectors stored with the padded
// row pitch op.px (the step kernel's own vectors) and gu in vectors of pitch
// op.nx (caller vectors, coefficient arrays); they coincide when px = nx.
// With px a multiple of 64, every 64-point row segment of a padded vector
// starts on a 128-byte line: at n_x = 255 a float32 segment otherwise spans
// three lines instead of two, and the step kernel's phases measured 15-19 %
// slower.
// Four register sets hold the own points of planes z-1, z, z+1 and z+2 (the
// last in flight while plane z is computed); the loop is unrolled four times
// so the sets change roles by position, never by register moves (a move
// would wait for the load in flight).  Every load is issued unconditionally
// (out-of-domain points read the zero page), so it stays in flight until its
// first use; the plane after the chunk's upper halo plane z1 reads the zero
// page too, since the next chunk reads it itself.  (Six sets for the phases
// with few raw values a point, more planes in flight, measured no faster:
// phase B 132 -> 138 us at 255^3.)
template <class M, bool VAR, class T, class Ph>
__device__ __forceinline__ void march_chunk(const DevOp& op, const Chunk& k, T* __restrict__ L, Ph& ph) {
    using Own = typename Ph::Own;
    using Ring = typename Ph::Ring;
    const long long plane = (long long)op.nx * op.ny;   // unpadded
    const long long pplane = (long long)op.px * op.ny;  // padded
    const int nz = op.nz;
    int cq[M::PPT];
    int bq[M::PPT], pq[M::PPT];  // in-plane offsets, unpadded and padded
    bool okq[M::PPT];
#pragma unroll
    for (int q = 0; q < M::PPT; ++q) {
        int lx, ly;
        own_point<M>(q, lx, ly, cq[q]);
        const int gx = k.x0 + lx, gy = k.y0 + ly;
        okq[q] = gx < op.nx && gy < op.ny;
        bq[q] = okq[q] ? gy * op.nx + gx : 0;
        pq[q] = okq[q] ? gy * op.px + gx : 0;
    }
    int cr[M::RPT];
    int br[M::RPT], pr[M::RPT];
    bool okr[M::RPT];
#pragma unroll
    for (int j = 0; j < M::RPT; ++j) {
        const int r = threadIdx.x + j * NT;
        int lx = 0, ly = 0, c = -1;
        if (r < M::NRING) ring_point<M>(r, lx, ly, c);
        const int gx = k.x0 + lx, gy = k.y0 + ly;
        cr[j] = c;
        okr[j] = c >= 0 && gx >= 0 && gx < op.nx && gy >= 0 && gy < op.ny;
        br[j] = okr[j] ? gy * op.nx + gx : 0;
        pr[j] = okr[j] ? gy * op.px + gx : 0;
    }
    auto load_own = [&](Own (&o)[M::PPT], int zz) {
        const bool okz = zz >= 0 && zz < nz && zz <= k.z1;
#pragma unroll
        for (int q = 0; q < M::PPT; ++q) {
            const bool ok = okq[q] && okz;
            ph.load(o[q], ok ? zz * pplane + pq[q] : -1LL, ok ? zz * plane + bq[q] : -1LL);
        }
    };
    auto load_ring = [&](Ring (&r)[M::RPT], int zz) {
        const bool okz = zz < k.z1;
#pragma unroll
        for (int j = 0; j < M::RPT; ++j) {
            const bool ok = okr[j] && okz;
            ph.load(r[j], ok ? zz * pplane + pr[j] : -1LL, ok ? zz * plane + br[j] : -1LL);
        }
    };
    // plane z: stage plane z (own points oc, ring rc) in LDS, issue the loads
    // of ring z + 1 (needed first) and of plane z + 2, compute plane z
    auto step = [&](const Own (&om)[M::PPT], const Own (&oc)[M::PPT], const Own (&op_)[M::PPT], Own (&on)[M::PPT],
                    const Ring (&rc)[M::RPT], Ring (&rn)[M::RPT], int z) {
#pragma unroll
        for (int q = 0; q < M::PPT; ++q) L[cq[q]] = ph.value(oc[q]);
#pragma unroll
        for (int j = 0; j < M::RPT; ++j)
            if (cr[j] >= 0) L[cr[j]] = ph.value(rc[j]);
        __syncthreads();
        load_ring(rn, z + 1);
        load_own(on, z + 2);
#pragma unroll
        for (int q = 0; q < M::PPT; ++q)
            if (okq[q]) {
                const long long gu = z * plane + bq[q];
                ph.emit(q, z * pplane + pq[q], gu, oc[q],
                        stencil_march<M, VAR, T>(op, L, cq[q], gu, ph.value(om[q]), ph.value(op_[q])));
            }
        if constexpr (Ph::PLANE_HOOK) {
            __syncthreads();
            ph.plane_done(k, z);
        }
        __syncthreads();
    };
    Own o0[M::PPT], o1[M::PPT], o2[M::PPT], o3[M::PPT];
    Ring r0[M::RPT], r1[M::RPT];
    const int z0 = k.z0, z1 = k.z1;
    load_own(o0, z0 - 1);
    load_own(o1, z0);
    load_own(o2, z0 + 1);
    load_ring(r0, z0);
    for (int z = z0; z < z1; z += 4) {
        step(o0, o1, o2, o3, r0, r1, z);
        if (z + 1 >= z1) break;
        step(o1, o2, o3, o0, r1, r0, z + 1);
        if (z + 2 >= z1) break;
        step(o2, o3, o0, o1, r0, r1, z + 2);
        if (z + 3 >= z1) break;
        step(o3, o0, o1, o2, r1, r0, z + 3);
    }
}

}  // namespace tgdk
