// Multigrid V-cycle kernels for a constant-coefficient operator (the
// preconditioner of Sec. 5, Example 5).  A V-cycle on a 511^2 grid visits nine
// levels, most of them a few thousand points or fewer, and every dependent
// pass over a level costs a kernel boundary (measured: 2.5 to 4.5 us per
// pass whatever the level's size), so the cost is the number of passes, not
// bytes.  Two things cut the passes:
//
//  * fused passes: the first two sweeps from z = 0 are one pass (the first
//    sweep's values s v are formed where the second needs them), the residual
//    is formed inside the full-weighting restriction, and the prolongated
//    correction is added inside the first post-smoothing sweep.  With two
//    sweeps a level is 4 passes instead of 7;
//  * the coarse tail of the hierarchy (every level from the first one whose
//    z, v and sweep temporary fit in 48 KiB of LDS, down to the coarsest)
//    runs as one workgroup: each pass on those levels is a pass over LDS
//    followed by a barrier, and only the tail's finest v comes in from and
//    its z goes out to global memory.
//
// Every value is computed with the operations of the separate-pass
// formulation, in the same order (stencil terms C, W, E, S, N, D, U; the
// Jacobi update z + s (v - A z); full weighting and linear interpolation
// summed x, then y, then z): a fused pass recomputes the intermediate values
// it needs rather than reading them, so the tail and the global levels give
// the same numbers as passes taken one at a time.
#include "device_common.h"
#include "launch.h"
#include "mg_shared.h"

namespace tgdk {

// (A f)(i, j, k) for the level's constant stencil, f a field given as
// f(i, j, k, linear index) and zero outside the grid.  A neighbour outside
// the grid is read at the point itself and the value dropped afterwards, so
// every read is in bounds and none sits behind a branch (a wave issues them
// all before it waits).
template <int DIM, class F>
__device__ __forceinline__ double mg_stencil(const MgLvl& L, F f, int i, int j, int k, int p) {
    const int sxy = L.nx * L.ny;
    const bool w = i > 0, e = i + 1 < L.nx, s = j > 0, n = j + 1 < L.ny;
    const double fc = f(i, j, k, p);
    const double fw = f(w ? i - 1 : i, j, k, w ? p - 1 : p);
    const double fe = f(e ? i + 1 : i, j, k, e ? p + 1 : p);
    const double fs = f(i, s ? j - 1 : j, k, s ? p - L.nx : p);
    const double fn = f(i, n ? j + 1 : j, k, n ? p + L.nx : p);
    double y = L.cc[0] * fc;
    y += L.cc[1] * (w ? fw : 0.0);
    y += L.cc[2] * (e ? fe : 0.0);
    y += L.cc[3] * (s ? fs : 0.0);
    y += L.cc[4] * (n ? fn : 0.0);
    if (DIM == 3) {
        const bool d = k > 0, u = k + 1 < L.nz;
        const double fd = f(i, j, d ? k - 1 : k, d ? p - sxy : p);
        const double fu = f(i, j, u ? k + 1 : k, u ? p + sxy : p);
        y += L.cc[5] * (d ? fd : 0.0);
        y += L.cc[6] * (u ? fu : 0.0);
    }
    return y;
}

// Linear interpolation of the coarse array c (ncx x ncy x ncz) at fine
// point (fi, fj, fk), per axis 1/2 c[(f - 1) >> 1] + 1/2 c[f >> 1] (zero
// outside): the two neighbours of an even fine index, or twice the
// coinciding coarse value of an odd one, whose two halves add back to it
// exactly.  No branch on the parity, so a wave issues all its loads at once.
__device__ __forceinline__ double mg_cval(const double* c, int ncx, int ncy, int ncz, int I, int J, int K) {
    const bool in = I >= 0 && I < ncx && J >= 0 && J < ncy && K >= 0 && K < ncz;
    const int Ic = min(max(I, 0), ncx - 1), Jc = min(max(J, 0), ncy - 1), Kc = min(max(K, 0), ncz - 1);
    const double x = c[(Kc * ncy + Jc) * ncx + Ic];   // always in bounds
    return in ? x : 0.0;
}
template <int DIM>
__device__ __forceinline__ double mg_prolong(const double* c, int ncx, int ncy, int ncz, int fi, int fj, int fk) {
    const int I0 = (fi - 1) >> 1, I1 = fi >> 1, J0 = (fj - 1) >> 1, J1 = fj >> 1;
    auto xy = [&](int K) {
        const double r0 = 0.5 * mg_cval(c, ncx, ncy, ncz, I0, J0, K) + 0.5 * mg_cval(c, ncx, ncy, ncz, I1, J0, K);
        const double r1 = 0.5 * mg_cval(c, ncx, ncy, ncz, I0, J1, K) + 0.5 * mg_cval(c, ncx, ncy, ncz, I1, J1, K);
        return 0.5 * r0 + 0.5 * r1;
    };
    if (DIM == 2) return xy(0);
    return 0.5 * xy((fk - 1) >> 1) + 0.5 * xy(fk >> 1);
}

// Full weighting at coarse point (I, J, K) of a fine field r(fi, fj, fk):
// weights 1/4, 1/2, 1/4 along x, then y, then z, each 1-D sum taken left to
// right (the products by 1/4 and 1/2 are exact, so accumulating term by term
// rounds as the three-term sum does).  The z loop is kept rolled so that a
// 3-D point holds one plane's residuals at a time.
template <int DIM, class R>
__device__ __forceinline__ double mg_restrict(R r, int I, int J, int K) {
    auto plane = [&](int fk) {
        double y = 0.0;
#pragma unroll
        for (int dj = 0; dj < 3; ++dj) {
            double x = 0.0;
#pragma unroll
            for (int di = 0; di < 3; ++di) x += (di == 1 ? 0.5 : 0.25) * r(2 * I + di, 2 * J + dj, fk);
            y += (dj == 1 ? 0.5 : 0.25) * x;
        }
        return y;
    };
    if (DIM == 2) return plane(0);
    double z = 0.0;
#pragma unroll 1
    for (int dk = 0; dk < 3; ++dk) z += (dk == 1 ? 0.5 : 0.25) * plane(2 * K + dk);
    return z;
}

// The value of one pass (mode without MG_ACC) at point p = (i, j, k) of
// level L; zc: the next coarser level's z (PSWEEP only; the sides of a level
// that has a coarser one are odd, n = 2 nc + 1).
template <int DIM>
__device__ __forceinline__ double mg_point(const MgLvl& L, const double* z, const double* v, const double* zc,
                                           int i, int j, int k, int p, int mode) {
    const double sc = L.sc;
    if (mode == MG_FIRST) return sc * v[p];
    if (mode == MG_FIRST2) {
        auto z1 = [&](int, int, int, int q) { return sc * v[q]; };
        return z1(i, j, k, p) + sc * (v[p] - mg_stencil<DIM>(L, z1, i, j, k, p));
    }
    if (mode == MG_PSWEEP) {
        const int ncx = L.nx >> 1, ncy = L.ny >> 1, ncz = DIM == 3 ? L.nz >> 1 : 1;
        auto zp = [&](int a, int b, int c, int q) { return z[q] + mg_prolong<DIM>(zc, ncx, ncy, ncz, a, b, c); };
        return zp(i, j, k, p) + sc * (v[p] - mg_stencil<DIM>(L, zp, i, j, k, p));
    }
    auto zf = [&](int, int, int, int q) { return z[q]; };
    const double az = mg_stencil<DIM>(L, zf, i, j, k, p);
    if (mode == MG_RESID) return v[p] - az;
    return z[p] + sc * (v[p] - az);
}

// Full weighting of the residual v - A z of level F at coarse point p of the
// next level (sides (F.n - 1) / 2).
template <int DIM>
__device__ __forceinline__ double mg_resid_restrict(const MgLvl& F, const double* z, const double* v, int ncx,
                                                    int ncy, int p) {
    const int I = p % ncx, q = p / ncx, J = q % ncy, K = q / ncy;
    auto zf = [&](int, int, int, int s) { return z[s]; };
    auto r = [&](int fi, int fj, int fk) {
        const int fp = (fk * F.ny + fj) * F.nx + fi;
        return v[fp] - mg_stencil<DIM>(F, zf, fi, fj, fk, fp);
    };
    return mg_restrict<DIM>(r, I, J, K);
}

// ------------------------------------------------------------ global levels
template <int DIM, int MODE>
__global__ __launch_bounds__(256) void k_mg_pass(MgLvl L, const double* __restrict__ z,
                                                 const double* __restrict__ v, const double* __restrict__ zc,
                                                 double* __restrict__ out, int acc) {
    const int n = L.nx * L.ny * L.nz;
    for (int p = blockIdx.x * 256 + threadIdx.x; p < n; p += gridDim.x * 256) {
        int i = 0, j = 0, k = 0;
        if (MODE != MG_FIRST) {
            const int q = p / L.nx;
            i = p - q * L.nx;
            j = DIM == 3 ? q % L.ny : q;
            k = DIM == 3 ? q / L.ny : 0;
        }
        const double r = mg_point<DIM>(L, z, v, zc, i, j, k, p, MODE);
        out[p] = acc ? out[p] + r : r;
    }
}

// vc = R (v - A z) on the next coarser level
template <int DIM>
__global__ __launch_bounds__(256) void k_mg_resid_restrict(MgLvl F, const double* __restrict__ z,
                                                           const double* __restrict__ v, double* __restrict__ vc) {
    const int ncx = F.nx >> 1, ncy = F.ny >> 1, ncz = DIM == 3 ? F.nz >> 1 : 1;
    const int nc = ncx * ncy * ncz;
    for (int p = blockIdx.x * 256 + threadIdx.x; p < nc; p += gridDim.x * 256)
        vc[p] = mg_resid_restrict<DIM>(F, z, v, ncx, ncy, p);
}

static int mg_blocks(long long n) {
    long long b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    return b < 1 ? 1 : (int)b;
}

template <int DIM>
static void mg_pass_dim(const MgLvl& L, const double* z, const double* v, const double* zc, double* out, int mode,
                        hipStream_t s) {
    const int nb = mg_blocks((long long)L.nx * L.ny * L.nz);
    const int acc = (mode & MG_ACC) ? 1 : 0;
    switch (mode & 7) {
        case MG_FIRST:
            hipLaunchKernelGGL((k_mg_pass<DIM, MG_FIRST>), dim3(nb), dim3(256), 0, s, L, z, v, zc, out, acc);
            break;
        case MG_FIRST2:
            hipLaunchKernelGGL((k_mg_pass<DIM, MG_FIRST2>), dim3(nb), dim3(256), 0, s, L, z, v, zc, out, acc);
            break;
        case MG_SWEEP:
            hipLaunchKernelGGL((k_mg_pass<DIM, MG_SWEEP>), dim3(nb), dim3(256), 0, s, L, z, v, zc, out, acc);
            break;
        case MG_PSWEEP:
            hipLaunchKernelGGL((k_mg_pass<DIM, MG_PSWEEP>), dim3(nb), dim3(256), 0, s, L, z, v, zc, out, acc);
            break;
        default:
            hipLaunchKernelGGL((k_mg_pass<DIM, MG_RESID>), dim3(nb), dim3(256), 0, s, L, z, v, zc, out, acc);
            break;
    }
}

void launch_mg_pass(int dim, const MgLvl& L, const double* z, const double* v, const double* zc, double* out,
                    int mode, hipStream_t s) {
    if (dim == 2)
        mg_pass_dim<2>(L, z, v, zc, out, mode, s);
    else
        mg_pass_dim<3>(L, z, v, zc, out, mode, s);
}

void launch_mg_resid_restrict(int dim, const MgLvl& F, const double* z, const double* v, double* vc,
                              hipStream_t s) {
    const long long nc = (long long)(F.nx >> 1) * (F.ny >> 1) * (dim == 3 ? F.nz >> 1 : 1);
    const int nb = mg_blocks(nc);
    if (dim == 2)
        hipLaunchKernelGGL(k_mg_resid_restrict<2>, dim3(nb), dim3(256), 0, s, F, z, v, vc);
    else
        hipLaunchKernelGGL(k_mg_resid_restrict<3>, dim3(nb), dim3(256), 0, s, F, z, v, vc);
}

// ------------------------------------------------------- the coarse tail
// Orders one wave's LDS writes before its later reads by other lanes of the
// same wave (LDS serves a wave's operations in order; the fences keep the
// compiler from moving them).
__device__ __forceinline__ void mg_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One V-cycle for the tail's finest level from z = 0 with right-hand side
// vin; the result goes to out (added to it if acc).  Every pass is over LDS;
// no pass writes an array it reads.  Passes over levels before wave_from use
// all threads and end in a workgroup barrier; the levels from wave_from on
// (at most 64 points each) are run by the first wave alone, a point per lane,
// ordered by wave-level fences, with a workgroup barrier where the work
// moves between the two.
template <int DIM, int NTT>
__global__ __launch_bounds__(NTT) void k_mg_tail(const MgTail* __restrict__ P, const double* __restrict__ vin,
                                                 double* __restrict__ out, int acc) {
    __shared__ double S[MG_TAIL_LDS];
    const int t = threadIdx.x;
    const int nlev = P->nlev, nu = P->nu, lw = P->wave_from;
    auto sync = [&](int l) {
        if (l >= lw)
            mg_wave_sync();
        else
            __syncthreads();
    };
    // the points of level l this thread computes: p = t, t + stride, ...
    auto stride = [&](int l) { return l >= lw ? (t < 64 ? 64 : 0) : NTT; };
    // one pass over level l: dst = pass(z at zin, v, coarse z at zcin)
    auto pass = [&](int l, int zin, int zcin, int dst, int mode) {
        const MgLvl L = P->lv[l];
        const int n = L.nx * L.ny * L.nz, st = stride(l);
        const double* v = S + P->voff[l];
        if (st)
            for (int p = t; p < n; p += st) {
                const int i = p % L.nx, q = p / L.nx, j = q % L.ny, k = q / L.ny;
                S[dst + p] = mg_point<DIM>(L, S + zin, v, S + zcin, i, j, k, p, mode);
            }
        sync(l);
    };
    // count sweeps from z = 0 (the first two as one pass), alternating
    // between z_l and t_l so that the last lands in z_l
    auto smooth0 = [&](int l, int count) {
        const int passes = count >= 2 ? count - 1 : 1;
        int cur = 0;
        for (int i = 0; i < passes; ++i) {
            const int dst = ((passes - 1 - i) & 1) ? P->toff[l] : P->zoff[l];
            pass(l, cur, 0, dst, i > 0 ? MG_SWEEP : (count >= 2 ? MG_FIRST2 : MG_FIRST));
            cur = dst;
        }
    };
    {
        const int n0 = P->lv[0].nx * P->lv[0].ny * P->lv[0].nz;
        for (int p = t; p < n0; p += NTT) S[P->voff[0] + p] = vin[p];
        __syncthreads();
    }
    for (int l = 0; l + 1 < nlev; ++l) {
        smooth0(l, nu);
        const MgLvl F = P->lv[l], C = P->lv[l + 1];
        const int nc = C.nx * C.ny * C.nz, st = stride(l);
        if (st)
            for (int p = t; p < nc; p += st)
                S[P->voff[l + 1] + p] = mg_resid_restrict<DIM>(F, S + P->zoff[l], S + P->voff[l], C.nx, C.ny, p);
        sync(l);
    }
    {
        const int lc = nlev - 1;
        const MgLvl L = P->lv[lc];
        if (L.nx * L.ny * L.nz == 1) {
            // a single point (every neighbour outside the grid): its sweeps
            // z <- z + s (v - C z) in one thread's registers
            if (t == 0) {
                const double v = S[P->voff[lc]], C = L.cc[0], sc = L.sc;
                double z = sc * v;
                for (int i = 1; i < P->coarsest_sweeps; ++i) z = z + sc * (v - C * z);
                S[P->zoff[lc]] = z;
            }
            sync(lc);
        } else {
            smooth0(lc, P->coarsest_sweeps);
        }
    }
    int cur = P->zoff[nlev - 1];   // z of the level below the one being finished
    for (int l = nlev - 2; l >= 0; --l) {
        if (l + 1 == lw) __syncthreads();   // the first wave's results, to every wave
        const int zl = P->zoff[l], tl = P->toff[l];
        pass(l, zl, cur, tl, MG_PSWEEP);
        int c = tl;
        for (int i = 1; i < nu; ++i) {
            const int dst = c == zl ? tl : zl;
            pass(l, c, 0, dst, MG_SWEEP);
            c = dst;
        }
        cur = c;
    }
    if (lw == 0) __syncthreads();
    const int n0 = P->lv[0].nx * P->lv[0].ny * P->lv[0].nz;
    for (int p = t; p < n0; p += NTT) out[p] = acc ? out[p] + S[cur + p] : S[cur + p];
}

void launch_mg_tail(int dim, const MgTail* P, const double* vin, double* out, int acc, hipStream_t s) {
    // 3-D passes hold more values per point (up to 8 coarse reads for each
    // of 7 interpolated points, all issued together): a quarter of the
    // threads, four times the registers each
    if (dim == 2)
        hipLaunchKernelGGL((k_mg_tail<2, MG_TAIL_NT>), dim3(1), dim3(MG_TAIL_NT), 0, s, P, vin, out, acc);
    else
        hipLaunchKernelGGL((k_mg_tail<3, MG_TAIL_NT / 4>), dim3(1), dim3(MG_TAIL_NT / 4), 0, s, P, vin, out, acc);
}

}  // namespace tgdk
