// Tall-skinny kernels: Gram products A^T B, V Y products, and the classical
// Gram-Schmidt steps of the Arnoldi process.  All reductions over the long
// dimension are deterministic: per-block partials, then one workgroup per
// value sums them in a fixed order (k_sum_partials).
#include "device_common.h"
#include "launch.h"

namespace tgdk {

constexpr int GS_ROWS_PER_BLOCK = NT;  // rows per block before the cap (grid-strided beyond)
constexpr int GS_MAX_BLOCKS = 1024;  // measured best on 1M rows x 25 columns (4 rows per thread)

int gs_blocks(long long n) {
    long long b = (n + GS_ROWS_PER_BLOCK - 1) / GS_ROWS_PER_BLOCK;
    if (b > GS_MAX_BLOCKS) b = GS_MAX_BLOCKS;
    if (b < 1) b = 1;
    return (int)b;
}

// Sums value i of per-block partials (partial[b * pstride + i], b < nblocks)
// in a fixed order: one workgroup per value, threads take blocks t, t + NT,
// ..., then the block combine.  out[i] = sum (or sqrt(sum) if root).
__global__ __launch_bounds__(NT) void k_sum_partials(const double* __restrict__ partial, int nblocks,
                                                     long long pstride, double* __restrict__ out, int root) {
    __shared__ double sh[NWAVE];
    const int i = blockIdx.x;
    double a = 0.0;
#pragma unroll 8
    for (int b = threadIdx.x; b < nblocks; b += NT) a += partial[(long long)b * pstride + i];
    const double s = block_sum_one(a, sh);
    if (threadIdx.x == 0) out[i] = root ? sqrt(s) : s;
}

template <class T>
__device__ __forceinline__ double ld(const void* p, long long i) {
    return (double)reinterpret_cast<const T*>(p)[i];
}

// ------------------------------------------------------------- Gram A^T B
// Matrix-core (v_mfma_f64_16x16x4f64) Gram product G = A^T B, K = the long
// dimension n.  Operand layout of the instruction on gfx950 (one wave):
//   A-operand  lane l holds A[l % 16][l / 16]   (16 x 4)
//   B-operand  lane l holds B[l / 16][l % 16]   (4 x 16)
//   result     lane l, register r holds D[l / 16 + 4 r][l % 16]  (16 x 16)
// Each workgroup stages 64-row chunks of A and B in LDS (coalesced column
// loads, float32 inputs widened exactly), and its four waves accumulate the
// 16 x 16 output tiles over the chunk; per-workgroup partial tiles are summed
// in a fixed order by k_sum_partials (one workgroup per entry).
typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int GRAM_MAX = 64;   // p, q <= 64
constexpr int GRAM_ROWS = 32;  // rows staged per chunk (two 32 x 65 float64 LDS tiles)

int gram_blocks(long long n) {
    long long b = (n + 4 * GRAM_ROWS - 1) / (4 * GRAM_ROWS);
    if (b > 1024) b = 1024;
    if (b < 1) b = 1;
    return (int)b;
}

template <class TA, class TB>
__global__ __launch_bounds__(NT) void k_gram(const void* A_, long long lda, int p, const void* B_, long long ldb,
                                             int q, long long n, double* G, double* partial, unsigned* counter) {
    __shared__ double As[GRAM_ROWS][GRAM_MAX + 1];
    __shared__ double Bs[GRAM_ROWS][GRAM_MAX + 1];
    const TA* A = reinterpret_cast<const TA*>(A_);
    const TB* B = reinterpret_cast<const TB*>(B_);
    const int pt = (p + 15) / 16, qt = (q + 15) / 16, ntile = pt * qt;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    constexpr int MAXT = (GRAM_MAX / 16) * (GRAM_MAX / 16) / NWAVE;  // tiles per wave
    d4_t acc[MAXT];
#pragma unroll
    for (int i = 0; i < MAXT; ++i) acc[i] = d4_t{0.0, 0.0, 0.0, 0.0};
    const long long nchunk = (n + GRAM_ROWS - 1) / GRAM_ROWS;
    for (long long ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
        const long long r0 = ch * GRAM_ROWS;
        for (int idx = threadIdx.x; idx < GRAM_ROWS * GRAM_MAX; idx += NT) {
            const int rr = idx % GRAM_ROWS, col = idx / GRAM_ROWS;
            const long long g = r0 + rr;
            As[rr][col] = (g < n && col < p) ? (double)A[col * lda + g] : 0.0;
            Bs[rr][col] = (g < n && col < q) ? (double)B[col * ldb + g] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < MAXT; ++s) {
            const int tile = w + s * NWAVE;
            if (tile < ntile) {
                const int i0 = (tile / qt) * 16, j0 = (tile % qt) * 16;
                d4_t a = acc[s];
#pragma unroll
                for (int k4 = 0; k4 < GRAM_ROWS; k4 += 4) {
                    const double av = As[k4 + (lane >> 4)][i0 + (lane & 15)];
                    const double bv = Bs[k4 + (lane >> 4)][j0 + (lane & 15)];
                    a = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, a, 0, 0, 0);
                }
                acc[s] = a;
            }
        }
        __syncthreads();
    }
    // per-workgroup partial, row-major p x q
    const int npair = p * q;
#pragma unroll
    for (int s = 0; s < MAXT; ++s) {
        const int tile = w + s * NWAVE;
        if (tile < ntile) {
            const int i0 = (tile / qt) * 16, j0 = (tile % qt) * 16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + (lane >> 4) + 4 * r, j = j0 + (lane & 15);
                if (i < p && j < q) partial[(long long)blockIdx.x * npair + i * q + j] = acc[s][r];
            }
        }
    }
    (void)counter;
    (void)G;
}

// Entry e = i * qb + j of the summed partials goes to out[i * ldo + j] (a
// GRAM_MAX x GRAM_MAX block of a larger row-major Gram matrix).
__global__ __launch_bounds__(NT) void k_sum_gram_block(const double* __restrict__ partial, int nblocks,
                                                       int npair, int qb, double* __restrict__ out, int ldo) {
    __shared__ double sh[NWAVE];
    const int e = blockIdx.x;
    double a = 0.0;
#pragma unroll 8
    for (int b = threadIdx.x; b < nblocks; b += NT) a += partial[(long long)b * npair + e];
    const double v = block_sum_one(a, sh);
    if (threadIdx.x == 0) out[(long long)(e / qb) * ldo + e % qb] = v;
}

// G (p x q, row-major) = A^T B in blocks of at most GRAM_MAX x GRAM_MAX (the
// kernel's tile limit), each block's per-workgroup partials summed into its
// place in G; the blocks run one after another on the stream and share the
// partial workspace (gram_blocks(n) * GRAM_MAX^2 doubles suffice).
void launch_gram(const void* A, int atype, long long lda, int p, const void* B, int btype, long long ldb, int q,
                 long long n, double* G, double* partial, unsigned* counter, hipStream_t s) {
    const int nb = gram_blocks(n);
    const size_t ea = atype ? 4 : 8, eb = btype ? 4 : 8;
    for (int i0 = 0; i0 < p; i0 += GRAM_MAX)
        for (int j0 = 0; j0 < q; j0 += GRAM_MAX) {
            const int pb = p - i0 < GRAM_MAX ? p - i0 : GRAM_MAX, qb = q - j0 < GRAM_MAX ? q - j0 : GRAM_MAX;
            const void* Ab = (const char*)A + (size_t)i0 * lda * ea;
            const void* Bb = (const char*)B + (size_t)j0 * ldb * eb;
            if (atype == 0 && btype == 0)
                hipLaunchKernelGGL((k_gram<double, double>), dim3(nb), dim3(NT), 0, s, Ab, lda, pb, Bb, ldb, qb, n, G,
                                   partial, counter);
            else if (atype == 1 && btype == 1)
                hipLaunchKernelGGL((k_gram<float, float>), dim3(nb), dim3(NT), 0, s, Ab, lda, pb, Bb, ldb, qb, n, G,
                                   partial, counter);
            else if (atype == 1 && btype == 0)
                hipLaunchKernelGGL((k_gram<float, double>), dim3(nb), dim3(NT), 0, s, Ab, lda, pb, Bb, ldb, qb, n, G,
                                   partial, counter);
            else
                hipLaunchKernelGGL((k_gram<double, float>), dim3(nb), dim3(NT), 0, s, Ab, lda, pb, Bb, ldb, qb, n, G,
                                   partial, counter);
            hipLaunchKernelGGL(k_sum_gram_block, dim3(pb * qb), dim3(NT), 0, s, partial, nb, pb * qb, qb,
                               G + (size_t)i0 * q + j0, q);
        }
}

size_t gram_partial_bytes(long long n, int p, int q) {
    const int pb = p < GRAM_MAX ? p : GRAM_MAX, qb = q < GRAM_MAX ? q : GRAM_MAX;
    return (size_t)gram_blocks(n) * pb * qb * sizeof(double);
}

// ---------------------------------------------------------------- V * Y
// Out (n x q) = V (n x p) Y (p x q) on the matrix cores, computed as
// Out^T = Y^T V^T so that each lane's V load is one of 16 consecutive rows of
// a column (coalesced): B-operand lane l = V[r0 + l % 16][k0 + l / 16],
// A-operand lane l = Y[k0 + l / 16][j0 + l % 16], result lane l, register r =
// Out[r0 + l % 16][j0 + l / 16 + 4 r].  One wave owns 16 rows and all q
// columns (q <= 144), loading V once.
constexpr int VMUL_MAXQT = 9;

template <class TV>
__global__ __launch_bounds__(NT) void k_vmul(const TV* __restrict__ V, long long ldv, int p,
                                             const double* __restrict__ Y, int q, double* __restrict__ Out,
                                             long long ldo, long long n) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int qt = (q + 15) / 16;
    const long long nrt = (n + 15) / 16;
    for (long long rt = (long long)blockIdx.x * NWAVE + w; rt < nrt; rt += (long long)gridDim.x * NWAVE) {
        const long long r0 = rt * 16;
        const long long row = r0 + (lane & 15);
        d4_t acc[VMUL_MAXQT];
#pragma unroll
        for (int t = 0; t < VMUL_MAXQT; ++t) acc[t] = d4_t{0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < p; k0 += 4) {
            const int kc = k0 + (lane >> 4);
            const double bv = (row < n && kc < p) ? (double)V[kc * ldv + row] : 0.0;
#pragma unroll
            for (int t = 0; t < VMUL_MAXQT; ++t) {
                if (t < qt) {
                    const int jc = t * 16 + (lane & 15);
                    const double av = (kc < p && jc < q) ? Y[(long long)jc * p + kc] : 0.0;
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
                }
            }
        }
        if (row < n) {
#pragma unroll
            for (int t = 0; t < VMUL_MAXQT; ++t) {
                if (t < qt) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int jc = t * 16 + (lane >> 4) + 4 * r;
                        if (jc < q) Out[jc * ldo + row] = acc[t][r];
                    }
                }
            }
        }
    }
}

// Out = V Y in column blocks of at most 16 * VMUL_MAXQT (the kernel's limit):
// block j0 takes Y's columns j0.. (column-major, leading dimension p) and
// writes Out's.
void launch_vmul(const double* V, long long ldv, int p, const double* Y, int q, double* Out, long long ldo,
                 long long n, hipStream_t s) {
    long long nb = ((n + 15) / 16 + NWAVE - 1) / NWAVE;
    if (nb > 8192) nb = 8192;
    constexpr int QB = 16 * VMUL_MAXQT;
    for (int j0 = 0; j0 < q; j0 += QB) {
        const int qb = q - j0 < QB ? q - j0 : QB;
        hipLaunchKernelGGL(k_vmul<double>, dim3((int)nb), dim3(NT), 0, s, V, ldv, p, Y + (size_t)j0 * p, qb,
                           Out + (size_t)j0 * ldo, ldo, n);
    }
}

__global__ __launch_bounds__(NT) void k_vmul_add(const double* __restrict__ V, long long ldv, int p,
                                                 const double* __restrict__ y, double* __restrict__ x, long long n) {
    __shared__ double ys[MAXK + 1];
    for (int i = threadIdx.x; i < p; i += NT) ys[i] = y[i];
    __syncthreads();
    for (long long g = blockIdx.x * (long long)NT + threadIdx.x; g < n; g += (long long)gridDim.x * NT) {
        double a = 0.0;
        for (int i = 0; i < p; ++i) a += V[i * ldv + g] * ys[i];
        x[g] += a;
    }
}

void launch_vmul_add(const double* V, long long ldv, int p, const double* y, double* x, long long n,
                     hipStream_t s) {
    long long nb = (n + NT - 1) / NT;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_vmul_add, dim3((int)nb), dim3(NT), 0, s, V, ldv, p, y, x, n);
}

// ------------------------------------------------- Gram-Schmidt (Arnoldi)
// gs_blocks blocks of NT threads, rows grid-strided (4 rows per thread at 1M rows).
// MODE 0: hout = V^T w.  MODE 1: w -= V h, then hout = V^T w, fused per row:
// the row's V values are read for the update and again, from cache, for the
// dot products.  MODE 2: w -= V h, then hout[0] = ||w||.
template <int MODE>
__global__ __launch_bounds__(NT) void k_gs(const double* __restrict__ V, long long ldv, int p, double* w,
                                           const double* __restrict__ h, long long n, double* hout,
                                           double* partial, unsigned* counter) {
    __shared__ double sh[NWAVE * 16];
    __shared__ double hs[MAXK + 1];
    const long long stride = (long long)gridDim.x * NT;
    const long long g0 = blockIdx.x * (long long)NT + threadIdx.x;
    if (MODE >= 1)
        for (int i = threadIdx.x; i < p; i += NT) hs[i] = h[i];
    __syncthreads();
    const int pstride = MAXK + 1;
    if (MODE <= 1) {
        for (int c0 = 0; c0 < p; c0 += 16) {
            const int nc = p - c0 < 16 ? p - c0 : 16;
            double acc[16];
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) acc[jj] = 0.0;
            for (long long g = g0; g < n; g += stride) {
                double wv = w[g];
                if (MODE == 1 && c0 == 0) {
                    // update of this row before its first dot products
#pragma unroll 8
                    for (int i = 0; i < p; ++i) wv -= V[i * ldv + g] * hs[i];
                    w[g] = wv;
                }
                // unconditional loads (columns past p re-read column c0, a
                // cache hit, and are masked), so all 16 are in flight at once
#pragma unroll
                for (int jj = 0; jj < 16; ++jj) {
                    const double v = V[(long long)(jj < nc ? c0 + jj : c0) * ldv + g];
                    acc[jj] += jj < nc ? v * wv : 0.0;
                }
            }
            double tot;
            block_sum<16>(acc, sh, tot);
            if (threadIdx.x < 16 && c0 + threadIdx.x < p)
                partial[(long long)blockIdx.x * pstride + c0 + threadIdx.x] = tot;
        }
    } else {
        double acc[1] = {0.0};
        for (long long g = g0; g < n; g += stride) {
            double a = w[g];
#pragma unroll 8
            for (int i = 0; i < p; ++i) a -= V[i * ldv + g] * hs[i];
            if (p > 0) w[g] = a;
            acc[0] += a * a;
        }
        double tot;
        block_sum<1>(acc, sh, tot);
        if (threadIdx.x == 0) partial[(long long)blockIdx.x * pstride] = tot;
    }
    (void)counter;
    (void)hout;
}

// The same passes with the columns split over the waves, for p <= NW CPW
// (NW waves of 64 threads per workgroup): wave w holds columns w, w + NW, ...,
// w + NW (CPW - 1) of a 64-row block (64 consecutive rows per column load),
// so every pass reads V once and the row loop has no per-chunk reductions.
// The update w -= V h of a row needs all columns: the waves exchange their
// partial sums of V h through LDS (double-buffered, one barrier per row
// block; summed over the waves in order) and every wave forms the same
// updated rows (wave 0 stores them), whose dot products then use the V values
// already in registers.  The next row block's loads are issued before the
// barrier, which does not wait for them.  Columns past p are read at column 0
// (a cache hit) and masked.
template <int MODE, int CPW, int NW>
__global__ __launch_bounds__(64 * NW) void k_gsc(const double* __restrict__ V, long long ldv, int p, double* w,
                                                 const double* __restrict__ h, long long n,
                                                 double* __restrict__ partial) {
    __shared__ double xs[2][NW][64];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const double* vc[CPW];
    double hc[CPW];
    bool cok[CPW];
#pragma unroll
    for (int i = 0; i < CPW; ++i) {
        const int c = wv + NW * i;
        cok[i] = c < p;
        vc[i] = V + (long long)(cok[i] ? c : 0) * ldv;
        hc[i] = (MODE >= 1 && cok[i]) ? h[c] : 0.0;
    }
    double acc[CPW];
#pragma unroll
    for (int i = 0; i < CPW; ++i) acc[i] = 0.0;
    double nacc = 0.0;
    const long long nrb = (n + 63) / 64, step = gridDim.x;
    auto load = [&](long long rb, double(&dv)[CPW], double& dw) {
        long long row = rb * 64 + lane;
        if (row >= n) row = n - 1;
#pragma unroll
        for (int i = 0; i < CPW; ++i) dv[i] = vc[i][row];
        dw = w[row];
    };
    double vv[CPW], wr = 0.0;
#pragma unroll
    for (int i = 0; i < CPW; ++i) vv[i] = 0.0;
    long long rb = blockIdx.x;
    if (rb < nrb) load(rb, vv, wr);
    int par = 0;
    for (; rb < nrb; rb += step) {
        double nv[CPW], nw = 0.0;
#pragma unroll
        for (int i = 0; i < CPW; ++i) nv[i] = 0.0;
        if (rb + step < nrb) load(rb + step, nv, nw);
        const long long row = rb * 64 + lane;
        const bool ok = row < n;
        double x = wr;
        if (MODE >= 1) {
            double u = 0.0;
#pragma unroll
            for (int i = 0; i < CPW; ++i) u += cok[i] ? vv[i] * hc[i] : 0.0;
            xs[par][wv][lane] = u;
            __syncthreads();
            double t = xs[par][0][lane];
#pragma unroll
            for (int q = 1; q < NW; ++q) t += xs[par][q][lane];
            x = wr - t;
            if (wv == 0 && ok) w[row] = x;
            par ^= 1;
        }
        if (MODE <= 1) {
#pragma unroll
            for (int i = 0; i < CPW; ++i) acc[i] += (ok && cok[i]) ? vv[i] * x : 0.0;
        } else if (wv == 0) {
            nacc += ok ? x * x : 0.0;
        }
#pragma unroll
        for (int i = 0; i < CPW; ++i) vv[i] = nv[i];
        wr = nw;
    }
    const long long pstride = MAXK + 1;
    if (MODE <= 1) {
#pragma unroll
        for (int i = 0; i < CPW; ++i) {
            const double t = wave_sum(acc[i]);
            if (lane == 0 && cok[i]) partial[(long long)blockIdx.x * pstride + wv + NW * i] = t;
        }
    } else if (wv == 0) {
        const double t = wave_sum(nacc);
        if (lane == 0) partial[(long long)blockIdx.x * pstride] = t;
    }
}

// k_gsc for 1 <= p <= 128: 4 waves with 1 ... 16 columns each up to 64
// columns; beyond, 8 waves with 16 each in half as many workgroups (the same
// threads).  Returns the number of workgroups (of partials) launched, or 0 if
// p is out of range.
template <int MODE>
static int launch_gsc(const double* V, long long ldv, int p, double* w, const double* h, long long n,
                      double* partial, int nb, hipStream_t s) {
    if (p < 1 || p > 8 * 16) return 0;
    const dim3 g(nb), b4(256);
    if (p <= 4)
        hipLaunchKernelGGL((k_gsc<MODE, 1, 4>), g, b4, 0, s, V, ldv, p, w, h, n, partial);
    else if (p <= 8)
        hipLaunchKernelGGL((k_gsc<MODE, 2, 4>), g, b4, 0, s, V, ldv, p, w, h, n, partial);
    else if (p <= 16)
        hipLaunchKernelGGL((k_gsc<MODE, 4, 4>), g, b4, 0, s, V, ldv, p, w, h, n, partial);
    else if (p <= 32)
        hipLaunchKernelGGL((k_gsc<MODE, 8, 4>), g, b4, 0, s, V, ldv, p, w, h, n, partial);
    else if (p <= 64)
        hipLaunchKernelGGL((k_gsc<MODE, 16, 4>), g, b4, 0, s, V, ldv, p, w, h, n, partial);
    else {
        nb = nb > 1 ? nb / 2 : 1;
        hipLaunchKernelGGL((k_gsc<MODE, 16, 8>), dim3(nb), dim3(512), 0, s, V, ldv, p, w, h, n, partial);
    }
    return nb;
}

void launch_gs_dot(const double* V, long long ldv, int p, const double* w, long long n, double* hout,
                   double* partial, unsigned* counter, hipStream_t s) {
    int nb = gs_blocks(n);
    if (const int used = launch_gsc<0>(V, ldv, p, const_cast<double*>(w), nullptr, n, partial, nb, s))
        nb = used;
    else
        hipLaunchKernelGGL((k_gs<0>), dim3(nb), dim3(NT), 0, s, V, ldv, p, const_cast<double*>(w),
                           (const double*)nullptr, n, hout, partial, counter);
    if (p > 0) hipLaunchKernelGGL(k_sum_partials, dim3(p), dim3(NT), 0, s, partial, nb, (long long)(MAXK + 1), hout, 0);
}
void launch_gs_update_dot(const double* V, long long ldv, int p, double* w, const double* h, long long n,
                          double* hout, double* partial, unsigned* counter, hipStream_t s) {
    int nb = gs_blocks(n);
    if (const int used = launch_gsc<1>(V, ldv, p, w, h, n, partial, nb, s))
        nb = used;
    else
        hipLaunchKernelGGL((k_gs<1>), dim3(nb), dim3(NT), 0, s, V, ldv, p, w, h, n, hout, partial, counter);
    if (p > 0) hipLaunchKernelGGL(k_sum_partials, dim3(p), dim3(NT), 0, s, partial, nb, (long long)(MAXK + 1), hout, 0);
}
void launch_gs_update_norm(const double* V, long long ldv, int p, double* w, const double* h, long long n,
                           double* nrm, double* partial, unsigned* counter, hipStream_t s) {
    int nb = gs_blocks(n);
    if (const int used = launch_gsc<2>(V, ldv, p, w, h, n, partial, nb, s))
        nb = used;
    else
        hipLaunchKernelGGL((k_gs<2>), dim3(nb), dim3(NT), 0, s, V, ldv, p, w, h, n, nrm, partial, counter);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(NT), 0, s, partial, nb, (long long)(MAXK + 1), nrm, 1);
}
void launch_norm2(const double* w, long long n, double* out, double* partial, unsigned* counter, hipStream_t s) {
    const int nb = gs_blocks(n);
    hipLaunchKernelGGL((k_gs<2>), dim3(nb), dim3(NT), 0, s, (const double*)nullptr, 0LL, 0,
                       const_cast<double*>(w), (const double*)nullptr, n, out, partial, counter);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(NT), 0, s, partial, nb, (long long)(MAXK + 1), out, 1);
}

__global__ void k_scale(const double* w, double* v, const double* __restrict__ nrm,
                        long long n) {
    const double s = *nrm;
    for (long long g = blockIdx.x * (long long)blockDim.x + threadIdx.x; g < n;
         g += (long long)gridDim.x * blockDim.x)
        v[g] = s > 0.0 ? w[g] / s : 0.0;
}
void launch_scale(const double* w, double* v, const double* nrm, long long n, hipStream_t s) {
    long long nb = (n + 255) / 256;
    if (nb > 8192) nb = 8192;
    hipLaunchKernelGGL(k_scale, dim3((int)nb), dim3(256), 0, s, w, v, nrm, n);
}

// c = a - b over n contiguous values (c may be b: each element is read
// before it is written by the same thread)
__global__ __launch_bounds__(NT) void k_sub(const double* __restrict__ a, const double* b, double* c, long long n) {
    for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT)
        c[i] = a[i] - b[i];
}

void launch_sub(const double* a, const double* b, double* c, long long n, hipStream_t s) {
    long long nb = (n + NT - 1) / NT;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_sub, dim3((int)nb), dim3(NT), 0, s, a, b, c, n);
}

// a += b over n values
__global__ __launch_bounds__(NT) void k_add(double* __restrict__ a, const double* __restrict__ b, long long n) {
    for (long long i = blockIdx.x * (long long)NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) a[i] += b[i];
}

void launch_add(double* a, const double* b, long long n, hipStream_t st) {
    long long nb = (n + NT - 1) / NT;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_add, dim3((int)nb), dim3(NT), 0, st, a, b, n);
}

}  // namespace tgdk
