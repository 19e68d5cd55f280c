// Arnoldi-E(m,k): improvement of a deflation space's approximate eigenvectors
// on its own grid (step 2 of the Two-grid Deflated GMRES and BiCGStab boxes,
// Sec. 3 and 4.1; Sec. 2.3).
//
// The basis Q and W = A Q live on the device.  A cycle runs m - k Arnoldi
// steps (stencil, classical Gram-Schmidt with one re-orthogonalisation) from
// the leading unconverged approximate eigenvector, keeping every A q_j, then
// appends the kept vectors (Gram-Schmidt against the basis; the host drops a
// vector that lost all but 1e-8 of its norm) and applies A to them in one
// multi-vector stencil launch.  The Rayleigh quotient B = Q^T W comes to the
// host in 64 x 64 Gram blocks (matrix cores); its eigenproblem and the choice
// of the kept pairs are solved there.  The kept vectors Y = Q G, A Y = W G and
// the residual block R = A Y - Y M (M the real block form of the kept values)
// are tall-skinny products on the device; the residual norms are the
// diagonal of R^T R (explicit, so small residuals do not cancel).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "dense.h"
#include "host.h"

namespace tgdk {

using cd = std::complex<double>;

namespace {

// G (p x q, row-major, host) = A^T B for n-row column-major blocks, in
// 64 x 64 pieces (the Gram kernel's limit).
int gram_host(tgdk_ctx ctx, const double* A, int p, const double* B, int q, long long n, double* dG,
              std::vector<double>& G) {
    hipStream_t s = ctx->stream;
    G.assign((size_t)p * q, 0.0);
    std::vector<double> blk(64 * 64);
    int rc = ctx->partial.ensure((size_t)gram_blocks(n) * 64 * 64 * sizeof(double));
    if (rc) return rc;
    for (int i0 = 0; i0 < p; i0 += 64)
        for (int j0 = 0; j0 < q; j0 += 64) {
            const int pi = std::min(64, p - i0), qj = std::min(64, q - j0);
            launch_gram(A + (size_t)i0 * n, 0, n, pi, B + (size_t)j0 * n, 0, n, qj, n, dG,
                        (double*)ctx->partial.p, ctx->counters, s);
            TGDK_HIP(hipMemcpyAsync(blk.data(), dG, sizeof(double) * pi * qj, hipMemcpyDeviceToHost, s));
            TGDK_HIP(hipStreamSynchronize(s));
            for (int i = 0; i < pi; ++i)
                for (int j = 0; j < qj; ++j) G[(size_t)(i0 + i) * q + j0 + j] = blk[(size_t)i * qj + j];
        }
    return TGDK_OK;
}

// The kept Ritz pairs of one Rayleigh-Ritz step.
struct Kept {
    std::vector<cd> theta;     // all Ritz values
    std::vector<int> chosen;   // kept, in keeping order (a pair: + imaginary part first)
    std::vector<int> col;      // chosen[i] -> its first real column
    int kk = 0;                // real columns
    std::vector<double> res;   // residual norm per chosen entry (relative to ||A||_1)
};

struct Work {
    tgdk_ctx ctx;
    long long n;
    double anorm;
    double *Q, *W, *Y, *AY, *T, *R;  // device
    double *dG, *dC, *dM;            // device small matrices
};

// Rayleigh-Ritz on range(Q) (ncol orthonormal columns, W = A Q): the k kept
// pairs, Y = Q Gr (their real basis) and the residual norms.
int rayleigh_ritz(Work& w, int ncol, int k, Kept& out) {
    hipStream_t s = w.ctx->stream;
    const long long n = w.n;
    std::vector<double> B;
    int rc = gram_host(w.ctx, w.Q, ncol, w.W, ncol, n, w.dG, B);
    if (rc) return rc;
    std::vector<cd> th(ncol), G((size_t)ncol * ncol);
    if (eig_real(ncol, B.data(), th.data(), G.data()) != 0)
        return fail(TGDK_E_SINGULAR, "Rayleigh-Ritz eigenproblem failed");
    std::vector<int> chosen = select_smallest(th, k);
    // real basis columns and the real block form M (column-major kk x kk)
    const int nch = (int)chosen.size();
    std::vector<int> col(nch);
    std::vector<std::vector<double>> cols;
    // (first column, theta index of the pair's + member) for a pair; (column, -1 - theta index) for a real value
    std::vector<std::pair<int, int>> blocks;
    for (int i = 0; i < nch;) {
        const int a = chosen[i];
        // a complex value (as select_smallest decides) is followed by its partner
        const bool cplx = i + 1 < nch && std::fabs(th[a].imag()) > 1e-10 * std::max(std::abs(th[a]), 1e-300);
        std::vector<double> re(ncol), im(ncol);
        for (int r = 0; r < ncol; ++r) {
            re[r] = G[(size_t)a * ncol + r].real();
            im[r] = G[(size_t)a * ncol + r].imag();
        }
        if (cplx) {
            col[i] = col[i + 1] = (int)cols.size();
            blocks.push_back({(int)cols.size(), a});
            cols.push_back(re);
            cols.push_back(im);
            i += 2;
        } else {
            col[i] = (int)cols.size();
            blocks.push_back({(int)cols.size(), -1 - a});
            cols.push_back(re);
            i += 1;
        }
    }
    const int kk = (int)cols.size();
    std::vector<double> Gr((size_t)ncol * kk), M((size_t)kk * kk, 0.0);
    for (int c = 0; c < kk; ++c)
        for (int r = 0; r < ncol; ++r) Gr[(size_t)c * ncol + r] = cols[c][r];
    for (const auto& bl : blocks) {
        const int c = bl.first;
        if (bl.second >= 0) {  // y = yr + i yi, A yr = tr yr - ti yi, A yi = ti yr + tr yi
            const double tr = th[bl.second].real(), ti = th[bl.second].imag();
            M[(size_t)c * kk + c] = tr;
            M[(size_t)c * kk + c + 1] = -ti;
            M[(size_t)(c + 1) * kk + c] = ti;
            M[(size_t)(c + 1) * kk + c + 1] = tr;
        } else {
            M[(size_t)c * kk + c] = th[-1 - bl.second].real();
        }
    }
    TGDK_HIP(hipMemcpyAsync(w.dC, Gr.data(), sizeof(double) * Gr.size(), hipMemcpyHostToDevice, s));
    TGDK_HIP(hipMemcpyAsync(w.dM, M.data(), sizeof(double) * M.size(), hipMemcpyHostToDevice, s));
    launch_vmul(w.Q, n, ncol, w.dC, kk, w.Y, n, n, s);
    launch_vmul(w.W, n, ncol, w.dC, kk, w.AY, n, n, s);
    launch_vmul(w.Y, n, kk, w.dM, kk, w.T, n, n, s);
    launch_sub(w.AY, w.T, w.R, n * kk, s);
    TGDK_HIP(hipGetLastError());
    std::vector<double> RR;
    if ((rc = gram_host(w.ctx, w.R, kk, w.R, kk, n, w.dG, RR))) return rc;
    std::vector<double> cres(kk), gnorm(kk);
    for (int c = 0; c < kk; ++c) {
        double g2 = 0.0;
        for (int r = 0; r < ncol; ++r) g2 += Gr[(size_t)c * ncol + r] * Gr[(size_t)c * ncol + r];
        gnorm[c] = g2;
        cres[c] = std::max(RR[(size_t)c * kk + c], 0.0);
    }
    out.theta = th;
    out.chosen = chosen;
    out.col = col;
    out.kk = kk;
    out.res.assign(nch, 0.0);
    for (const auto& bl : blocks) {
        const int c = bl.first;
        const bool pair = bl.second >= 0;
        const double num = pair ? cres[c] + cres[c + 1] : cres[c];
        const double den = pair ? gnorm[c] + gnorm[c + 1] : gnorm[c];
        const double r = std::sqrt(num / den) / w.anorm;
        for (int i = 0; i < nch; ++i)
            if (col[i] == c) out.res[i] = r;
    }
    return TGDK_OK;
}

}  // namespace

}  // namespace tgdk

using namespace tgdk;

extern "C" int tgdk_defl_improve(tgdk_defl in, const tgdk_arnoldie_params* prm, int store_dtype, tgdk_defl* out,
                                 tgdk_arnoldie_report* rep) {
    if (!in || !prm || !out) return fail(TGDK_E_INVALID, "NULL argument");
    if (in->precond) return fail(TGDK_E_INVALID, "improve the Galerkin space, then precondition it");
    const int k = in->k, m = prm->m;
    if (m <= k || m > MAXK) return fail(TGDK_E_INVALID, "need k < m <= 256");
    if (prm->nev < 0 || prm->nev > k || prm->maxcyc < 0 || !(prm->tol > 0.0))
        return fail(TGDK_E_INVALID, "need 0 <= nev <= k, maxcyc >= 0, tol > 0");
    if (store_dtype != TGDK_F64 && store_dtype != TGDK_F32) return fail(TGDK_E_INVALID, "store dtype");
    const auto t0 = std::chrono::steady_clock::now();
    tgdk_op op = in->op;
    tgdk_ctx ctx = op->ctx;
    TGDK_HIP(hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    const long long n = op->N;
    const int tr = in->transpose;
    const DevOp dop = make_devop(op, tr);
    const int nev = prm->nev;
    const int cq = m + 2, cy = k + 2;  // column capacities of Q, W and of the kept blocks
    // device memory: Q, W (n x cq), Y, AY, T, R (n x cy), w (n), small matrices
    const size_t vec = (size_t)n;
    double* base = nullptr;
    const size_t nd = vec * (2 * (size_t)cq + 4 * (size_t)cy + 1) + 64 * 64 + (size_t)cq * cy + (size_t)cy * cy +
                      4 * (size_t)cq + 8;
    if (hipMalloc((void**)&base, nd * sizeof(double)) != hipSuccess)
        return fail(TGDK_E_NOMEM, "Arnoldi-E workspace allocation failed");
    Work w;
    w.ctx = ctx;
    w.n = n;
    w.anorm = op_norm1(op, tr);
    double* p = base;
    w.Q = p; p += vec * cq;
    w.W = p; p += vec * cq;
    w.Y = p; p += vec * cy;
    w.AY = p; p += vec * cy;
    w.T = p; p += vec * cy;
    w.R = p; p += vec * cy;
    double* wv = p; p += vec;
    w.dG = p; p += 64 * 64;
    w.dC = p; p += (size_t)cq * cy;
    w.dM = p; p += (size_t)cy * cy;
    double* dh1 = p; p += cq;
    double* dh2 = p; p += cq;
    double* dnrm = p; p += cq;
    double* dsc = p;  // [0]: ||z||^2 before, [1]: ||z|| after
    auto done = [&](int code) {
        (void)hipStreamSynchronize(s);
        (void)hipFree(base);
        return code;
    };
    // the partial sums of both the Gram-Schmidt and the 64 x 64 Gram kernels,
    // reserved once (a later growth would move the buffer under `part`)
    const size_t need = std::max((size_t)gs_blocks(n) * (MAXK + 1), (size_t)gram_blocks(n) * 64 * 64);
    int rc = ctx->partial.ensure(need * sizeof(double));
    if (rc) return done(rc);
    double* part = (double*)ctx->partial.p;
    // the space's vectors, their images and the first Rayleigh-Ritz step
    if (in->store == TGDK_F64)
        TGDK_HIP(hipMemcpyAsync(w.Q, in->V, sizeof(double) * vec * k, hipMemcpyDeviceToDevice, s));
    else
        launch_to_f64((const float*)in->V, w.Q, (long long)vec * k, s);
    launch_apply<double>(dop, w.Q, w.W, k, op->tile_id[0], s);
    long long mvps = k;
    int ncol = k, cycles = 0;
    Kept K;
    if ((rc = rayleigh_ritz(w, ncol, k, K))) return done(rc);
    std::vector<double> res_start(K.res.begin(), K.res.begin() + std::min<int>(nev, (int)K.res.size()));
    const int pk = m - k;  // Arnoldi steps per cycle
    auto lead_ok = [&](const Kept& kp) {
        for (int i = 0; i < nev && i < (int)kp.res.size(); ++i)
            if (!(kp.res[i] <= prm->tol)) return false;
        return true;
    };
    while (!lead_ok(K) && cycles < prm->maxcyc) {
        ++cycles;
        // start vector: the real column of the first unconverged leading pair
        int sidx = 0;
        while (sidx < nev - 1 && K.res[sidx] <= prm->tol) ++sidx;
        const int kk = K.kk;
        // the kept vectors Y = Q Gr move out of Q's way (into AY's buffer)
        TGDK_HIP(hipMemcpyAsync(w.AY, w.Y, sizeof(double) * vec * kk, hipMemcpyDeviceToDevice, s));
        const double* Z = w.AY;
        // q_0 = z_s / ||z_s|| (a Gram-Schmidt step against no columns gives the norm)
        TGDK_HIP(hipMemcpyAsync(wv, Z + (size_t)K.col[sidx] * vec, sizeof(double) * vec, hipMemcpyDeviceToDevice,
                                s));
        launch_gs_update_norm(w.Q, n, 0, wv, dh1, n, dnrm, part, ctx->counters, s);
        launch_scale(wv, w.Q, dnrm, n, s);
        // Arnoldi: pk steps, A q_j kept in W
        for (int j = 0; j < pk; ++j) {
            launch_apply<double>(dop, w.Q + (size_t)j * vec, wv, 1, op->tile_id[0], s);
            TGDK_HIP(hipMemcpyAsync(w.W + (size_t)j * vec, wv, sizeof(double) * vec, hipMemcpyDeviceToDevice, s));
            launch_gs_dot(w.Q, n, j + 1, wv, n, dh1, part, ctx->counters, s);
            launch_gs_update_dot(w.Q, n, j + 1, wv, dh1, n, dh2, part, ctx->counters, s);
            launch_gs_update_norm(w.Q, n, j + 1, wv, dh2, n, dnrm + 1 + j, part, ctx->counters, s);
            launch_scale(wv, w.Q + (size_t)(j + 1) * vec, dnrm + 1 + j, n, s);
        }
        TGDK_HIP(hipGetLastError());
        std::vector<double> nr(pk + 1);
        TGDK_HIP(hipMemcpyAsync(nr.data(), dnrm, sizeof(double) * (pk + 1), hipMemcpyDeviceToHost, s));
        TGDK_HIP(hipStreamSynchronize(s));
        if (!(nr[0] > 0.0)) return done(fail(TGDK_E_SINGULAR, "Arnoldi-E start vector is zero"));
        // Krylov columns: an invariant subspace ends the basis early (columns
        // 0 .. nk-1 then all have A q_j in W from the loop)
        int nk = pk + 1;
        for (int j = 0; j < pk; ++j)
            if (!(nr[1 + j] > 0.0)) {
                nk = j + 1;
                break;
            }
        const int from = nk == pk + 1 ? pk : nk;  // first column still without A q in W
        // append the kept vectors, orthonormalised against the basis
        int cur = nk;
        for (int c = 0; c < kk && cur < cq; ++c) {
            TGDK_HIP(hipMemcpyAsync(wv, Z + (size_t)c * vec, sizeof(double) * vec, hipMemcpyDeviceToDevice, s));
            launch_norm2(wv, n, dsc, part, ctx->counters, s);
            launch_gs_dot(w.Q, n, cur, wv, n, dh1, part, ctx->counters, s);
            launch_gs_update_dot(w.Q, n, cur, wv, dh1, n, dh2, part, ctx->counters, s);
            launch_gs_update_norm(w.Q, n, cur, wv, dh2, n, dsc + 1, part, ctx->counters, s);
            double sc[2];  // ||z|| before and after
            TGDK_HIP(hipMemcpyAsync(sc, dsc, sizeof(sc), hipMemcpyDeviceToHost, s));
            TGDK_HIP(hipStreamSynchronize(s));
            if (sc[1] > 1e-8 * sc[0]) {
                launch_scale(wv, w.Q + (size_t)cur * vec, dsc + 1, n, s);
                ++cur;
            }
        }
        // A on the last Krylov column and the appended ones, one launch
        if (cur > from)
            launch_apply<double>(dop, w.Q + (size_t)from * vec, w.W + (size_t)from * vec, cur - from,
                                 op->tile_id[0], s);
        TGDK_HIP(hipGetLastError());
        mvps += cur;  // one application per basis vector
        ncol = cur;
        if ((rc = rayleigh_ritz(w, ncol, k, K))) return done(rc);
    }
    // the improved space over an orthonormal basis of the kept span
    const int kk = K.kk;
    double* V64 = nullptr;
    if (hipMalloc((void**)&V64, sizeof(double) * vec * kk) != hipSuccess)
        return done(fail(TGDK_E_NOMEM, "Arnoldi-E output allocation failed"));
    TGDK_HIP(hipMemcpyAsync(V64, w.Y, sizeof(double) * vec * kk, hipMemcpyDeviceToDevice, s));
    if ((rc = cholqr2(ctx, V64, n, kk)) || (rc = defl_finish(op, tr, V64, kk, store_dtype, out, TGDK_PROJ_GALERKIN))) {
        (void)hipFree(V64);
        return done(rc);
    }
    if (rep) {
        memset(rep, 0, sizeof(*rep));
        rep->cycles = cycles;
        rep->k_out = kk;
        rep->mvps = mvps;
        int nconv = 0;
        for (int i = 0; i < nev && i < (int)K.res.size(); ++i) nconv += K.res[i] <= prm->tol;
        rep->nconv = nconv;
        for (int i = 0; i < (int)K.chosen.size() && i <= TGDK_MAX_DEFL; ++i) {
            rep->theta_re[i] = K.theta[K.chosen[i]].real();
            rep->theta_im[i] = K.theta[K.chosen[i]].imag();
            rep->eigres[i] = K.res[i];
        }
        for (int i = 0; i < (int)res_start.size(); ++i) rep->eigres_start[i] = res_start[i];
        rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return done(TGDK_OK);
}
