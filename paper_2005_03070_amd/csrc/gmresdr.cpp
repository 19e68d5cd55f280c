// Coarse-grid GMRES-DR(m,k) (Sec. 2.1; phase 1 of the Sec. 3 algorithm).
//
// The Krylov basis lives on the device; the Arnoldi steps are GPU kernels
// (stencil, then classical Gram-Schmidt with one re-orthogonalisation).  At
// the end of every cycle the (m+1) x m matrix Hbar comes to the host, where
// the float64 least-squares problem, the harmonic Ritz eigenproblem and the QR
// of the restart matrix are solved; the restart V_{k+1} = V_{m+1} P_{k+1} is a
// tall-skinny product on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <vector>

#include "dense.h"
#include "host.h"

namespace tgdk {

using cd = std::complex<double>;

struct Ritz {
    std::vector<cd> theta;
    std::vector<cd> G;  // column-major m x m
};

static int harmonic_ritz(int m, const std::vector<double>& Hbar, Ritz& out) {
    // Hbar row-major (m+1) x m
    std::vector<double> HmT((size_t)m * m), Hm((size_t)m * m);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < m; ++j) {
            Hm[(size_t)i * m + j] = Hbar[(size_t)i * m + j];
            HmT[(size_t)j * m + i] = Hbar[(size_t)i * m + j];
        }
    std::vector<int> piv(m);
    if (lu_factor(m, HmT.data(), piv.data()) != 0) return 1;
    std::vector<double> f(m, 0.0);
    f[m - 1] = 1.0;
    lu_solve(m, HmT.data(), piv.data(), f.data());
    const double h = Hbar[(size_t)m * m + (m - 1)];
    for (int i = 0; i < m; ++i) Hm[(size_t)i * m + (m - 1)] += h * h * f[i];
    out.theta.assign(m, 0.0);
    out.G.assign((size_t)m * m, 0.0);
    if (eig_real(m, Hm.data(), out.theta.data(), out.G.data()) != 0) return 2;
    return TGDK_OK;
}

static double eig_residual(int m, const std::vector<double>& Hbar, const Ritz& R, int i) {
    // ||Hbar g - rho [g; 0]|| with ||g|| = 1 and rho = g^H H_m g
    std::vector<cd> g(m);
    double nrm = 0.0;
    for (int r = 0; r < m; ++r) {
        g[r] = R.G[(size_t)i * m + r];
        nrm += std::norm(g[r]);
    }
    nrm = std::sqrt(nrm);
    for (auto& v : g) v /= nrm;
    std::vector<cd> Hg(m + 1, 0.0);
    for (int r = 0; r <= m; ++r)
        for (int c = 0; c < m; ++c) Hg[r] += Hbar[(size_t)r * m + c] * g[c];
    cd rho = 0.0;
    for (int r = 0; r < m; ++r) rho += std::conj(g[r]) * Hg[r];
    double s = 0.0;
    for (int r = 0; r <= m; ++r) s += std::norm(Hg[r] - (r < m ? rho * g[r] : cd(0.0)));
    return std::sqrt(s);
}

}  // namespace tgdk

using namespace tgdk;

extern "C" int tgdk_coarse_setup(tgdk_op op, const double* b, double* x, const tgdk_gmresdr_params* prm,
                                 tgdk_defl* out, tgdk_gmresdr_report* rep) {
    if (!op || !b || !x || !prm || !out) return fail(TGDK_E_INVALID, "NULL argument");
    const int m = prm->m, k = prm->k, nev = prm->nev;
    if (k < 1 || k >= m || m > MAXK || nev < 0 || nev > k)
        return fail(TGDK_E_INVALID, "need 1 <= k < m <= 256, nev <= k");
    const auto t0 = std::chrono::steady_clock::now();
    TGDK_HIP(hipSetDevice(op->ctx->device));
    tgdk_ctx ctx = op->ctx;
    hipStream_t s = ctx->stream;
    const long long n = op->N;
    const int tr = prm->transpose ? 1 : 0;
    const DevOp dop = make_devop(op, tr);
    const int maxcyc = prm->maxcyc > 0 ? prm->maxcyc : 300;
    const double anorm = op_norm1(op, tr);
    const bool verbose = getenv("TGDK_VERBOSE") != nullptr;

    double *V = nullptr, *Vt = nullptr, *w = nullptr, *Hd = nullptr, *dP = nullptr;
    const size_t hsz = (size_t)(m + 1) * m;
    auto cleanup = [&]() {
        if (V) (void)hipFree(V);
        if (Vt) (void)hipFree(Vt);
        if (w) (void)hipFree(w);
        if (Hd) (void)hipFree(Hd);
        if (dP) (void)hipFree(dP);
    };
    if (hipMalloc((void**)&V, sizeof(double) * n * (m + 1)) != hipSuccess ||
        hipMalloc((void**)&Vt, sizeof(double) * n * (m + 1)) != hipSuccess ||
        hipMalloc((void**)&w, sizeof(double) * n * (prm->precond ? 2 : 1)) != hipSuccess ||
        hipMalloc((void**)&Hd, sizeof(double) * (2 * hsz + m + 16)) != hipSuccess ||
        hipMalloc((void**)&dP, sizeof(double) * (m + 1) * (m + 2)) != hipSuccess) {
        cleanup();
        return fail(TGDK_E_NOMEM, "GMRES-DR workspace allocation failed");
    }
    double* H1 = Hd;
    double* H2 = Hd + hsz;
    double* Nd = Hd + 2 * hsz;
    double* dsc = Nd + m;  // 16 device scalars
    int rc = ctx->partial.ensure((size_t)gs_blocks(n) * (MAXK + 1) * sizeof(double));
    if (rc) {
        cleanup();
        return rc;
    }
    double* part = (double*)ctx->partial.p;
    unsigned* cnt = ctx->counters;

    // right preconditioning (Sec. 5, Example 5): the Arnoldi process runs on
    // A M^{-1}; x accumulates u and becomes M^{-1} u at the end
    double* pz = prm->precond ? w + n : nullptr;
    int prc = TGDK_OK;
    auto arnoldi = [&](int j0) {
        for (int j = j0; j < m; ++j) {
            if (pz) {
                if (!prc) prc = prm->precond(prm->precond_user, V + (size_t)j * n, pz, 1);
                launch_apply<double>(dop, pz, w, 1, op->tile_id[0], s);
            } else {
                launch_apply<double>(dop, V + (size_t)j * n, w, 1, op->tile_id[0], s);
            }
            launch_gs_dot(V, n, j + 1, w, n, H1 + (size_t)j * (m + 1), part, cnt, s);
            launch_gs_update_dot(V, n, j + 1, w, H1 + (size_t)j * (m + 1), n, H2 + (size_t)j * (m + 1), part, cnt, s);
            launch_gs_update_norm(V, n, j + 1, w, H2 + (size_t)j * (m + 1), n, Nd + j, part, cnt, s);
            launch_scale(w, V + (size_t)(j + 1) * n, Nd + j, n, s);
        }
    };
    std::vector<double> h1(hsz), h2(hsz), nrm(m);
    auto fetch_columns = [&](std::vector<double>& Hbar, int j0) -> int {
        TGDK_HIP(hipMemcpyAsync(h1.data(), H1, sizeof(double) * hsz, hipMemcpyDeviceToHost, s));
        TGDK_HIP(hipMemcpyAsync(h2.data(), H2, sizeof(double) * hsz, hipMemcpyDeviceToHost, s));
        TGDK_HIP(hipMemcpyAsync(nrm.data(), Nd, sizeof(double) * m, hipMemcpyDeviceToHost, s));
        TGDK_HIP(hipStreamSynchronize(s));
        for (int j = j0; j < m; ++j) {
            for (int i = 0; i <= j; ++i)
                Hbar[(size_t)i * m + j] = h1[(size_t)j * (m + 1) + i] + h2[(size_t)j * (m + 1) + i];
            Hbar[(size_t)(j + 1) * m + j] = nrm[j];
        }
        return TGDK_OK;
    };

    // cycle 1: GMRES(m) from x = 0
    TGDK_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, s));
    launch_norm2(b, n, dsc, part, cnt, s);
    double beta = 0.0;
    TGDK_HIP(hipMemcpyAsync(&beta, dsc, sizeof(double), hipMemcpyDeviceToHost, s));
    TGDK_HIP(hipStreamSynchronize(s));
    if (!(beta > 0.0) || !std::isfinite(beta)) {
        cleanup();
        return fail(beta == 0.0 ? TGDK_E_INVALID : TGDK_E_NONFINITE, "coarse right-hand side is zero or not finite");
    }
    const double bnorm = beta;
    launch_scale(b, V, dsc, n, s);
    arnoldi(0);
    std::vector<double> Hbar(hsz, 0.0), c(m + 1, 0.0), y(m), q(m + 1);
    if ((rc = fetch_columns(Hbar, 0))) {
        cleanup();
        return rc;
    }
    c[0] = beta;
    long long mvps = m;
    int cyc = 0, nconv = 0, kk = 0;
    std::vector<int> chosen;
    std::vector<double> dbg_prevH, dbg_prevQ, dbg_prevc;
    Ritz R;
    double lin = 0.0;
    double* W = nullptr;
    for (cyc = 1; cyc <= maxcyc; ++cyc) {
        lstsq(m + 1, m, Hbar.data(), c.data(), y.data(), q.data());
        TGDK_HIP(hipMemcpyAsync(dP, y.data(), sizeof(double) * m, hipMemcpyHostToDevice, s));
        launch_vmul_add(V, n, m, dP, x, n, s);
        lin = 0.0;
        for (double v : q) lin += v * v;
        lin = std::sqrt(lin);
        if ((rc = harmonic_ritz(m, Hbar, R))) {
            const char* dump = getenv("TGDK_DEBUG_DUMP");
            if (dump) {
                FILE* f = fopen(dump, "w");
                if (f) {
                    fprintf(f, "%d %d %d %d\n", m, cyc, rc, kk);
                    for (double v : Hbar) fprintf(f, "%.17g\n", v);
                    for (double v : dbg_prevH) fprintf(f, "%.17g\n", v);
                    for (double v : dbg_prevQ) fprintf(f, "%.17g\n", v);
                    for (double v : dbg_prevc) fprintf(f, "%.17g\n", v);
                    fclose(f);
                }
            }
            cleanup();
            return fail(TGDK_E_SINGULAR, rc == 1 ? "harmonic Ritz step: H_m is singular"
                                                 : "harmonic Ritz step: QR iteration did not converge");
        }
        chosen = select_smallest(R.theta, k);
        nconv = 0;
        double worst = 0.0;
        for (int i = 0; i < (int)chosen.size() && i < nev; ++i) {
            const double er = eig_residual(m, Hbar, R, chosen[i]) / anorm;
            worst = std::max(worst, er);
            if (er <= prm->rtolev) ++nconv;
        }
        const bool done = lin <= prm->rtol * bnorm && nconv >= nev;
        if (verbose) {
            double orth = 0.0;
            if (cyc % 5 == 1 || done) {  // loss of orthogonality of the basis
                std::vector<double> G((size_t)(m + 1) * (m + 1));
                double* dG = nullptr;
                if (hipMalloc((void**)&dG, sizeof(double) * G.size()) == hipSuccess &&
                    ctx->partial.ensure(gram_partial_bytes(n, m + 1, m + 1)) == TGDK_OK) {
                    launch_gram(V, 0, n, m + 1, V, 0, n, m + 1, n, dG, (double*)ctx->partial.p, ctx->counters, s);
                    (void)hipMemcpy(G.data(), dG, sizeof(double) * G.size(), hipMemcpyDeviceToHost);
                    for (int i = 0; i <= m; ++i)
                        for (int j = 0; j <= m; ++j)
                            orth = std::max(orth, std::fabs(G[(size_t)i * (m + 1) + j] - (i == j ? 1.0 : 0.0)));
                    (void)hipFree(dG);
                    (void)ctx->partial.ensure((size_t)gs_blocks(n) * (MAXK + 1) * sizeof(double));
                    part = (double*)ctx->partial.p;
                }
            }
            fprintf(stderr, "[tgdk] gmres-dr cycle %d lin %.3e nconv %d worst %.3e kk %d orth %.1e\n", cyc,
                    lin / bnorm, nconv, worst, (int)chosen.size(), orth);
        }
        // real basis of the chosen vectors, then P_{k+1} = qr([G 0; q])
        std::vector<std::vector<double>> cols;
        for (size_t ii = 0; ii < chosen.size();) {
            const int a = chosen[ii];
            const bool cp = ii + 1 < chosen.size() &&
                            std::fabs(R.theta[a].imag()) > 1e-10 * std::max(std::abs(R.theta[a]), 1e-300);
            std::vector<double> re(m), im(m);
            for (int r = 0; r < m; ++r) {
                re[r] = R.G[(size_t)a * m + r].real();
                im[r] = R.G[(size_t)a * m + r].imag();
            }
            cols.push_back(re);
            if (cp) {
                cols.push_back(im);
                ii += 2;
            } else {
                ii += 1;
            }
        }
        kk = (int)cols.size();
        std::vector<double> P((size_t)(m + 1) * (kk + 1), 0.0), Q((size_t)(m + 1) * (kk + 1)), Rr((size_t)(kk + 1) * (kk + 1));
        for (int cidx = 0; cidx < kk; ++cidx)
            for (int r = 0; r < m; ++r) P[(size_t)r * (kk + 1) + cidx] = cols[cidx][r];
        // only the direction of q enters P_{k+1}; once the coarse system has
        // converged q keeps shrinking toward the subnormal range, so scale it
        double qmax = 0.0;
        for (double v : q) qmax = std::max(qmax, std::fabs(v));
        for (int r = 0; r <= m; ++r) P[(size_t)r * (kk + 1) + kk] = qmax > 0.0 ? q[r] / qmax : 0.0;
        householder_qr(m + 1, kk + 1, P.data(), Q.data(), Rr.data());
        dbg_prevH = Hbar;
        dbg_prevQ = Q;
        dbg_prevc = c;
        std::vector<double> Qc((size_t)(m + 1) * (kk + 1));  // column-major for the device
        for (int r = 0; r <= m; ++r)
            for (int cidx = 0; cidx <= kk; ++cidx) Qc[(size_t)cidx * (m + 1) + r] = Q[(size_t)r * (kk + 1) + cidx];
        TGDK_HIP(hipMemcpyAsync(dP, Qc.data(), sizeof(double) * Qc.size(), hipMemcpyHostToDevice, s));
        launch_vmul(V, n, m + 1, dP, kk + 1, Vt, n, n, s);
        if (done || cyc == maxcyc) {
            if (hipMalloc((void**)&W, sizeof(double) * n * kk) != hipSuccess) {
                cleanup();
                return fail(TGDK_E_NOMEM, "basis allocation failed");
            }
            TGDK_HIP(hipMemcpyAsync(W, Vt, sizeof(double) * n * kk, hipMemcpyDeviceToDevice, s));
            TGDK_HIP(hipStreamSynchronize(s));
            break;
        }
        // Hbar_k = Q^T Hbar Q[:m, :kk];  c = Q^T q
        std::vector<double> T((size_t)(m + 1) * kk, 0.0), Hn(hsz, 0.0), cn(m + 1, 0.0);
        for (int r = 0; r <= m; ++r)
            for (int cidx = 0; cidx < kk; ++cidx) {
                double sacc = 0.0;
                for (int l = 0; l < m; ++l) sacc += Hbar[(size_t)r * m + l] * Q[(size_t)l * (kk + 1) + cidx];
                T[(size_t)r * kk + cidx] = sacc;
            }
        for (int i = 0; i <= kk; ++i) {
            for (int cidx = 0; cidx < kk; ++cidx) {
                double sacc = 0.0;
                for (int r = 0; r <= m; ++r) sacc += Q[(size_t)r * (kk + 1) + i] * T[(size_t)r * kk + cidx];
                Hn[(size_t)i * m + cidx] = sacc;
            }
            double sc = 0.0;
            for (int r = 0; r <= m; ++r) sc += Q[(size_t)r * (kk + 1) + i] * q[r];
            cn[i] = sc;
        }
        std::swap(V, Vt);
        // re-orthogonalise v_{k+1} against v_1..v_k, then continue Arnoldi
        double* vk = V + (size_t)kk * n;
        launch_gs_dot(V, n, kk, vk, n, H1, part, cnt, s);  // column 0 of H1/H2 is scratch here
        launch_gs_update_dot(V, n, kk, vk, H1, n, H2, part, cnt, s);
        launch_gs_update_norm(V, n, kk, vk, H2, n, dsc + 2, part, cnt, s);
        launch_scale(vk, vk, dsc + 2, n, s);
        arnoldi(kk);
        mvps += m - kk;
        Hbar = Hn;
        c = cn;
        if ((rc = fetch_columns(Hbar, kk))) {
            cleanup();
            return rc;
        }
    }
    if (cyc > maxcyc) cyc = maxcyc;
    if (!rc && prc) rc = prc;
    if (!rc && pz) {  // x = M^{-1} u
        if ((rc = prm->precond(prm->precond_user, x, pz, 1)) == TGDK_OK)
            TGDK_HIP(hipMemcpyAsync(x, pz, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    }
    if (rc) {
        cleanup();
        if (W) (void)hipFree(W);
        return rc;
    }
    // final true residual of the coarse solution: ||A x - b||
    launch_apply<double>(dop, x, w, 1, op->tile_id[0], s);
    const double one = 1.0;
    TGDK_HIP(hipMemcpyAsync(dsc + 3, &one, sizeof(double), hipMemcpyHostToDevice, s));
    launch_gs_update_norm(b, n, 1, w, dsc + 3, n, dsc + 4, part, cnt, s);
    double resn = 0.0;
    TGDK_HIP(hipMemcpyAsync(&resn, dsc + 4, sizeof(double), hipMemcpyDeviceToHost, s));
    TGDK_HIP(hipStreamSynchronize(s));
    cleanup();
    tgdk_defl d = nullptr;
    rc = defl_finish(op, tr, W, kk, TGDK_F64, &d, TGDK_PROJ_GALERKIN);
    if (rc) {
        (void)hipFree(W);
        return rc;
    }
    *out = d;
    if (rep) {
        memset(rep, 0, sizeof(*rep));
        rep->cycles = cyc;
        rep->nconv = nconv;
        rep->k_out = kk;
        rep->mvps = mvps;
        rep->relres = resn / bnorm;
        for (size_t i = 0; i < chosen.size() && i <= (size_t)MAXK; ++i) {
            rep->theta_re[i] = R.theta[chosen[i]].real();
            rep->theta_im[i] = R.theta[chosen[i]].imag();
            rep->eigres[i] = eig_residual(m, Hbar, R, chosen[i]) / anorm;
        }
        rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    const bool converged = (nconv >= nev) && (lin <= prm->rtol * bnorm);
    return converged ? TGDK_OK : TGDK_NOT_CONVERGED;
}
