// Small dense float64 linear algebra on the host: the k x k projection
// system, the Hessenberg least-squares problem and the harmonic Ritz
// eigenproblem of GMRES-DR.  Sizes are at most a few hundred, so plain
// textbook algorithms suffice:
//  - LU with partial pivoting (row interchanges recorded LAPACK-style);
//  - Cholesky G = R^T R;
//  - Householder QR (positive diagonal of R) and least squares via QR;
//  - eigenvalues and eigenvectors of a real matrix: Householder reduction to
//    Hessenberg form, shifted QR iteration in complex arithmetic to a complex
//    Schur form T = Z^H A Z (Wilkinson shifts, Givens bulge chasing), and
//    eigenvectors of T by back substitution, mapped back with Z.
#include "dense.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <numeric>
#include <vector>

namespace tgdk {

using cd = std::complex<double>;

// Smallest |theta| first; ties by real part, then positive imaginary part
// first; a kept complex value brings its conjugate partner along.
std::vector<int> select_smallest(const std::vector<std::complex<double>>& th, int k) {
    using cd = std::complex<double>;
    const int m = (int)th.size();
    auto is_cplx = [&](int i) { return std::fabs(th[i].imag()) > 1e-10 * std::max(std::abs(th[i]), 1e-300); };
    std::vector<int> order(m);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int a, int b) {
        const double aa = std::abs(th[a]), ab = std::abs(th[b]);
        if (aa != ab) return aa < ab;
        if (th[a].real() != th[b].real()) return th[a].real() < th[b].real();
        return th[a].imag() > th[b].imag();
    });
    std::vector<int> chosen;
    std::vector<char> used(m, 0);
    for (int i : order) {
        if ((int)chosen.size() >= k) break;
        if (used[i]) continue;
        if (is_cplx(i)) {
            int best = -1;
            double bd = INFINITY;
            for (int j = 0; j < m; ++j) {
                if (used[j] || j == i) continue;
                const double d = std::abs(th[j] - std::conj(th[i]));
                if (d < bd) {
                    bd = d;
                    best = j;
                }
            }
            int ip = i, jn = best;
            if (th[i].imag() < 0 && best >= 0) std::swap(ip, jn);
            chosen.push_back(ip);
            used[ip] = 1;
            if (jn >= 0) {
                chosen.push_back(jn);
                used[jn] = 1;
            }
        } else {
            chosen.push_back(i);
            used[i] = 1;
        }
    }
    return chosen;
}


int lu_factor(int n, double* A, int* piv) {
    int info = 0;
    for (int j = 0; j < n; ++j) {
        int p = j;
        double best = std::fabs(A[j * n + j]);
        for (int i = j + 1; i < n; ++i) {
            const double v = std::fabs(A[i * n + j]);
            if (v > best) {
                best = v;
                p = i;
            }
        }
        piv[j] = p;
        if (p != j)
            for (int c = 0; c < n; ++c) std::swap(A[j * n + c], A[p * n + c]);
        const double d = A[j * n + j];
        if (d == 0.0 || !std::isfinite(d)) {
            if (!info) info = j + 1;
            continue;
        }
        for (int i = j + 1; i < n; ++i) {
            const double l = A[i * n + j] / d;
            A[i * n + j] = l;
            for (int c = j + 1; c < n; ++c) A[i * n + c] -= l * A[j * n + c];
        }
    }
    return info;
}

void lu_solve(int n, const double* LU, const int* piv, double* b) {
    for (int i = 0; i < n; ++i)
        if (piv[i] != i) std::swap(b[i], b[piv[i]]);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j) b[i] -= LU[i * n + j] * b[j];
    for (int i = n - 1; i >= 0; --i) {
        for (int j = i + 1; j < n; ++j) b[i] -= LU[i * n + j] * b[j];
        b[i] /= LU[i * n + i];
    }
}

double cond_estimate_lu(int n, const double* LU) {
    double mx = 0.0, mn = INFINITY;
    for (int i = 0; i < n; ++i) {
        const double d = std::fabs(LU[i * n + i]);
        mx = std::max(mx, d);
        mn = std::min(mn, d);
    }
    return mn > 0 ? mx / mn : INFINITY;
}

int cholesky_upper(int n, double* G) {
    // G (row-major, symmetric) -> upper triangular R with G = R^T R; lower part zeroed.
    // A pivot below 64 eps of its diagonal entry (the column keeps less than
    // about 1.2e-7 of its norm outside the span of the earlier ones) counts
    // as rank deficient: exact duplicates leave a rounding-size positive
    // pivot, and a Cholesky QR of such a basis would not be orthonormal.
    for (int j = 0; j < n; ++j) {
        const double g0 = G[j * n + j];
        double d = g0;
        for (int k = 0; k < j; ++k) d -= G[k * n + j] * G[k * n + j];
        if (!(d > 64.0 * 2.220446049250313e-16 * g0) || !std::isfinite(d)) return j + 1;
        const double r = std::sqrt(d);
        G[j * n + j] = r;
        for (int c = j + 1; c < n; ++c) {
            double v = G[j * n + c];
            for (int k = 0; k < j; ++k) v -= G[k * n + j] * G[k * n + c];
            G[j * n + c] = v / r;
        }
        for (int i = j + 1; i < n; ++i) G[i * n + j] = 0.0;
    }
    return 0;
}

void upper_inverse(int n, const double* R, double* Rinv) {
    std::fill(Rinv, Rinv + (size_t)n * n, 0.0);
    for (int c = 0; c < n; ++c) {
        // solve R x = e_c
        for (int i = n - 1; i >= 0; --i) {
            double v = (i == c) ? 1.0 : 0.0;
            for (int j = i + 1; j < n; ++j) v -= R[i * n + j] * Rinv[j * n + c];
            Rinv[i * n + c] = v / R[i * n + i];
        }
    }
}

void householder_qr(int m, int n, const double* A, double* Q, double* R) {
    // A row-major m x n (m >= n).  Q row-major m x n with orthonormal columns,
    // R row-major n x n upper triangular with R_ii >= 0.
    // Reflectors are kept as unit vectors (beta = 2) and every norm is
    // formed after scaling by the largest magnitude, so columns of any size
    // (down to the subnormal range) neither overflow nor underflow.
    std::vector<double> W(A, A + (size_t)m * n);
    std::vector<std::vector<double>> vs;
    std::vector<double> betas;
    for (int j = 0; j < n; ++j) {
        std::vector<double> v(m, 0.0);
        double amax = 0.0;
        for (int i = j; i < m; ++i) amax = std::max(amax, std::fabs(W[i * n + j]));
        double beta = 0.0;
        if (amax > 0.0 && std::isfinite(amax)) {
            for (int i = j; i < m; ++i) v[i] = W[i * n + j] / amax;
            double nrm = 0.0;
            for (int i = j; i < m; ++i) nrm += v[i] * v[i];
            nrm = std::sqrt(nrm);
            const double alpha = (v[j] >= 0.0) ? -nrm : nrm;
            v[j] -= alpha;
            double vmax = 0.0;
            for (int i = j; i < m; ++i) vmax = std::max(vmax, std::fabs(v[i]));
            double vn = 0.0;
            for (int i = j; i < m; ++i) vn += (v[i] / vmax) * (v[i] / vmax);
            vn = vmax * std::sqrt(vn);
            if (vn > 0.0) {
                for (int i = j; i < m; ++i) v[i] /= vn;
                beta = 2.0;
                for (int c = j; c < n; ++c) {
                    double s = 0.0;
                    for (int i = j; i < m; ++i) s += v[i] * W[i * n + c];
                    s *= beta;
                    for (int i = j; i < m; ++i) W[i * n + c] -= s * v[i];
                }
            }
        }
        vs.push_back(v);
        betas.push_back(beta);
    }
    // R and sign fix
    std::vector<double> sgn(n, 1.0);
    for (int i = 0; i < n; ++i) {
        sgn[i] = (W[i * n + i] < 0.0) ? -1.0 : 1.0;
        for (int c = 0; c < n; ++c) R[i * n + c] = (c >= i) ? sgn[i] * W[i * n + c] : 0.0;
    }
    // Q = H_0 ... H_{n-1} [I_n; 0], columns scaled by sgn
    std::vector<double> Qf((size_t)m * n, 0.0);
    for (int i = 0; i < n; ++i) Qf[i * n + i] = 1.0;
    for (int j = n - 1; j >= 0; --j) {
        const std::vector<double>& v = vs[j];
        const double beta = betas[j];
        if (beta == 0.0) continue;
        for (int c = 0; c < n; ++c) {
            double s = 0.0;
            for (int i = j; i < m; ++i) s += v[i] * Qf[i * n + c];
            s *= beta;
            for (int i = j; i < m; ++i) Qf[i * n + c] -= s * v[i];
        }
    }
    for (int i = 0; i < m; ++i)
        for (int c = 0; c < n; ++c) Q[i * n + c] = Qf[i * n + c] * sgn[c];
}

int lstsq(int m, int n, const double* A, const double* b, double* x, double* resid) {
    std::vector<double> Q((size_t)m * n), R((size_t)n * n);
    householder_qr(m, n, A, Q.data(), R.data());
    std::vector<double> qtb(n, 0.0);
    for (int c = 0; c < n; ++c) {
        double s = 0.0;
        for (int i = 0; i < m; ++i) s += Q[i * n + c] * b[i];
        qtb[c] = s;
    }
    int info = 0;
    for (int i = n - 1; i >= 0; --i) {
        double v = qtb[i];
        for (int j = i + 1; j < n; ++j) v -= R[i * n + j] * x[j];
        if (R[i * n + i] == 0.0) {
            info = i + 1;
            x[i] = 0.0;
        } else {
            x[i] = v / R[i * n + i];
        }
    }
    if (resid) {
        for (int i = 0; i < m; ++i) {
            double s = b[i];
            for (int j = 0; j < n; ++j) s -= A[i * n + j] * x[j];
            resid[i] = s;
        }
    }
    return info;
}

// ---------------------------------------------------------- eigenproblem
static void hessenberg_reduce(int n, std::vector<cd>& H, std::vector<cd>& Z) {
    // H row-major n x n, Z accumulates the unitary transforms (H = Z^H A Z).
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Z[i * n + j] = (i == j) ? 1.0 : 0.0;
    for (int k = 0; k + 2 < n; ++k) {
        double nrm = 0.0;
        for (int i = k + 1; i < n; ++i) nrm += std::norm(H[i * n + k]);
        nrm = std::sqrt(nrm);
        if (nrm == 0.0) continue;
        std::vector<cd> v(n, 0.0);
        const cd a = H[(k + 1) * n + k];
        const cd phase = (std::abs(a) > 0.0) ? a / std::abs(a) : cd(1.0);
        for (int i = k + 1; i < n; ++i) v[i] = H[i * n + k];
        v[k + 1] += phase * nrm;
        double vn = 0.0;
        for (int i = k + 1; i < n; ++i) vn += std::norm(v[i]);
        if (vn == 0.0) continue;
        const double beta = 2.0 / vn;
        // H <- (I - beta v v^H) H
        for (int c = 0; c < n; ++c) {
            cd s = 0.0;
            for (int i = k + 1; i < n; ++i) s += std::conj(v[i]) * H[i * n + c];
            s *= beta;
            for (int i = k + 1; i < n; ++i) H[i * n + c] -= s * v[i];
        }
        // H <- H (I - beta v v^H);  Z <- Z (I - beta v v^H)
        for (int r = 0; r < n; ++r) {
            cd s = 0.0, sz = 0.0;
            for (int i = k + 1; i < n; ++i) {
                s += H[r * n + i] * v[i];
                sz += Z[r * n + i] * v[i];
            }
            s *= beta;
            sz *= beta;
            for (int i = k + 1; i < n; ++i) {
                H[r * n + i] -= s * std::conj(v[i]);
                Z[r * n + i] -= sz * std::conj(v[i]);
            }
        }
        for (int i = k + 2; i < n; ++i) H[i * n + k] = 0.0;
    }
}

// Givens rotation G = [c s; -conj(s) c] with G [x; y] = [r; 0], c real.
static void givens(cd x, cd y, double& c, cd& s) {
    const double ax = std::abs(x), ay = std::abs(y);
    if (ay == 0.0) {
        c = 1.0;
        s = 0.0;
        return;
    }
    if (ax == 0.0) {
        c = 0.0;
        s = std::conj(y) / ay;
        return;
    }
    const double nrm = std::hypot(ax, ay);
    c = ax / nrm;
    s = (x / ax) * std::conj(y) / nrm;
}

int eig_real(int n, const double* A, cd* w, cd* X) {
    std::vector<cd> H((size_t)n * n), Z((size_t)n * n);
    for (int i = 0; i < n * n; ++i) H[i] = A[i];
    hessenberg_reduce(n, H, Z);
    double anorm = 0.0;
    for (int i = 0; i < n * n; ++i) anorm = std::max(anorm, std::abs(H[i]));
    const double eps = 2.220446049250313e-16;
    int hi = n - 1;
    int iter = 0, total = 0;
    while (hi > 0) {
        int l = hi;
        while (l > 0) {
            const double sub = std::abs(H[l * n + l - 1]);
            double ref = std::abs(H[(l - 1) * n + l - 1]) + std::abs(H[l * n + l]);
            if (ref == 0.0) ref = anorm;
            if (sub <= eps * ref) {
                H[l * n + l - 1] = 0.0;
                break;
            }
            --l;
        }
        if (l == hi) {
            --hi;
            iter = 0;
            continue;
        }
        if (++total > 100 * n) return 1;
        ++iter;
        // Wilkinson shift from the trailing 2x2 block of the active part
        const cd a = H[(hi - 1) * n + hi - 1], b = H[(hi - 1) * n + hi];
        const cd c = H[hi * n + hi - 1], d = H[hi * n + hi];
        cd mu;
        if (iter % 11 == 10) {
            mu = d + cd(std::abs(c), 0.0);  // exceptional shift
        } else {
            const cd tr2 = 0.5 * (a + d);
            const cd disc = std::sqrt(0.25 * (a - d) * (a - d) + b * c);
            const cd m1 = tr2 + disc, m2 = tr2 - disc;
            mu = (std::abs(m1 - d) < std::abs(m2 - d)) ? m1 : m2;
        }
        // one implicit single-shift QR sweep on rows/cols l..hi
        cd x = H[l * n + l] - mu, y = H[(l + 1) * n + l];
        for (int k = l; k < hi; ++k) {
            if (k > l) {
                x = H[k * n + k - 1];
                y = H[(k + 1) * n + k - 1];
            }
            double cc;
            cd ss;
            givens(x, y, cc, ss);
            // rows k, k+1 (columns k-1 .. n-1)
            for (int j = std::max(k - 1, 0); j < n; ++j) {
                const cd u = H[k * n + j], v = H[(k + 1) * n + j];
                H[k * n + j] = cc * u + ss * v;
                H[(k + 1) * n + j] = -std::conj(ss) * u + cc * v;
            }
            if (k > l) H[(k + 1) * n + k - 1] = 0.0;
            // columns k, k+1 (rows 0 .. min(k+2, hi))
            const int rmax = std::min(k + 2, hi);
            for (int r = 0; r <= rmax; ++r) {
                const cd u = H[r * n + k], v = H[r * n + k + 1];
                H[r * n + k] = cc * u + std::conj(ss) * v;
                H[r * n + k + 1] = -ss * u + cc * v;
            }
            for (int r = 0; r < n; ++r) {
                const cd u = Z[r * n + k], v = Z[r * n + k + 1];
                Z[r * n + k] = cc * u + std::conj(ss) * v;
                Z[r * n + k + 1] = -ss * u + cc * v;
            }
        }
    }
    for (int i = 0; i < n; ++i) w[i] = H[i * n + i];
    // eigenvectors of the triangular T = H, then X = Z Y (column-major X)
    const double small = eps * std::max(anorm, 1e-300);
    std::vector<cd> y(n);
    for (int i = 0; i < n; ++i) {
        std::fill(y.begin(), y.end(), cd(0.0));
        y[i] = 1.0;
        for (int j = i - 1; j >= 0; --j) {
            cd s = 0.0;
            for (int l2 = j + 1; l2 <= i; ++l2) s += H[j * n + l2] * y[l2];
            cd den = H[j * n + j] - w[i];
            if (std::abs(den) < small) den = small;
            y[j] = -s / den;
            // keep the partial solution bounded (near-defective T can grow it
            // by 1/eps per step); only the direction matters
            const double a = std::abs(y[j]);
            if (a > 1.0) {
                for (int l2 = j; l2 <= i; ++l2) y[l2] /= a;
            }
        }
        double nrm = 0.0;
        for (int r = 0; r < n; ++r) {
            cd s = 0.0;
            for (int l2 = 0; l2 <= i; ++l2) s += Z[r * n + l2] * y[l2];
            X[(size_t)i * n + r] = s;
            nrm += std::norm(s);
        }
        nrm = std::sqrt(nrm);
        if (!(nrm > 0.0) || !std::isfinite(nrm)) return 2;
        // phase: make the largest component real and positive
        int imax = 0;
        for (int r = 1; r < n; ++r)
            if (std::abs(X[(size_t)i * n + r]) > std::abs(X[(size_t)i * n + imax])) imax = r;
        const cd ph = std::abs(X[(size_t)i * n + imax]) > 0 ? std::conj(X[(size_t)i * n + imax]) /
                                                                   std::abs(X[(size_t)i * n + imax])
                                                             : cd(1.0);
        for (int r = 0; r < n; ++r) X[(size_t)i * n + r] *= ph / nrm;
    }
    return 0;
}

}  // namespace tgdk

// ---------------------------------------------------------------- exports
extern "C" {

int tgdk_host_eig(int n, const double* A, double* wr, double* wi, double* Xr, double* Xi) {
    if (n < 1 || !A || !wr || !wi) return -1;
    std::vector<tgdk::cd> w(n), X((size_t)n * n);
    const int rc = tgdk::eig_real(n, A, w.data(), X.data());
    for (int i = 0; i < n; ++i) {
        wr[i] = w[i].real();
        wi[i] = w[i].imag();
    }
    if (Xr && Xi)
        for (size_t i = 0; i < (size_t)n * n; ++i) {
            Xr[i] = X[i].real();
            Xi[i] = X[i].imag();
        }
    return rc;
}

int tgdk_host_lstsq(int m, int n, const double* A, const double* b, double* x, double* resid) {
    if (m < n || n < 1 || !A || !b || !x) return -1;
    return tgdk::lstsq(m, n, A, b, x, resid);
}

int tgdk_host_lu_solve(int n, const double* A, double* b) {
    if (n < 1 || !A || !b) return -1;
    std::vector<double> LU(A, A + (size_t)n * n);
    std::vector<int> piv(n);
    if (tgdk::lu_factor(n, LU.data(), piv.data()) != 0) return -4;
    tgdk::lu_solve(n, LU.data(), piv.data(), b);
    return 0;
}

int tgdk_host_qr(int m, int n, const double* A, double* Q, double* R) {
    if (m < n || n < 1 || !A || !Q || !R) return -1;
    tgdk::householder_qr(m, n, A, Q, R);
    return 0;
}

}  // extern "C"
