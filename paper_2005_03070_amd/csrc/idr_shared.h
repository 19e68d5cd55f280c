// Structs of the IDR(s) inner cycles shared by host code and kernels.
#pragma once

#include "tgdk_shared.h"

namespace tgdk {

// IDR(s) inner cycles: scalars of one cycle, kept on the device.  The
// one-workgroup epilogues of the IDR kernels take every decision and write
// here; the vector kernels read it.
constexpr int IDR_SMAX = 32;  // largest shadow-space dimension s
struct IdrState {
    int gate;      // 0 while the cycle runs; nonzero: every IDR kernel returns at once
    int status;    // IN_RUNNING, IN_CONVERGED, IN_BREAK_NOUPD (breakdown), IN_MAXIT
    int s;
    int round0;    // first round of the cycle (G = U = 0)
    int efirst;    // e not yet written this cycle (e = 0)
    int mvps, maxit;
    int pad_;
    double om, kappa, target2, rr, beta;
    double M[IDR_SMAX * IDR_SMAX];  // M = P^T G, row-major, lower triangular
    double f[IDR_SMAX];             // P^T r
    double c[IDR_SMAX];             // coefficients of the next step's direction
    double alpha[IDR_SMAX];         // coefficients that make g_k orthogonal to p_0 .. p_(k-1)
};

// Pointers of the IDR kernels (by value); vectors of the inner type, n x s
// blocks column-major with leading dimension n.
struct IdrArgs {
    void* r;        // inner residual
    void* e;        // correction of the cycle
    void* t;        // A r of the dimension reduction
    void* G;        // g_0 .. g_(s-1)
    void* U;        // u_0 .. u_(s-1)
    const void* P;  // orthonormal shadow matrix
    double* x;      // float64 iterate (the cycle's correction is folded in)
    long long n;
    int nb, s;      // workgroups of the vector kernels; shadow dimension
    double* part;   // nb partial sums per value, value-major
    IdrState* st;
    SolveState* ss;
    Mirror* mirror;
};

}  // namespace tgdk
