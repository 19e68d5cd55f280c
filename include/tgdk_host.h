/*
 * tgdk host algebra -- the small dense float64 routines the solvers run on
 * the host, exported so they can be checked without a GPU.  All matrices are
 * row-major host arrays owned by the caller.  Return 0 on success.
 */
#ifndef TGDK_HOST_H
#define TGDK_HOST_H

#ifdef __cplusplus
extern "C" {
#endif

/* Eigenvalues (wr + i wi) and unit eigenvectors of a real n x n matrix A:
 * eigenvector j is Xr[j*n + r] + i Xi[j*n + r].  Used for the harmonic Ritz
 * eigenproblem of GMRES-DR (Sec. 2.1).  Returns nonzero if the QR iteration
 * does not converge. */
int tgdk_host_eig(int n, const double* A, double* wr, double* wi, double* Xr, double* Xi);

/* x = argmin ||b - A x|| for A m x n (m >= n) by Householder QR; resid
 * (length m, may be NULL) receives b - A x.  The GMRES least-squares step. */
int tgdk_host_lstsq(int m, int n, const double* A, const double* b, double* x, double* resid);

/* Solves A x = b in place (b -> x) by LU with partial pivoting, as for the
 * projection system H d = c (Sec. 2.2).  Returns TGDK_E_SINGULAR (-4) for a
 * zero pivot. */
int tgdk_host_lu_solve(int n, const double* A, double* b);

/* Thin QR A = Q R (A m x n, m >= n) with R_ii >= 0. */
int tgdk_host_qr(int m, int n, const double* A, double* Q, double* R);

#ifdef __cplusplus
}
#endif
#endif /* TGDK_HOST_H */
