// Small dense float64 linear algebra on the host (row-major storage).
#pragma once

#include <complex>
#include <vector>

namespace tgdk {

// LU with partial pivoting in place; piv[j] = row swapped with row j at step j.
// Returns 0, or j+1 if the j-th pivot is zero.
int lu_factor(int n, double* A, int* piv);
void lu_solve(int n, const double* LU, const int* piv, double* b);
double cond_estimate_lu(int n, const double* LU);
// G = R^T R, R upper triangular written over G.  Returns 0 or j+1 on failure.
int cholesky_upper(int n, double* G);
void upper_inverse(int n, const double* R, double* Rinv);
// Thin QR of an m x n matrix (m >= n) with R_ii >= 0.
void householder_qr(int m, int n, const double* A, double* Q, double* R);
// x = argmin ||b - A x|| (A m x n, m >= n); resid = b - A x if not null.
int lstsq(int m, int n, const double* A, const double* b, double* x, double* resid);
// Eigenvalues w[n] and unit eigenvectors X (column i at X + i*n) of a real
// n x n matrix.  Returns 0 on success.
int eig_real(int n, const double* A, std::complex<double>* w, std::complex<double>* X);
// Indices of the k values of smallest modulus (ties by real part, then
// positive imaginary part first); a kept complex value brings its conjugate
// partner along (listed right after it), so k+1 may be returned.
std::vector<int> select_smallest(const std::vector<std::complex<double>>& th, int k);

}  // namespace tgdk
