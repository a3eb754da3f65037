// Host FP64 linear algebra behind the C ABI: Cholesky, symmetric
// eigendecomposition, and the CVA / PCA solves from accumulated moments.
#pragma once
#include <cstdint>
#include <string>

namespace cvamx {

// Lower Cholesky factor of the symmetric n x n matrix A (row-major, lower
// triangle read).  Returns 0, or CVAMX_E_NOT_PD when a pivot is not
// positive (relative to the diagonal entry it came from).
int cholesky_lower(int n, const double* A, double* L);

// Symmetric eigendecomposition, eigenvalues descending, eigenvectors in the
// columns of V (row-major n x n).  No sign rule.  Returns 0 or
// CVAMX_E_NUMERIC.
int sym_eig_desc(int n, const double* A, double* w, double* V);

// All eigenvalues descending into w[n], and the eigenvectors of the k
// largest into the columns of V (row-major n x k): eigenvalues by implicit
// QR on the tridiagonal form without vectors, the k vectors by inverse
// iteration on it and the stored reflectors (the full decomposition when k
// is more than a quarter of n).  No sign rule.  Returns 0 or a CVAMX status.
int sym_eig_top(int n, const double* A, int k, double* w, double* V);

// Make the largest-magnitude entry of each of the nc columns of the
// rows x nc row-major matrix W positive (ties: lowest row).
void sign_rule(int rows, int nc, double* W);

// CVA solve from class moments.  counts may be real (soft weights), so it
// is passed as double.  Sb_out may be null.  Returns a CVAMX status.
int cva_solve(int K, int B, const double* counts, const double* class_means,
              const double* Sw, double ridge, int n_comp, double* W,
              double* eigvals, double* mean, double* Sb_out, std::string* err);

}  // namespace cvamx
