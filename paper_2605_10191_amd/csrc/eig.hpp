// Host eigensolvers of the Lanczos matrix and the Rayleigh-Ritz projection
// (plain C++, built without the HIP headers; errors are std::runtime_error).
#pragma once
#include <vector>

namespace polfed {

// Symmetric tridiagonal eigenproblem by implicit QL.  d[n] diagonal, e[n-1]
// off-diagonal.  Accumulates the rotations into the rows of Z (nz x n,
// row-major) that the caller initializes (identity rows for eigenvectors,
// the last unit row for last components only).  Eigenvalues ascending, Z
// columns permuted alike.
void tridiag_eig(int n, std::vector<double>& d, std::vector<double> e,
                 std::vector<double>& Z, int nz);
// Dense symmetric eigenproblem (n x n col-major A): eigenvalues ascending in
// w, eigenvectors in the columns of Z (col-major).
void sym_eig(int n, std::vector<double>& A, std::vector<double>& w,
             std::vector<double>& Z);
// The eigenvalues (ascending) and only the last r rows of the eigenvector
// matrix: Ztail is r x n row-major, Ztail[i n + j] = component n - r + i of
// eigenvector j.
void sym_eig_tail(int n, const std::vector<double>& A, int r, std::vector<double>& w,
                  std::vector<double>& Ztail);

}  // namespace polfed
