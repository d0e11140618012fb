// FP64 dense symmetric eigensolver used at plan time for the leaf sub-GFTs.
//
// Method (Golub & Van Loan, "Matrix Computations", Sec. 8.3): Householder reduction to
// tridiagonal form, then implicit symmetric QR steps with the Wilkinson shift, with the
// rotations accumulated into the eigenvector matrix.  Backward stable; eigenvalues and
// eigenvectors are accurate to O(n * eps * ||A||).
#pragma once

#include <vector>

namespace gft {

// A: n*n row-major symmetric (only read).  On success lambda (n, ascending) and V (n*n
// row-major, V[i*n + k] = component i of eigenvector k) are filled and true returned;
// false if the QR iteration did not converge.
bool symmetric_eigen(int n, const std::vector<double> &A, std::vector<double> &lambda,
                     std::vector<double> &V);

}  // namespace gft
