// Host FP64 dense helpers for Rayleigh-Ritz (internal).
#pragma once

#include <complex>
#include <vector>

namespace pvd {

using cd = std::complex<double>;

// A (n x n, row-major, Hermitian positive definite) -> R upper with A = R^H R.
// Returns false when A is not numerically positive definite.
bool cholesky_upper(int n, std::vector<cd>& A);

// M = R^{-1} for upper-triangular R.
void invert_upper(int n, const std::vector<cd>& R, std::vector<cd>& M);

// Eigen-decomposition of a Hermitian A (destroyed): ascending w, V columns
// the orthonormal eigenvectors (row-major, V[i*n + c] = component i of vector c).
void heev_jacobi(int n, std::vector<cd>& A, std::vector<double>& w, std::vector<cd>& V);

}  // namespace pvd
