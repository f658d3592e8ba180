// Diag of the static subspace method (internal to libgw).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace gw {

struct DiagParams {
    double tol = 1e-10;     // residual |A x - t x| / |A| of every kept pair
    int max_iter = 60;      // filtered subspace iterations
    int guard = 0;          // extra block columns (0: max(16, n_eig / 8))
    int max_degree = 16;    // Chebyshev degree cap
    uint64_t seed = 0;      // start block
    const double* weight = nullptr;  // device [ng]: diagonalise W chi W, W = diag(weight)
};

struct DiagResult {
    int iterations = 0;
    int degree = 0;         // filter degree of the last iteration
    double residual = 0.0;  // largest relative residual of the kept pairs
    double bound = 0.0;     // Gershgorin bound of |chi|
    int sweeps = 0;         // Jacobi sweeps of the Rayleigh-Ritz steps, in all
};

// Device scratch of run_subspace_basis (guard 0 = the default; weighted: with a
// weight vector).
size_t subspace_basis_bytes(int ng, int n_eig, int guard, bool weighted);

// basis [ng][n_eig] (columns: eigenvectors of chi for its n_eig most negative
// eigenvalues, orthonormal), eigenvalues [n_eig] in increasing order (most
// negative first).  chi: device [ng][ng], Hermitian, negative semidefinite;
// with prm.weight the matrix diagonalised is W chi W.
// Waits for the stream (the iteration reads convergence data back).
DiagResult run_subspace_basis(const double2* chi, int ng, int n_eig, double2* basis,
                              double* eigenvalues, const DiagParams& prm, char* base,
                              hipStream_t s);

}  // namespace gw
