// Dense complex FP64 linear algebra on the device (internal to libgw): the
// GEMMs, the small Hermitian eigensolver and the elementwise kernels that the
// static-subspace, dielectric and self-energy paths are built from.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gw {

// op(X): X as stored, its transpose, or its conjugate transpose.
enum ZOp { kOpN = 0, kOpT = 1, kOpC = 2 };

// C = alpha op(A) op(B) + beta C for `batch` independent products (pointers
// advanced by the strides), row-major: op(A) is m x k, op(B) k x n, C m x n;
// A is stored m x k (kOpN) or k x m (kOpT, kOpC) with leading dimension lda,
// likewise B.  beta = 0 never reads C.  FP64 MFMA, 64 x 64 tiles, each complex
// multiply-add as three real products.
struct ZGemm {
    int m = 0, n = 0, k = 0;
    const double2* a = nullptr;
    int64_t lda = 0, stride_a = 0;
    const double2* b = nullptr;
    int64_t ldb = 0, stride_b = 0;
    double2* c = nullptr;
    int64_t ldc = 0, stride_c = 0;
    double2 alpha = {1.0, 0.0};
    double2 beta = {0.0, 0.0};
    int batch = 1;
};
void launch_zgemm(ZOp opa, ZOp opb, const ZGemm& g, hipStream_t s);

// z = a x + b y over n elements (z may alias x or y).
void launch_zaxpby(int64_t n, double2 a, const double2* x, double2 b, const double2* y,
                   double2* z, hipStream_t s);

// out[i][j] = w[i] in[i][j] for an [rows][cols] block (out may be in).
void launch_scale_rows(const double2* in, double2* out, const double* w, int64_t rows,
                       int64_t cols, hipStream_t s);

// out[b][j] = Re a[b][j][j] for `batch` n x n matrices (batch stride n*n).
void launch_diag_re(const double2* a, int n, int batch, double* out, hipStream_t s);

// out[b][:, j] = in[b][:, perm[b][j]] for `batch` [rows][n_in] blocks (perm
// [batch][n_out]).
void launch_gather_cols(const double2* in, double2* out, int rows, int n_in, int n_out,
                        const int* perm, int batch, hipStream_t s);

// Eigen-decomposition of `batch` Hermitian n x n matrices (row-major, leading
// dimension n, batch stride n*n) by cyclic two-sided Jacobi rotations in
// parallel (round-robin) order, for n >= 64 grouped into blocks of 16 whose
// pairs are rotated in LDS and applied as 32 x 32 unitaries: on return the
// diagonal of a holds the eigenvalues, v (n x n, columns = eigenvectors)
// satisfies A0 v = v diag(a).
// `work` holds jacobi_work_bytes(n, batch) bytes.  Sweeps until the
// off-diagonal Frobenius norm is below tol times the Frobenius norm, or
// max_sweeps; returns the sweeps made (reads one scalar per sweep back: the
// call waits for the stream).
size_t jacobi_work_bytes(int n, int batch);

// Inverse of the upper Cholesky factor of an n x n Hermitian positive
// semidefinite G (row-major): G = R^H R, rinv = R^-1 (upper triangular,
// n x n), blocked by 64 (the diagonal blocks factored and inverted in LDS, the
// panels and trailing updates as GEMMs).  A pivot at or below 1e-26 of G's
// largest diagonal entry marks its direction as lost: that row of R and that
// row and column of rinv are zero, so Y rinv has a zero column there.  G is
// overwritten (R in its upper triangle).  work: chol_work_bytes(n).  Only
// enqueues.
size_t chol_work_bytes(int n);
void chol_inverse(double2* g, double2* rinv, int n, void* work, hipStream_t s);
int jacobi_eigh(double2* a, double2* v, int n, int batch, double tol, int max_sweeps, void* work,
                hipStream_t s);

}  // namespace gw
