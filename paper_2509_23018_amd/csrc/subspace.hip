// Diag of the static subspace method (Fast Full-Frequency GW section of the
// paper): the n_eig most significant eigenvectors of the Hermitian static
// polarizability, found by Chebyshev-filtered subspace iteration with
// Rayleigh-Ritz steps, on the device.
//
// chi0(0) is negative semidefinite (Delta < 0 at z = 0 when every valence
// energy lies below every conduction energy), so its most significant
// eigenvalues are its most negative ones: the iteration works on A = -chi,
// which is positive semidefinite, and keeps the largest eigenvalues of A.
//
// One iteration, on a block of nb = n_eig + guard orthonormal columns X:
//   1. filter  Y = p_m(A) X, p_m the Chebyshev polynomial of degree m that is
//      bounded by 1 on [0, a_cut] (a_cut: the smallest Ritz value of the block,
//      below which lies what is not wanted) and grows fastest above it,
//      scaled by its value at the upper bound b of the spectrum (three-term
//      recurrence of the scaled polynomials); m is chosen so that the filter
//      amplifies the largest Ritz value (times 1.2, a margin for what the
//      block has not yet found) by at most 2e6 over a_cut, which keeps Y well
//      enough conditioned for the Gram-matrix orthonormalisation below;
//   2. orthonormalise Y twice (Cholesky-QR): G = Y^H Y = R^H R, Y <- Y R^-1
//      (chol_inverse: blocked, directions lost to rounding dropped);
//   3. Rayleigh-Ritz: H = X^H A X = W T W^H (Jacobi, to 1e-3 of the previous
//      iteration's largest residual, at least 1e-15), X <- X W, Ritz values
//      in decreasing order;
//   4. residuals r_j = |A x_j - t_j x_j| / b for the n_eig kept pairs.
// It stops when every kept residual is below tol.  b is the largest absolute
// row sum of chi (Gershgorin: an upper bound of the spectrum).
//
// With a weight w the matrix is W chi W, W = diag(w), applied as three steps
// (scale the rows of the block, the GEMM with chi, scale the rows again), so
// the weighted matrix is never formed.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "common.hpp"
#include "linalg.hpp"
#include "prof.hpp"
#include "subspace.hpp"

namespace gw {
namespace {

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// Start block: entries uniform in [-1/2, 1/2) + i [-1/2, 1/2) from a
// counter-based hash of (seed, index).
__global__ __launch_bounds__(256) void random_block_kernel(double2* __restrict__ x, int64_t n,
                                                           uint64_t seed) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const uint64_t h1 = splitmix64(seed ^ (2 * static_cast<uint64_t>(i)));
        const uint64_t h2 = splitmix64(seed ^ (2 * static_cast<uint64_t>(i) + 1));
        x[i] = make_double2(static_cast<double>(h1 >> 11) * 0x1.0p-53 - 0.5,
                            static_cast<double>(h2 >> 11) * 0x1.0p-53 - 0.5);
    }
}

// Absolute row sums of W a W (w NULL: W = I) for a [n][n]: one workgroup per row.
__global__ __launch_bounds__(256) void row_abs_sum_kernel(const double2* __restrict__ a, int n,
                                                          const double* __restrict__ w,
                                                          double* __restrict__ out) {
    const int64_t i = blockIdx.x;
    double acc = 0.0;
    for (int j = threadIdx.x; j < n; j += 256) {
        const double2 x = a[i * n + j];
        acc += hypot(x.x, x.y) * (w ? fabs(w[j]) : 1.0);
    }
    __shared__ double s[256];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[i] = s[0] * (w ? fabs(w[i]) : 1.0);
}

// out[:, j] = in[:, perm[j]] for an [rows][n] block.
__global__ __launch_bounds__(256) void gather_cols_kernel(const double2* __restrict__ in,
                                                          double2* __restrict__ out, int rows,
                                                          int n_in, int n_out,
                                                          const int* __restrict__ perm) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(rows) * n_out) return;
    const int64_t i = t / n_out;
    const int j = static_cast<int>(t % n_out);
    out[t] = in[i * n_in + perm[j]];
}

// diag(h)[perm[j]] -> theta[j]
__global__ void take_diag_kernel(const double2* __restrict__ h, int n,
                                 const int* __restrict__ perm, int count,
                                 double* __restrict__ theta, double scale) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= count) return;
    const int p = perm[j];
    theta[j] = scale * h[static_cast<int64_t>(p) * n + p].x;
}

// r[j] = |ax[:, j] - theta[j] x[:, j]|, one workgroup per column j < count.
__global__ __launch_bounds__(256) void residual_kernel(const double2* __restrict__ x,
                                                       const double2* __restrict__ ax, int rows,
                                                       int nb, const double* __restrict__ theta,
                                                       double* __restrict__ r) {
    const int j = blockIdx.x;
    const double t = theta[j];
    double acc = 0.0;
    for (int i = threadIdx.x; i < rows; i += 256) {
        const int64_t o = static_cast<int64_t>(i) * nb + j;
        const double re = ax[o].x - t * x[o].x, im = ax[o].y - t * x[o].y;
        acc += re * re + im * im;
    }
    __shared__ double s[256];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) r[j] = sqrt(s[0]);
}

struct Carve {
    size_t off = 0;
    size_t take(size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~static_cast<size_t>(255);
        return o;
    }
};

struct DiagLayout {
    int nb = 0;
    size_t big[4] = {0, 0, 0, 0};      // [ng][nb] blocks
    size_t wx = 0;                     // [ng][nb]: W x (weighted only)
    size_t g = 0, u = 0, w = 0, jw = 0;  // [nb][nb]: Gram / Ritz matrix, vectors, sorted vectors
    size_t cw = 0;                       // Cholesky work
    size_t vec = 0;                    // [ng] doubles (row sums), [nb] doubles (residuals)
    size_t theta = 0, perm = 0;
    size_t total = 0;
};

DiagLayout diag_layout(int ng, int n_eig, int guard, bool weighted) {
    DiagLayout L;
    L.nb = std::min(ng, n_eig + guard);
    const size_t blk = static_cast<size_t>(ng) * L.nb * sizeof(double2);
    const size_t sm = static_cast<size_t>(L.nb) * L.nb * sizeof(double2);
    Carve cv;
    for (auto& b : L.big) b = cv.take(blk);
    L.wx = cv.take(weighted ? blk : 0);
    L.g = cv.take(sm);
    L.u = cv.take(sm);
    L.w = cv.take(sm);
    L.jw = cv.take(jacobi_work_bytes(L.nb, 1));
    L.cw = cv.take(chol_work_bytes(L.nb));
    L.vec = cv.take(static_cast<size_t>(std::max(ng, L.nb)) * sizeof(double));
    L.theta = cv.take(static_cast<size_t>(L.nb) * sizeof(double));
    L.perm = cv.take(static_cast<size_t>(L.nb) * sizeof(int));
    L.total = cv.off;
    return L;
}

int default_guard(int n_eig) { return std::max(16, n_eig / 8); }

// out[j] = -in[j]
__global__ void negate_kernel(const double* __restrict__ in, double* __restrict__ out, int n) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) out[j] = -in[j];
}

}  // namespace

size_t subspace_basis_bytes(int ng, int n_eig, int guard, bool weighted) {
    return diag_layout(ng, n_eig, guard > 0 ? guard : default_guard(n_eig), weighted).total;
}

DiagResult run_subspace_basis(const double2* chi, int ng, int n_eig, double2* basis,
                              double* eigenvalues, const DiagParams& prm, char* base,
                              hipStream_t s) {
    const int guard = prm.guard > 0 ? prm.guard : default_guard(n_eig);
    const double* wgt = prm.weight;
    const DiagLayout L = diag_layout(ng, n_eig, guard, wgt != nullptr);
    const int nb = L.nb;
    double2* pool[4];
    for (int i = 0; i < 4; ++i) pool[i] = reinterpret_cast<double2*>(base + L.big[i]);
    double2* g = reinterpret_cast<double2*>(base + L.g);
    double2* u = reinterpret_cast<double2*>(base + L.u);
    double2* w = reinterpret_cast<double2*>(base + L.w);
    void* jw = base + L.jw;
    void* cwk = base + L.cw;
    double* vec = reinterpret_cast<double*>(base + L.vec);
    double* theta = reinterpret_cast<double*>(base + L.theta);
    int* perm_d = reinterpret_cast<int*>(base + L.perm);
    const int64_t blk = static_cast<int64_t>(ng) * nb;
    const int64_t nn = static_cast<int64_t>(nb) * nb;
    const double2 one = make_double2(1.0, 0.0), zero = make_double2(0.0, 0.0);

    auto gemm = [&](ZOp oa, ZOp ob, int m, int n, int k, double2 alpha, const double2* a,
                    int64_t lda, const double2* b, int64_t ldb, double2* c, int64_t ldc) {
        ZGemm gg;
        gg.m = m;
        gg.n = n;
        gg.k = k;
        gg.a = a;
        gg.lda = lda;
        gg.b = b;
        gg.ldb = ldb;
        gg.c = c;
        gg.ldc = ldc;
        gg.alpha = alpha;
        gg.beta = zero;
        launch_zgemm(oa, ob, gg, s);
    };
    // y = scale * A x = -scale * W chi W x for an [ng][nb] block
    double2* wx = reinterpret_cast<double2*>(base + L.wx);
    auto apply_a = [&](const double2* x, double2* y, double scale) {
        if (!wgt) {
            gemm(kOpN, kOpN, ng, nb, ng, make_double2(-scale, 0.0), chi, ng, x, nb, y, nb);
            return;
        }
        launch_scale_rows(x, wx, wgt, ng, nb, s);
        gemm(kOpN, kOpN, ng, nb, ng, make_double2(-scale, 0.0), chi, ng, wx, nb, y, nb);
        launch_scale_rows(y, y, wgt, ng, nb, s);
    };
    // the real diagonal of an [nb][nb] matrix, gathered on the device and read back
    std::vector<double> dg(nb);
    auto read_diag = [&](const double2* m) {
        launch_diag_re(m, nb, 1, vec, s);
        GW_HIP_TRY(hipMemcpyAsync(dg.data(), vec, nb * sizeof(double), hipMemcpyDeviceToHost, s));
        GW_HIP_TRY(hipStreamSynchronize(s));
    };
    // orthonormalise y into z: two passes of Cholesky-QR (tmp: scratch)
    auto orth = [&](const double2* y, double2* z, double2* tmp) {
        const double2* src = y;
        for (int pass = 0; pass < 2; ++pass) {
            double2* dst = pass == 0 ? tmp : z;
            gemm(kOpC, kOpN, nb, nb, ng, one, src, nb, src, nb, g, nb);
            chol_inverse(g, u, nb, cwk, s);
            gemm(kOpN, kOpN, ng, nb, nb, one, src, nb, u, nb, dst, nb);
            src = dst;
        }
    };
    int xi = 0;  // pool[xi] holds the current orthonormal block
    auto spare = [&](int k) {  // k-th pool buffer other than the current block
        for (int i = 0; i < 4; ++i)
            if (i != xi && k-- == 0) return i;
        return -1;
    };

    DiagResult res;
    // spectrum bound of A (Gershgorin)
    hipLaunchKernelGGL(row_abs_sum_kernel, dim3(ng), dim3(256), 0, s, chi, ng, wgt, vec);
    GW_HIP_TRY(hipGetLastError());
    std::vector<double> h(std::max(ng, nb));
    GW_HIP_TRY(hipMemcpyAsync(h.data(), vec, ng * sizeof(double), hipMemcpyDeviceToHost, s));
    GW_HIP_TRY(hipStreamSynchronize(s));
    const double bup = *std::max_element(h.begin(), h.begin() + ng);
    res.bound = bup;
    if (!(bup > 0.0)) {
        // chi = 0: the first unit vectors, eigenvalues 0
        std::vector<double2> e(static_cast<size_t>(ng) * n_eig, zero);
        for (int j = 0; j < n_eig; ++j) e[static_cast<size_t>(j) * n_eig + j] = one;
        std::vector<double> z(n_eig, 0.0);
        GW_HIP_TRY(hipMemcpyAsync(basis, e.data(), e.size() * sizeof(double2),
                                  hipMemcpyHostToDevice, s));
        GW_HIP_TRY(hipMemcpyAsync(eigenvalues, z.data(), n_eig * sizeof(double),
                                  hipMemcpyHostToDevice, s));
        GW_HIP_TRY(hipStreamSynchronize(s));
        return res;
    }

    hipLaunchKernelGGL(random_block_kernel,
                       dim3(static_cast<unsigned>(std::min<int64_t>(ceil_div64(blk, 256), 8192))),
                       dim3(256), 0, s, pool[1], blk, prm.seed);
    GW_HIP_TRY(hipGetLastError());
    orth(pool[1], pool[0], pool[2]);
    std::vector<int> perm(nb);
    double acut = 0.0, top = 0.0;
    for (int it = 0;; ++it) {
        if (it > 0) {
            // Chebyshev filter on [0, acut] scaled at bup: p_m(A) X, then orthonormalised
            const double e = 0.5 * acut, c = 0.5 * acut;
            const double bdeg = std::min(bup, std::max(1.2 * top, 1.001 * acut));
            const double ach = std::acosh(std::max((bdeg - c) / e, 1.0 + 1e-12));
            const int m =
                std::max(1, std::min(prm.max_degree, static_cast<int>(std::log(2e6) / ach)));
            res.degree = m;
            const double s1 = e / (bup - c);
            double sg = s1;
            int prev = xi, cur = spare(0), next = spare(1);
            apply_a(pool[prev], pool[cur], s1 / e);
            launch_zaxpby(blk, one, pool[cur], make_double2(-c * s1 / e, 0.0), pool[prev],
                          pool[cur], s);
            for (int i = 2; i <= m; ++i) {
                const double sn = 1.0 / (2.0 / s1 - sg);
                apply_a(pool[cur], pool[next], 2.0 * sn / e);
                launch_zaxpby(blk, one, pool[next], make_double2(-2.0 * sn * c / e, 0.0),
                              pool[cur], pool[next], s);
                launch_zaxpby(blk, one, pool[next], make_double2(-sg * sn, 0.0), pool[prev],
                              pool[next], s);
                sg = sn;
                const int t = prev;
                prev = cur;
                cur = next;
                next = t;
            }
            // pool[cur] is filtered; prev and next are free, and so is the fourth
            int fourth = 0;
            while (fourth == cur || fourth == prev || fourth == next) ++fourth;
            orth(pool[cur], pool[fourth], pool[prev]);
            xi = fourth;
        }
        // Rayleigh-Ritz: H = X^H A X = W T W^H
        const int ti = spare(0), yi = spare(1), ai = spare(2);
        apply_a(pool[xi], pool[ti], 1.0);
        gemm(kOpC, kOpN, nb, nb, ng, one, pool[xi], nb, pool[ti], nb, g, nb);
        const double rr_tol = it == 0 ? 1e-6 : std::max(1e-15, std::min(1e-6, 1e-3 * res.residual));
        res.sweeps += jacobi_eigh(g, u, nb, 1, rr_tol, 60, jw, s);
        read_diag(g);
        std::iota(perm.begin(), perm.end(), 0);
        std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return dg[a] > dg[b]; });
        GW_HIP_TRY(hipMemcpyAsync(perm_d, perm.data(), nb * sizeof(int), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(gather_cols_kernel, dim3(static_cast<unsigned>(ceil_div64(nn, 256))),
                           dim3(256), 0, s, u, w, nb, nb, nb, perm_d);
        hipLaunchKernelGGL(take_diag_kernel, dim3(ceil_div(nb, 256)), dim3(256), 0, s, g, nb,
                           perm_d, nb, theta, 1.0);
        GW_HIP_TRY(hipGetLastError());
        gemm(kOpN, kOpN, ng, nb, nb, one, pool[xi], nb, w, nb, pool[yi], nb);  // Ritz vectors
        gemm(kOpN, kOpN, ng, nb, nb, one, pool[ti], nb, w, nb, pool[ai], nb);  // A times them
        hipLaunchKernelGGL(residual_kernel, dim3(n_eig), dim3(256), 0, s, pool[yi], pool[ai], ng,
                           nb, theta, vec);
        GW_HIP_TRY(hipGetLastError());
        GW_HIP_TRY(hipMemcpyAsync(h.data(), vec, n_eig * sizeof(double), hipMemcpyDeviceToHost, s));
        GW_HIP_TRY(hipStreamSynchronize(s));
        double rmax = 0.0;
        for (int j = 0; j < n_eig; ++j) rmax = std::max(rmax, h[j] / bup);
        res.residual = rmax;
        res.iterations = it + 1;
        xi = yi;
        // below the smallest Ritz value of the block lies what is not wanted;
        // a zero floor (chi of lower rank than the block) still filters
        acut = std::max(dg[perm[nb - 1]], 1e-6 * bup);
        top = dg[perm[0]];
        if (rmax <= prm.tol || it + 1 >= prm.max_iter || nb == ng) break;
    }
    // the first n_eig Ritz vectors; eigenvalues of chi are minus those of A
    std::iota(perm.begin(), perm.end(), 0);
    GW_HIP_TRY(hipMemcpyAsync(perm_d, perm.data(), nb * sizeof(int), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(gather_cols_kernel,
                       dim3(static_cast<unsigned>(ceil_div64(static_cast<int64_t>(ng) * n_eig, 256))),
                       dim3(256), 0, s, pool[xi], basis, ng, nb, n_eig, perm_d);
    hipLaunchKernelGGL(negate_kernel, dim3(ceil_div(n_eig, 256)), dim3(256), 0, s, theta,
                       eigenvalues, n_eig);
    GW_HIP_TRY(hipGetLastError());
    GW_HIP_TRY(hipStreamSynchronize(s));  // host vectors staged above are read by now
    return res;
}

}  // namespace gw
