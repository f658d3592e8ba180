// Inverse dielectric matrix of Eq. (3): eps^-1(z) = [I - v chi(z)]^-1, v the
// diagonal Coulomb matrix, for every frequency, on the device.
//
// eps = I - v chi is built in the output buffer and inverted there by block
// Gauss-Jordan elimination without pivoting, 64 columns at a time.  For the
// block K of columns/rows:
//   D^-1   the inverse of the diagonal block A[K,K] (one workgroup, scalar
//          Gauss-Jordan in LDS);
//   L      = A[:, K] with its K rows zeroed (saved), then A[not K, K] = 0;
//   R      = D^-1 A[K, :], with R[:, K] = D^-1, written back as A[K, :];
//   A     -= L R  (one GEMM of N_G x 64 x N_G on FP64 MFMA).
// After the last block A holds eps^-1.  Without pivoting the elimination
// needs nonsingular leading blocks: eps = v^1/2 eps~ v^-1/2 with
// eps~ = I - v^1/2 chi v^1/2 Hermitian positive definite (eigenvalues >= 1)
// whenever chi is Hermitian negative semidefinite (zero and imaginary
// frequencies), so there every pivot block is well conditioned; on the real
// axis eps is not guaranteed to be.
#include <algorithm>

#include "common.hpp"
#include "epsinv.hpp"
#include "linalg.hpp"
#include "prof.hpp"

namespace gw {
namespace {

constexpr int kB = 64;  // block width

// out[w] = I - diag(v) chi[w]
__global__ __launch_bounds__(256) void build_eps_kernel(const double2* __restrict__ chi,
                                                        const double* __restrict__ v, int ng,
                                                        double2* __restrict__ out) {
    const int64_t w = blockIdx.z;
    const int64_t nn = static_cast<int64_t>(ng) * ng;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < nn;
         t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int i = static_cast<int>(t / ng), j = static_cast<int>(t % ng);
        const double2 c = chi[w * nn + t];
        out[w * nn + t] = make_double2((i == j ? 1.0 : 0.0) - v[i] * c.x, -v[i] * c.y);
    }
}

// d[w] = A[w][K,K]^-1 for the bk x bk block at (k0, k0): scalar Gauss-Jordan in
// LDS, no pivoting.
__global__ __launch_bounds__(256) void block_inverse_kernel(const double2* __restrict__ a, int ng,
                                                            int k0, int bk,
                                                            double2* __restrict__ d) {
    __shared__ double2 s[kB][kB + 1];
    const int64_t w = blockIdx.x;
    const double2* aw = a + w * static_cast<int64_t>(ng) * ng;
    for (int e = threadIdx.x; e < bk * bk; e += 256) {
        const int i = e / bk, j = e % bk;
        s[i][j] = aw[static_cast<int64_t>(k0 + i) * ng + k0 + j];
    }
    __syncthreads();
    for (int p = 0; p < bk; ++p) {
        const double2 piv = s[p][p];
        const double den = piv.x * piv.x + piv.y * piv.y;
        const double2 inv = make_double2(piv.x / den, -piv.y / den);
        __syncthreads();
        // row p scaled (its pivot becomes 1/pivot)
        for (int j = threadIdx.x; j < bk; j += 256)
            s[p][j] = j == p ? inv : cmul(inv, s[p][j]);
        __syncthreads();
        // other rows: a_ij -= a_ip a_pj (j != p), a_ip = -a_ip / pivot
        for (int e = threadIdx.x; e < bk * bk; e += 256) {
            const int i = e / bk, j = e % bk;
            if (i == p) continue;
            const double2 aip = s[i][p];
            if (j == p) continue;
            const double2 pr = cmul(aip, s[p][j]);
            s[i][j] = make_double2(s[i][j].x - pr.x, s[i][j].y - pr.y);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < bk; i += 256)
            if (i != p) {
                const double2 m = cmul(s[i][p], inv);
                s[i][p] = make_double2(-m.x, -m.y);
            }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < bk * bk; e += 256) {
        const int i = e / bk, j = e % bk;
        d[w * kB * kB + i * kB + j] = s[i][j];
    }
}

// L[w] = A[w][:, K] (rows in K zeroed), then A[w][i, K] = 0 for rows i not in K
__global__ __launch_bounds__(256) void take_panel_kernel(double2* __restrict__ a, int ng, int k0,
                                                         int bk, double2* __restrict__ l) {
    const int64_t w = blockIdx.z;
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(ng) * bk) return;
    const int i = static_cast<int>(t / bk), j = static_cast<int>(t % bk);
    double2* src = a + w * static_cast<int64_t>(ng) * ng + static_cast<int64_t>(i) * ng + k0 + j;
    const bool in_k = i >= k0 && i < k0 + bk;
    l[w * static_cast<int64_t>(ng) * kB + static_cast<int64_t>(i) * kB + j] =
        in_k ? make_double2(0.0, 0.0) : *src;
    if (!in_k) *src = make_double2(0.0, 0.0);
}

// R[w][:, K] = D^-1, then A[w][K, :] = R[w]
__global__ __launch_bounds__(256) void put_rows_kernel(double2* __restrict__ a, int ng, int k0,
                                                       int bk, double2* __restrict__ r,
                                                       const double2* __restrict__ d) {
    const int64_t w = blockIdx.z;
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(bk) * ng) return;
    const int i = static_cast<int>(t / ng), j = static_cast<int>(t % ng);
    double2* rr = r + w * static_cast<int64_t>(kB) * ng + static_cast<int64_t>(i) * ng + j;
    double2 x = *rr;
    if (j >= k0 && j < k0 + bk) {
        x = d[w * kB * kB + i * kB + (j - k0)];
        *rr = x;
    }
    a[w * static_cast<int64_t>(ng) * ng + static_cast<int64_t>(k0 + i) * ng + j] = x;
}

}  // namespace

size_t epsinv_bytes(int ng, int nz) {
    const size_t d = static_cast<size_t>(nz) * kB * kB * sizeof(double2);
    const size_t p = static_cast<size_t>(nz) * ng * kB * sizeof(double2);
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    return al(d) + 2 * al(p);
}

void run_epsinv(const double2* chi, int ng, int nz, const double* v, double2* out, char* base,
                hipStream_t s) {
    if (ng <= 0 || nz <= 0) return;
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    double2* d = reinterpret_cast<double2*>(base);
    double2* l = reinterpret_cast<double2*>(base + al(static_cast<size_t>(nz) * kB * kB * 16));
    double2* r = reinterpret_cast<double2*>(base + al(static_cast<size_t>(nz) * kB * kB * 16) +
                                            al(static_cast<size_t>(nz) * ng * kB * 16));
    const int64_t nn = static_cast<int64_t>(ng) * ng;
    {
        ProfScope ps("eps_build", s);
        hipLaunchKernelGGL(build_eps_kernel,
                           dim3(static_cast<unsigned>(std::min<int64_t>(ceil_div64(nn, 256), 4096)), 1, nz),
                           dim3(256), 0, s, chi, v, ng, out);
        GW_HIP_TRY(hipGetLastError());
    }
    ProfScope ps("eps_invert", s);
    for (int k0 = 0; k0 < ng; k0 += kB) {
        const int bk = std::min(kB, ng - k0);
        hipLaunchKernelGGL(block_inverse_kernel, dim3(nz), dim3(256), 0, s, out, ng, k0, bk, d);
        hipLaunchKernelGGL(take_panel_kernel,
                           dim3(static_cast<unsigned>(ceil_div64(static_cast<int64_t>(ng) * bk, 256)), 1, nz),
                           dim3(256), 0, s, out, ng, k0, bk, l);
        GW_HIP_TRY(hipGetLastError());
        ZGemm g1;  // R = D^-1 A[K, :]
        g1.m = bk;
        g1.n = ng;
        g1.k = bk;
        g1.a = d;
        g1.lda = kB;
        g1.stride_a = kB * kB;
        g1.b = out + static_cast<int64_t>(k0) * ng;
        g1.ldb = ng;
        g1.stride_b = nn;
        g1.c = r;
        g1.ldc = ng;
        g1.stride_c = static_cast<int64_t>(kB) * ng;
        g1.batch = nz;
        launch_zgemm(kOpN, kOpN, g1, s);
        hipLaunchKernelGGL(put_rows_kernel,
                           dim3(static_cast<unsigned>(ceil_div64(static_cast<int64_t>(bk) * ng, 256)), 1, nz),
                           dim3(256), 0, s, out, ng, k0, bk, r, d);
        GW_HIP_TRY(hipGetLastError());
        ZGemm g2;  // A -= L R
        g2.m = ng;
        g2.n = ng;
        g2.k = bk;
        g2.a = l;
        g2.lda = kB;
        g2.stride_a = static_cast<int64_t>(ng) * kB;
        g2.b = r;
        g2.ldb = ng;
        g2.stride_b = static_cast<int64_t>(kB) * ng;
        g2.c = out;
        g2.ldc = ng;
        g2.stride_c = nn;
        g2.alpha = make_double2(-1.0, 0.0);
        g2.beta = make_double2(1.0, 0.0);
        g2.batch = nz;
        launch_zgemm(kOpN, kOpN, g2, s);
    }
}

}  // namespace gw
