// Inverse dielectric matrix of Eq. (3): eps^-1(z) = [I - v chi(z)]^-1, v the
// diagonal Coulomb matrix, for every frequency, on the device.
//
// eps = I - v chi is built in the output buffer and inverted there by block
// Gauss-Jordan elimination without pivoting, 512 columns at a time (at most
// N_G rounded up to 64).  For the block K of columns/rows:
//   D^-1   the inverse of the diagonal block A[K,K]: a copy of the block
//          inverted by the same elimination 64 columns at a time, whose
//          64 x 64 pivot blocks are inverted by one workgroup in LDS (scalar
//          Gauss-Jordan);
//   L      = A[:, K] with its K rows zeroed (saved), then A[not K, K] = 0;
//   R      = D^-1 A[K, :], with R[:, K] = D^-1, written back as A[K, :];
//   A     -= L R  (one GEMM of N_G x 512 x N_G on FP64 MFMA: 64 flops per
//          byte of A read and written, against 16 at 64 columns).
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

constexpr int kB = 64;   // width of the pivot blocks inverted in LDS
constexpr int kW = 512;  // width of the elimination's blocks

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

// Matrices below are row-major n x n with leading dimension n, matrix w of the
// batch at a + w * sa.

// d[w] = A[w][K,K]^-1 for the bk x bk block at (k0, k0) (bk <= 64): scalar
// Gauss-Jordan in LDS, no pivoting; d[w] at d + w * kB * kB, leading dimension kB.
__global__ __launch_bounds__(256) void block_inverse_kernel(const double2* __restrict__ a, int n,
                                                            int64_t sa, int k0, int bk,
                                                            double2* __restrict__ d) {
    __shared__ double2 s[kB][kB + 1];
    const int64_t w = blockIdx.x;
    const double2* aw = a + w * sa;
    for (int e = threadIdx.x; e < bk * bk; e += 256) {
        const int i = e / bk, j = e % bk;
        s[i][j] = aw[static_cast<int64_t>(k0 + i) * n + k0 + j];
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

// L[w] = A[w][:, K] (rows in K zeroed), then A[w][i, K] = 0 for rows i not in
// K; L[w] at l + w * n * kb, leading dimension kb
__global__ __launch_bounds__(256) void take_panel_kernel(double2* __restrict__ a, int n,
                                                         int64_t sa, int k0, int bk, int kb,
                                                         double2* __restrict__ l) {
    const int64_t w = blockIdx.z;
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(n) * bk) return;
    const int i = static_cast<int>(t / bk), j = static_cast<int>(t % bk);
    double2* src = a + w * sa + static_cast<int64_t>(i) * n + k0 + j;
    const bool in_k = i >= k0 && i < k0 + bk;
    l[w * static_cast<int64_t>(n) * kb + static_cast<int64_t>(i) * kb + j] =
        in_k ? make_double2(0.0, 0.0) : *src;
    if (!in_k) *src = make_double2(0.0, 0.0);
}

// R[w][:, K] = D^-1, then A[w][K, :] = R[w]; R[w] at r + w * kb * n (leading
// dimension n), D^-1 of w at d + w * sd (leading dimension ldd)
__global__ __launch_bounds__(256) void put_rows_kernel(double2* __restrict__ a, int n, int64_t sa,
                                                       int k0, int bk, int kb,
                                                       double2* __restrict__ r,
                                                       const double2* __restrict__ d, int64_t sd,
                                                       int ldd) {
    const int64_t w = blockIdx.z;
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(bk) * n) return;
    const int i = static_cast<int>(t / n), j = static_cast<int>(t % n);
    double2* rr = r + w * static_cast<int64_t>(kb) * n + static_cast<int64_t>(i) * n + j;
    double2 x = *rr;
    if (j >= k0 && j < k0 + bk) {
        x = d[w * sd + static_cast<int64_t>(i) * ldd + (j - k0)];
        *rr = x;
    }
    a[w * sa + static_cast<int64_t>(k0 + i) * n + j] = x;
}

// D[w] = A[w][K, K] (bk x bk, leading dimension bk, at d + w * sd)
__global__ __launch_bounds__(256) void copy_pivot_kernel(const double2* __restrict__ a, int n,
                                                         int64_t sa, int k0, int bk,
                                                         double2* __restrict__ d, int64_t sd) {
    const int64_t w = blockIdx.z;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= bk * bk) return;
    const int i = t / bk, j = t % bk;
    d[w * sd + t] = a[w * sa + static_cast<int64_t>(k0 + i) * n + k0 + j];
}

size_t al256(size_t b) { return (b + 255) & ~size_t(255); }

// scratch of one gj_invert level with blocks of width kb on n x n matrices
size_t level_bytes(int n, int nz, int kb) {
    const size_t p = static_cast<size_t>(nz) * n * kb * sizeof(double2);
    const size_t d = static_cast<size_t>(nz) * kb * kb * sizeof(double2);
    return al256(d) + 2 * al256(p);
}

// In-place Gauss-Jordan inversion of nz matrices (n x n, batch stride sa),
// blocks of width kb: 64 (pivot blocks inverted in LDS) or more (pivot blocks
// copied and inverted by this routine at width 64).
void gj_invert(double2* a, int n, int64_t sa, int nz, int kb, char* ws, hipStream_t s) {
    double2* d = reinterpret_cast<double2*>(ws);
    double2* l = reinterpret_cast<double2*>(ws + al256(static_cast<size_t>(nz) * kb * kb * 16));
    double2* r = reinterpret_cast<double2*>(ws + al256(static_cast<size_t>(nz) * kb * kb * 16) +
                                            al256(static_cast<size_t>(nz) * n * kb * 16));
    char* inner = ws + level_bytes(n, nz, kb);
    for (int k0 = 0; k0 < n; k0 += kb) {
        const int bk = std::min(kb, n - k0);
        int64_t sd;
        int ldd;
        if (kb == kB) {
            hipLaunchKernelGGL(block_inverse_kernel, dim3(nz), dim3(256), 0, s, a, n, sa, k0, bk, d);
            GW_HIP_TRY(hipGetLastError());
            sd = kB * kB;
            ldd = kB;
        } else {
            sd = static_cast<int64_t>(kb) * kb;
            ldd = bk;
            hipLaunchKernelGGL(copy_pivot_kernel, dim3(ceil_div(bk * bk, 256), 1, nz), dim3(256), 0,
                               s, a, n, sa, k0, bk, d, sd);
            GW_HIP_TRY(hipGetLastError());
            gj_invert(d, bk, sd, nz, kB, inner, s);
        }
        hipLaunchKernelGGL(take_panel_kernel,
                           dim3(static_cast<unsigned>(ceil_div64(static_cast<int64_t>(n) * bk, 256)), 1, nz),
                           dim3(256), 0, s, a, n, sa, k0, bk, kb, l);
        GW_HIP_TRY(hipGetLastError());
        ZGemm g1;  // R = D^-1 A[K, :]
        g1.m = bk;
        g1.n = n;
        g1.k = bk;
        g1.a = d;
        g1.lda = ldd;
        g1.stride_a = sd;
        g1.b = a + static_cast<int64_t>(k0) * n;
        g1.ldb = n;
        g1.stride_b = sa;
        g1.c = r;
        g1.ldc = n;
        g1.stride_c = static_cast<int64_t>(kb) * n;
        g1.batch = nz;
        launch_zgemm(kOpN, kOpN, g1, s);
        hipLaunchKernelGGL(put_rows_kernel,
                           dim3(static_cast<unsigned>(ceil_div64(static_cast<int64_t>(bk) * n, 256)), 1, nz),
                           dim3(256), 0, s, a, n, sa, k0, bk, kb, r, d, sd, ldd);
        GW_HIP_TRY(hipGetLastError());
        ZGemm g2;  // A -= L R
        g2.m = n;
        g2.n = n;
        g2.k = bk;
        g2.a = l;
        g2.lda = kb;
        g2.stride_a = static_cast<int64_t>(n) * kb;
        g2.b = r;
        g2.ldb = n;
        g2.stride_b = static_cast<int64_t>(kb) * n;
        g2.c = a;
        g2.ldc = n;
        g2.stride_c = sa;
        g2.alpha = make_double2(-1.0, 0.0);
        g2.beta = make_double2(1.0, 0.0);
        g2.batch = nz;
        launch_zgemm(kOpN, kOpN, g2, s);
    }
}

// the elimination's block width for N_G: kW, or N_G rounded up to kB if less
int block_width(int ng) { return std::min(kW, ceil_div(ng, kB) * kB); }

}  // namespace

size_t epsinv_bytes(int ng, int nz) {
    const int kb = block_width(ng);
    return level_bytes(ng, nz, kb) + (kb > kB ? level_bytes(kb, nz, kB) : 0);
}

void run_epsinv(const double2* chi, int ng, int nz, const double* v, double2* out, char* base,
                hipStream_t s) {
    if (ng <= 0 || nz <= 0) return;
    const int64_t nn = static_cast<int64_t>(ng) * ng;
    {
        ProfScope ps("eps_build", s);
        hipLaunchKernelGGL(build_eps_kernel,
                           dim3(static_cast<unsigned>(std::min<int64_t>(ceil_div64(nn, 256), 4096)), 1, nz),
                           dim3(256), 0, s, chi, v, ng, out);
        GW_HIP_TRY(hipGetLastError());
    }
    ProfScope ps("eps_invert", s);
    gj_invert(out, ng, nn, nz, block_width(ng), base, s);
}

}  // namespace gw
