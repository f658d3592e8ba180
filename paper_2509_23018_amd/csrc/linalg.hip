// Dense complex FP64 linear algebra on gfx950 (linalg.hpp): a GEMM on the
// FP64 matrix cores, an elementwise axpby and a Hermitian Jacobi eigensolver.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "linalg.hpp"
#include "prof.hpp"

namespace gw {
namespace {

// ---------------------------------------------------------------- GEMM
//
// One workgroup of 4 waves per 64 x 64 tile of C; each wave owns a 32 x 32
// quarter as 2 x 2 blocks of the 16x16x4 FP64 MFMA.  The k dimension is
// staged through LDS 16 at a time; the next stage's global loads are issued
// into registers before the current stage's MFMAs (loads unconditional on
// clamped addresses, masks and conjugation applied at the LDS write).  Each
// complex multiply-add takes three real products (p1 = ar br, p2 = ai bi,
// p3 = (ar + ai)(br + bi); Re = p1 - p2, Im = p3 - p1 - p2).

template <int OPA, int OPB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void zgemm_kernel(
    ZGemm g) {
    __shared__ double2 s_a[64][17];  // [m][k]
    __shared__ double2 s_b[16][65];  // [k][n]
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63, row = lane & 15, kq = lane >> 4;
    const int wi = wave >> 1, wj = wave & 1;
    const int64_t bz = blockIdx.z;
    const double2* A = g.a + bz * g.stride_a;
    const double2* B = g.b + bz * g.stride_b;
    double2* C = g.c + bz * g.stride_c;
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    const int mlast = g.m - 1, nlast = g.n - 1, klast = g.k - 1;

    dbl4 p1[2][2], p2[2][2], p3[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) p1[x][y] = p2[x][y] = p3[x][y] = zero4();

    double2 ra[4], rb[4];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + 256 * u;
            const double2* sa;
            if (OPA == kOpN)
                sa = A + static_cast<int64_t>(min(i0 + (e >> 4), mlast)) * g.lda +
                     min(k0 + (e & 15), klast);
            else
                sa = A + static_cast<int64_t>(min(k0 + (e >> 6), klast)) * g.lda +
                     min(i0 + (e & 63), mlast);
            ra[u].x = sa->x;
            ra[u].y = sa->y;
            const double2* sb;
            if (OPB == kOpN)
                sb = B + static_cast<int64_t>(min(k0 + (e >> 6), klast)) * g.ldb +
                     min(j0 + (e & 63), nlast);
            else
                sb = B + static_cast<int64_t>(min(j0 + (e >> 4), nlast)) * g.ldb +
                     min(k0 + (e & 15), klast);
            rb[u].x = sb->x;
            rb[u].y = sb->y;
        }
    };
    if (g.k > 0) fetch(0);
    for (int k0 = 0; k0 < g.k; k0 += 16) {
        __syncthreads();  // every wave is done with the previous stage
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + 256 * u;
            int mm, kk;
            if (OPA == kOpN) {
                mm = e >> 4;
                kk = e & 15;
            } else {
                kk = e >> 6;
                mm = e & 63;
            }
            const bool oka = i0 + mm < g.m && k0 + kk < g.k;
            s_a[mm][kk] = oka ? make_double2(ra[u].x, OPA == kOpC ? -ra[u].y : ra[u].y)
                              : make_double2(0.0, 0.0);
            int nn;
            if (OPB == kOpN) {
                kk = e >> 6;
                nn = e & 63;
            } else {
                nn = e >> 4;
                kk = e & 15;
            }
            const bool okb = j0 + nn < g.n && k0 + kk < g.k;
            s_b[kk][nn] = okb ? make_double2(rb[u].x, OPB == kOpC ? -rb[u].y : rb[u].y)
                              : make_double2(0.0, 0.0);
        }
        __syncthreads();
        __builtin_amdgcn_s_setprio(1);
        if (k0 + 16 < g.k) fetch(k0 + 16);
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_setprio(2);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            double2 a[2], b[2];
            double as[2], bs[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                a[x] = s_a[wi * 32 + x * 16 + row][s * 4 + kq];
                as[x] = a[x].x + a[x].y;
            }
#pragma unroll
            for (int y = 0; y < 2; ++y) {
                b[y] = s_b[s * 4 + kq][wj * 32 + y * 16 + row];
                bs[y] = b[y].x + b[y].y;
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    p1[x][y] = mfma_f64(a[x].x, b[y].x, p1[x][y]);
                    p2[x][y] = mfma_f64(a[x].y, b[y].y, p2[x][y]);
                    p3[x][y] = mfma_f64(as[x], bs[y], p3[x][y]);
                }
        }
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_setprio(0);
    }
    const bool use_beta = g.beta.x != 0.0 || g.beta.y != 0.0;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int r = i0 + wi * 32 + x * 16 + 4 * t + kq;
                const int c = j0 + wj * 32 + y * 16 + row;
                if (r >= g.m || c >= g.n) continue;
                const double2 acc = make_double2(p1[x][y][t] - p2[x][y][t],
                                                 p3[x][y][t] - p1[x][y][t] - p2[x][y][t]);
                double2 v = cmul(g.alpha, acc);
                double2* dst = C + static_cast<int64_t>(r) * g.ldc + c;
                if (use_beta) {
                    const double2 o = cmul(g.beta, *dst);
                    v.x += o.x;
                    v.y += o.y;
                }
                *dst = v;
            }
}

template <int OPA, int OPB>
void zgemm_launch(const ZGemm& g, hipStream_t s) {
    const dim3 grid(static_cast<unsigned>(ceil_div(g.n, 64)),
                    static_cast<unsigned>(ceil_div(g.m, 64)), static_cast<unsigned>(g.batch));
    ProfScope ps("zgemm", s);
    hipLaunchKernelGGL((zgemm_kernel<OPA, OPB>), grid, dim3(256), 0, s, g);
    GW_HIP_TRY(hipGetLastError());
}

// z may alias x or y (elementwise), so the pointers are not restrict
__global__ __launch_bounds__(256) void zaxpby_kernel(int64_t n, double2 a, const double2* x,
                                                     double2 b, const double2* y, double2* z) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const double2 u = cmul(a, x[i]);
        const double2 v = cmul(b, y[i]);
        z[i] = make_double2(u.x + v.x, u.y + v.y);
    }
}

__global__ __launch_bounds__(256) void scale_rows_kernel(const double2* in, double2* out,
                                                         const double* __restrict__ w,
                                                         int64_t n, int64_t cols) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const double f = w[i / cols];
        const double2 x = in[i];
        out[i] = make_double2(f * x.x, f * x.y);
    }
}

__global__ __launch_bounds__(256) void diag_re_kernel(const double2* __restrict__ a, int n,
                                                      double* __restrict__ out) {
    const int64_t b = blockIdx.y;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) out[b * n + j] = a[b * n * n + static_cast<int64_t>(j) * n + j].x;
}

// ---------------------------------------------------------------- Cholesky

constexpr int kCB = 64;  // Cholesky block

// out[0] = the largest real diagonal entry of g (one workgroup)
__global__ __launch_bounds__(256) void diag_max_kernel(const double2* __restrict__ g, int n,
                                                       double* __restrict__ out) {
    __shared__ double s[256];
    double m = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) m = fmax(m, g[static_cast<int64_t>(i) * n + i].x);
    s[threadIdx.x] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = s[0];
}

// Diagonal block K = [k0, k0 + kb) of g: the upper Cholesky factor R_KK of
// g[K][K] (g[K][K] = R_KK^H R_KK) written back over it (lower part zero), and
// X = R_KK^-1 into x ([kCB][kCB], upper; rows and columns of lost directions
// zero).  A pivot at or below 1e-26 * gmax[0] is a lost direction.
__global__ __launch_bounds__(256) void chol_block_kernel(double2* __restrict__ g, int n, int k0,
                                                         int kb, const double* __restrict__ gmax,
                                                         double2* __restrict__ x) {
    __shared__ double2 r[kCB][kCB + 1];
    __shared__ double2 xi[kCB][kCB + 1];
    const int tid = threadIdx.x;
    const double thr = 1e-26 * gmax[0];
    for (int e = tid; e < kb * kb; e += 256) {
        const int i = e / kb, j = e % kb;
        r[i][j] = g[static_cast<int64_t>(k0 + i) * n + k0 + j];
    }
    __syncthreads();
    for (int k = 0; k < kb; ++k) {
        const double piv = r[k][k].x;
        const bool lost = !(piv > thr);
        const double rk = lost ? 0.0 : sqrt(piv);
        __syncthreads();  // every thread has read the pivot
        for (int j = k + tid; j < kb; j += 256) {
            if (lost)
                r[k][j] = make_double2(0.0, 0.0);
            else if (j == k)
                r[k][k] = make_double2(rk, 0.0);
            else
                r[k][j] = make_double2(r[k][j].x / rk, r[k][j].y / rk);
        }
        __syncthreads();
        // trailing upper part: r[i][j] -= conj(r[k][i]) r[k][j], k < i <= j
        const int m = kb - k - 1;
        for (int e = tid; e < m * m; e += 256) {
            const int i = k + 1 + e / m, j = k + 1 + e % m;
            if (j < i) continue;
            const double2 a = r[k][i], b = r[k][j];
            r[i][j].x -= a.x * b.x + a.y * b.y;  // conj(a) b
            r[i][j].y -= a.x * b.y - a.y * b.x;
        }
        __syncthreads();
    }
    // X = R^-1, column j by thread j: back substitution upwards
    if (tid < kb) {
        const int j = tid;
        for (int i = 0; i < kb; ++i) xi[i][j] = make_double2(0.0, 0.0);
        const double rjj = r[j][j].x;
        xi[j][j] = make_double2(rjj > 0.0 ? 1.0 / rjj : 0.0, 0.0);
        for (int i = j - 1; i >= 0; --i) {
            const double rii = r[i][i].x;
            if (!(rii > 0.0)) continue;  // lost direction: row i of X stays zero
            double sr = 0.0, si = 0.0;
            for (int k = i + 1; k <= j; ++k) {
                const double2 a = r[i][k], b = xi[k][j];
                sr += a.x * b.x - a.y * b.y;
                si += a.x * b.y + a.y * b.x;
            }
            xi[i][j] = make_double2(-sr / rii, -si / rii);
        }
    }
    __syncthreads();
    for (int e = tid; e < kb * kb; e += 256) {
        const int i = e / kb, j = e % kb;
        g[static_cast<int64_t>(k0 + i) * n + k0 + j] = j >= i ? r[i][j] : make_double2(0.0, 0.0);
        x[i * kCB + j] = xi[i][j];
    }
}

// dst[i][j] = src[i][j] for an [rows][cols] block (leading dimensions lds, ldd)
__global__ __launch_bounds__(256) void copy_block_kernel(const double2* __restrict__ src,
                                                         int64_t lds, double2* __restrict__ dst,
                                                         int64_t ldd, int rows, int cols) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(rows) * cols) return;
    const int64_t i = t / cols, j = t % cols;
    dst[i * ldd + j] = src[i * lds + j];
}

__global__ __launch_bounds__(256) void zero_fill_kernel(double2* __restrict__ p, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = make_double2(0.0, 0.0);
}

// ---------------------------------------------------------------- Jacobi
//
// Round-robin order on n' = n rounded up to even: in step r (r < n' - 1) the
// n'/2 pairs are (L[k], L[n'-1-k]) with L[0] = 0 and
// L[j] = 1 + (j - 1 + r) mod (n' - 1); every pair meets once per sweep.  An
// index n (odd n) is a phantom: its pair does not rotate.
//
// Rotation of pair (p, q) (p < q), from h_pp, h_qq and b = h_pq = |b| e^{i phi}:
// tau = (h_qq - h_pp) / (2 |b|), t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
// c = 1 / sqrt(1 + t^2), S = t c e^{i phi}; J = [[c, S], [-conj(S), c]] on
// (p, q) makes (J^H H J)_pq = 0.  One step applies the n'/2 disjoint
// rotations at once: A <- J^H A J and V <- V J.  A and V are read from one
// buffer and written to the other (the rotation of every pair is computed from
// the read buffer by each thread that needs it), so a step is one launch.

__device__ __forceinline__ int rr_index(int j, int r, int np) {
    return j == 0 ? 0 : 1 + (j - 1 + r) % (np - 1);
}

__device__ __forceinline__ void rr_pair(int k, int r, int np, int& p, int& q) {
    const int a = rr_index(k, r, np), b = rr_index(np - 1 - k, r, np);
    p = min(a, b);
    q = max(a, b);
}

struct Rot {
    double c;
    double2 s;  // S
};

__device__ __forceinline__ Rot rotation_of(double hpp, double hqq, double2 b) {
    Rot r{1.0, make_double2(0.0, 0.0)};
    const double ab = hypot(b.x, b.y);
    if (ab == 0.0) return r;
    const double tau = (hqq - hpp) / (2.0 * ab);
    const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
    // c = 1 / sqrt(1 + t^2), then one Newton step on c^2 (1 + t^2) = 1 with the
    // products kept exact by fma: for small t the rounded c alone leaves
    // c^2 + |S|^2 - 1 at about +eps/2 on average, a bias that thousands of
    // rotations per entry turn into a (1 + O(1e-13)) scaling of the spectrum
    const double c0 = 1.0 / sqrt(1.0 + t * t);
    const double pp = c0 * c0, pe = fma(c0, c0, -pp);
    const double qq = t * t, qe = fma(t, t, -qq);
    const double res = (pp - 1.0) + pe + fma(pp, qq, pp * qe + pe * qq);
    const double c = c0 - 0.5 * c0 * res;
    const double sc = t * c / ab;  // S = t c b / |b|
    r.c = c;
    r.s = make_double2(sc * b.x, sc * b.y);
    return r;
}

__device__ __forceinline__ Rot rotation(const double2* __restrict__ a, int n, int p, int q) {
    if (q >= n) return Rot{1.0, make_double2(0.0, 0.0)};
    return rotation_of(a[static_cast<int64_t>(p) * n + p].x, a[static_cast<int64_t>(q) * n + q].x,
                       a[static_cast<int64_t>(p) * n + q]);
}

// blocks [0, na): 2 x 2 blocks (k1, k2) of A; blocks [na, ...): (row, pair) of V
__global__ __launch_bounds__(256) void jacobi_step_kernel(const double2* __restrict__ a_in,
                                                          double2* __restrict__ a_out,
                                                          const double2* __restrict__ v_in,
                                                          double2* __restrict__ v_out, int n,
                                                          int np, int r, int64_t na_threads,
                                                          int64_t batch_stride) {
    const int64_t bz = blockIdx.z;
    a_in += bz * batch_stride;
    a_out += bz * batch_stride;
    v_in += bz * batch_stride;
    v_out += bz * batch_stride;
    const int half = np / 2;
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t < na_threads) {
        const int k1 = static_cast<int>(t / half), k2 = static_cast<int>(t % half);
        int p1, q1, p2, q2;
        rr_pair(k1, r, np, p1, q1);
        rr_pair(k2, r, np, p2, q2);
        const Rot r1 = rotation(a_in, n, p1, q1);
        const Rot r2 = k2 == k1 ? r1 : rotation(a_in, n, p2, q2);
        const bool q1ok = q1 < n, q2ok = q2 < n;
        auto ld = [&](int i, int j, bool ok) {
            return ok ? a_in[static_cast<int64_t>(i) * n + j] : make_double2(0.0, 0.0);
        };
        const double2 app = ld(p1, p2, true), apq = ld(p1, q2, q2ok);
        const double2 aqp = ld(q1, p2, q1ok), aqq = ld(q1, q2, q1ok && q2ok);
        // right: [x_p, x_q] <- [c x_p - conj(S) x_q, S x_p + c x_q]
        const double2 s2 = r2.s, s2c = make_double2(s2.x, -s2.y);
        auto right = [&](double2 xp, double2 xq, double2& op, double2& oq) {
            const double2 u = cmul(s2c, xq), w = cmul(s2, xp);
            op = make_double2(r2.c * xp.x - u.x, r2.c * xp.y - u.y);
            oq = make_double2(w.x + r2.c * xq.x, w.y + r2.c * xq.y);
        };
        double2 bpp, bpq, bqp, bqq;
        right(app, apq, bpp, bpq);
        right(aqp, aqq, bqp, bqq);
        // left: rows p' = c row_p - S row_q, q' = conj(S) row_p + c row_q
        const double2 s1 = r1.s, s1c = make_double2(s1.x, -s1.y);
        auto left = [&](double2 xp, double2 xq, double2& op, double2& oq) {
            const double2 u = cmul(s1, xq), w = cmul(s1c, xp);
            op = make_double2(r1.c * xp.x - u.x, r1.c * xp.y - u.y);
            oq = make_double2(w.x + r1.c * xq.x, w.y + r1.c * xq.y);
        };
        double2 cpp, cqp, cpq, cqq;
        left(bpp, bqp, cpp, cqp);
        left(bpq, bqq, cpq, cqq);
        if (k1 == k2) {  // the rotated pair: exact zeros off the diagonal, real diagonal
            cpq = cqp = make_double2(0.0, 0.0);
            cpp.y = 0.0;
            cqq.y = 0.0;
        }
        a_out[static_cast<int64_t>(p1) * n + p2] = cpp;
        if (q2ok) a_out[static_cast<int64_t>(p1) * n + q2] = cpq;
        if (q1ok) a_out[static_cast<int64_t>(q1) * n + p2] = cqp;
        if (q1ok && q2ok) a_out[static_cast<int64_t>(q1) * n + q2] = cqq;
        return;
    }
    const int64_t tv = t - na_threads;
    if (tv >= static_cast<int64_t>(n) * half) return;
    const int i = static_cast<int>(tv / half), k = static_cast<int>(tv % half);
    int p, q;
    rr_pair(k, r, np, p, q);
    const Rot ro = rotation(a_in, n, p, q);
    const double2 xp = v_in[static_cast<int64_t>(i) * n + p];
    if (q >= n) {
        v_out[static_cast<int64_t>(i) * n + p] = xp;
        return;
    }
    const double2 xq = v_in[static_cast<int64_t>(i) * n + q];
    const double2 sc = make_double2(ro.s.x, -ro.s.y);
    const double2 u = cmul(sc, xq), w = cmul(ro.s, xp);
    v_out[static_cast<int64_t>(i) * n + p] = make_double2(ro.c * xp.x - u.x, ro.c * xp.y - u.y);
    v_out[static_cast<int64_t>(i) * n + q] = make_double2(w.x + ro.c * xq.x, w.y + ro.c * xq.y);
}

// ---------------------------------------------------------------- block Jacobi
//
// For n >= kBJMin the same rotations are grouped by blocks of kBJ = 16
// indices.  The blocks (n rounded up to whole blocks, then to an even count;
// a block past n is a phantom) meet in the round-robin order above, and in
// one block step each pair of blocks (I, J) owns the 32 x 32 Hermitian
// sub-matrix S = A[I u J, I u J]:
//   1. one workgroup per pair runs one cyclic sweep of the element rotations
//      on S in LDS (31 steps of 16 disjoint rotations) and accumulates them
//      into the unitary Q = J_1 J_2 ... J_31;
//   2. one launch applies every pair's Q at once: the tile of A on rows
//      I_k u J_k and columns I_l u J_l becomes Q_k^H A[., .] Q_l, and the
//      columns I_l u J_l of V become V[:, .] Q_l.
// A tile depends only on its own entries and two Q's, so step 2 is in place;
// the tiles with k <= l are computed and the others written as their
// conjugate transposes, which keeps A exactly Hermitian.  A block sweep
// (blocks - 1 steps) meets every pair of indices at least once, as an element
// sweep does, but reads and writes A and V once per block step instead of
// once per element step.  Entries past n are zero in S, so their rotations
// are the identity and never couple them with the others; they are neither
// read nor written.

constexpr int kBJ = 16, kBP = 2 * kBJ, kBJMin = 64;

struct Quad {  // a 2 x 2 block of complex entries
    double2 a00, a01, a10, a11;
};

__device__ __forceinline__ double2 cfma(double2 a, double2 b, double2 c) {  // c + a b
    return make_double2(fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y)));
}
__device__ __forceinline__ double2 cfma_conj_a(double2 a, double2 b, double2 c) {  // c + conj(a) b
    return make_double2(fma(a.x, b.x, fma(a.y, b.y, c.x)), fma(a.x, b.y, fma(-a.y, b.x, c.y)));
}

__device__ __forceinline__ int bj_row(int t, int bp, int bq) {  // local index -> global index
    return t < kBJ ? bp * kBJ + t : bq * kBJ + (t - kBJ);
}

// one pair's sweep; q_out[pair] = Q (32 x 32, row-major)
__global__ __launch_bounds__(256) void bj_inner_kernel(const double2* __restrict__ a, int n,
                                                       int nbp, int r,
                                                       double2* __restrict__ q_out,
                                                       int64_t a_stride, int64_t q_stride) {
    const int64_t bz = blockIdx.z;
    a += bz * a_stride;
    q_out += bz * q_stride + static_cast<int64_t>(blockIdx.x) * kBP * kBP;
    const int bp = rr_index(blockIdx.x, r, nbp), bq = rr_index(nbp - 1 - blockIdx.x, r, nbp);
    __shared__ double2 sm[kBP][kBP + 1];
    __shared__ double2 qm[kBP][kBP + 1];
    __shared__ double rc[kBP / 2];
    __shared__ double2 rs[kBP / 2];
    const int t = threadIdx.x;
    for (int e = t; e < kBP * kBP; e += 256) {
        const int i = e / kBP, j = e % kBP;
        const int gi = bj_row(i, bp, bq), gj = bj_row(j, bp, bq);
        sm[i][j] = gi < n && gj < n ? a[static_cast<int64_t>(gi) * n + gj] : make_double2(0.0, 0.0);
        qm[i][j] = make_double2(i == j ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    const int k1 = t / (kBP / 2), k2 = t % (kBP / 2);
    for (int r2 = 0; r2 < kBP - 1; ++r2) {
        if (t < kBP / 2) {
            int p, q;
            rr_pair(t, r2, kBP, p, q);
            const Rot ro = rotation_of(sm[p][p].x, sm[q][q].x, sm[p][q]);
            rc[t] = ro.c;
            rs[t] = ro.s;
        }
        __syncthreads();
        int p1, q1, p2, q2;
        rr_pair(k1, r2, kBP, p1, q1);
        rr_pair(k2, r2, kBP, p2, q2);
        const double c1 = rc[k1], c2 = rc[k2];
        const double2 s1 = rs[k1], s2 = rs[k2];
        const double2 s1c = make_double2(s1.x, -s1.y), s2c = make_double2(s2.x, -s2.y);
        // right: [x_p, x_q] <- [c x_p - conj(S) x_q, S x_p + c x_q]
        auto right = [&](double2 xp, double2 xq, double2& op, double2& oq) {
            const double2 u = cmul(s2c, xq), w = cmul(s2, xp);
            op = make_double2(c2 * xp.x - u.x, c2 * xp.y - u.y);
            oq = make_double2(w.x + c2 * xq.x, w.y + c2 * xq.y);
        };
        // left: rows p' = c row_p - S row_q, q' = conj(S) row_p + c row_q
        auto left = [&](double2 xp, double2 xq, double2& op, double2& oq) {
            const double2 u = cmul(s1, xq), w = cmul(s1c, xp);
            op = make_double2(c1 * xp.x - u.x, c1 * xp.y - u.y);
            oq = make_double2(w.x + c1 * xq.x, w.y + c1 * xq.y);
        };
        double2 bpp, bpq, bqp, bqq, cpp, cpq, cqp, cqq;
        right(sm[p1][p2], sm[p1][q2], bpp, bpq);
        right(sm[q1][p2], sm[q1][q2], bqp, bqq);
        left(bpp, bqp, cpp, cqp);
        left(bpq, bqq, cpq, cqq);
        if (k1 == k2) {  // the rotated pair: exact zeros off the diagonal, real diagonal
            cpq = cqp = make_double2(0.0, 0.0);
            cpp.y = 0.0;
            cqq.y = 0.0;
        }
        sm[p1][p2] = cpp;
        sm[p1][q2] = cpq;
        sm[q1][p2] = cqp;
        sm[q1][q2] = cqq;
        // Q <- Q J on rows k1 and k1 + 16, columns (p2, q2)
        for (int h = 0; h < 2; ++h) {
            const int i = k1 + h * (kBP / 2);
            double2 op, oq;
            right(qm[i][p2], qm[i][q2], op, oq);
            qm[i][p2] = op;
            qm[i][q2] = oq;
        }
        __syncthreads();
    }
    for (int e = t; e < kBP * kBP; e += 256) q_out[e] = qm[e / kBP][e % kBP];
}

// Workgroups [0, na): tiles (k, l), k <= l, of A, numbered row by row of the
// upper triangle of pairs; [na, na + ceil(n / 32) * npair): tiles (row chunk,
// pair l) of V.  Each thread owns a 2 x 2 block of the 32 x 32 tile.
__global__ __launch_bounds__(256) void bj_update_kernel(double2* __restrict__ a,
                                                        double2* __restrict__ v, int n, int nbp,
                                                        int r, const double2* __restrict__ qs,
                                                        int64_t a_stride, int64_t q_stride,
                                                        int na) {
    const int64_t bz = blockIdx.z;
    a += bz * a_stride;
    v += bz * a_stride;
    qs += bz * q_stride;
    const int npair = nbp / 2;
    __shared__ double2 xm[kBP][kBP + 1];
    __shared__ double2 ym[kBP][kBP + 1];
    __shared__ double2 qk[kBP][kBP + 1];
    __shared__ double2 ql[kBP][kBP + 1];
    const int t = threadIdx.x;
    const int i0 = 2 * (t / (kBP / 2)), j0 = 2 * (t % (kBP / 2));
    const double2 zero = make_double2(0.0, 0.0);
    // (x q_l)[i0.., j0..]
    auto mul_right = [&]() {
        const double2 z = make_double2(0.0, 0.0);
        Quad acc{z, z, z, z};
#pragma unroll 4
        for (int c = 0; c < kBP; ++c) {
            const double2 x0 = xm[i0][c], x1 = xm[i0 + 1][c];
            const double2 b0 = ql[c][j0], b1 = ql[c][j0 + 1];
            acc.a00 = cfma(x0, b0, acc.a00);
            acc.a01 = cfma(x0, b1, acc.a01);
            acc.a10 = cfma(x1, b0, acc.a10);
            acc.a11 = cfma(x1, b1, acc.a11);
        }
        return acc;
    };
    int blk = blockIdx.x;
    if (blk < na) {
        int k = 0;
        while (blk >= npair - k) {
            blk -= npair - k;
            ++k;
        }
        const int l = k + blk;
        const int bpk = rr_index(k, r, nbp), bqk = rr_index(nbp - 1 - k, r, nbp);
        const int bpl = rr_index(l, r, nbp), bql = rr_index(nbp - 1 - l, r, nbp);
        for (int e = t; e < kBP * kBP; e += 256) {
            const int i = e / kBP, j = e % kBP;
            const int gi = bj_row(i, bpk, bqk), gj = bj_row(j, bpl, bql);
            xm[i][j] = gi < n && gj < n ? a[static_cast<int64_t>(gi) * n + gj] : make_double2(0.0, 0.0);
            qk[i][j] = qs[static_cast<int64_t>(k) * kBP * kBP + e];
            ql[i][j] = qs[static_cast<int64_t>(l) * kBP * kBP + e];
        }
        __syncthreads();
        const Quad y = mul_right();
        ym[i0][j0] = y.a00;
        ym[i0][j0 + 1] = y.a01;
        ym[i0 + 1][j0] = y.a10;
        ym[i0 + 1][j0 + 1] = y.a11;
        __syncthreads();
        // T = q_k^H y
        Quad tt{zero, zero, zero, zero};
#pragma unroll 4
        for (int c = 0; c < kBP; ++c) {
            const double2 h0 = qk[c][i0], h1 = qk[c][i0 + 1];
            const double2 y0 = ym[c][j0], y1 = ym[c][j0 + 1];
            tt.a00 = cfma_conj_a(h0, y0, tt.a00);
            tt.a01 = cfma_conj_a(h0, y1, tt.a01);
            tt.a10 = cfma_conj_a(h1, y0, tt.a10);
            tt.a11 = cfma_conj_a(h1, y1, tt.a11);
        }
        // xm is free (every thread has read it in mul_right before the barrier)
        xm[i0][j0] = tt.a00;
        xm[i0][j0 + 1] = tt.a01;
        xm[i0 + 1][j0] = tt.a10;
        xm[i0 + 1][j0 + 1] = tt.a11;
        __syncthreads();
        for (int e = t; e < kBP * kBP; e += 256) {
            const int i = e / kBP, j = e % kBP;
            if (k == l) {  // Hermitian part of the diagonal tile
                const int gi = bj_row(i, bpk, bqk), gj = bj_row(j, bpk, bqk);
                if (gi < n && gj < n) {
                    const double2 x = xm[i][j], y = xm[j][i];
                    a[static_cast<int64_t>(gi) * n + gj] =
                        make_double2(0.5 * (x.x + y.x), i == j ? 0.0 : 0.5 * (x.y - y.y));
                }
            } else {
                const int gi = bj_row(i, bpk, bqk), gj = bj_row(j, bpl, bql);
                if (gi < n && gj < n) a[static_cast<int64_t>(gi) * n + gj] = xm[i][j];
                // row i of the mirrored tile: rows I_l u J_l, columns I_k u J_k
                const int hi = bj_row(i, bpl, bql), hj = bj_row(j, bpk, bqk);
                if (hi < n && hj < n) {
                    const double2 x = xm[j][i];
                    a[static_cast<int64_t>(hi) * n + hj] = make_double2(x.x, -x.y);
                }
            }
        }
        return;
    }
    blk -= na;
    const int chunk = blk / npair, l = blk % npair;
    const int bpl = rr_index(l, r, nbp), bql = rr_index(nbp - 1 - l, r, nbp);
    const int row0 = chunk * kBP;
    for (int e = t; e < kBP * kBP; e += 256) {
        const int i = e / kBP, j = e % kBP;
        const int gj = bj_row(j, bpl, bql);
        xm[i][j] = row0 + i < n && gj < n ? v[static_cast<int64_t>(row0 + i) * n + gj] : make_double2(0.0, 0.0);
        ql[i][j] = qs[static_cast<int64_t>(l) * kBP * kBP + e];
    }
    __syncthreads();
    const Quad y = mul_right();
    const double2 out[4] = {y.a00, y.a01, y.a10, y.a11};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int gi = row0 + i0 + e / 2, gj = bj_row(j0 + e % 2, bpl, bql);
        if (gi < n && gj < n) v[static_cast<int64_t>(gi) * n + gj] = out[e];
    }
}

__global__ __launch_bounds__(256) void eye_kernel(double2* __restrict__ v, int n, int64_t stride) {
    const int64_t bz = blockIdx.z;
    const int64_t nn = static_cast<int64_t>(n) * n;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < nn;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        v[bz * stride + i] = make_double2(i / n == i % n ? 1.0 : 0.0, 0.0);
}

// Partial sums of (off-diagonal |a|^2, all |a|^2) per workgroup, then one
// workgroup adds the partials: out[2*b], out[2*b + 1] per batch entry b.
constexpr int kRedBlocks = 256;

__global__ __launch_bounds__(256) void offnorm_partial_kernel(const double2* __restrict__ a,
                                                              int n, int64_t stride,
                                                              double* __restrict__ part) {
    const int64_t bz = blockIdx.z;
    const int64_t nn = static_cast<int64_t>(n) * n;
    double off = 0.0, all = 0.0;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < nn;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const double2 x = a[bz * stride + i];
        const double m2 = x.x * x.x + x.y * x.y;
        all += m2;
        if (i / n != i % n) off += m2;
    }
    __shared__ double s_off[256], s_all[256];
    s_off[threadIdx.x] = off;
    s_all[threadIdx.x] = all;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s_off[threadIdx.x] += s_off[threadIdx.x + w];
            s_all[threadIdx.x] += s_all[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[(bz * kRedBlocks + blockIdx.x) * 2] = s_off[0];
        part[(bz * kRedBlocks + blockIdx.x) * 2 + 1] = s_all[0];
    }
}

__global__ __launch_bounds__(256) void offnorm_final_kernel(const double* __restrict__ part,
                                                            double* __restrict__ out) {
    const int64_t bz = blockIdx.x;
    __shared__ double s_off[256], s_all[256];
    s_off[threadIdx.x] = part[(bz * kRedBlocks + threadIdx.x) * 2];
    s_all[threadIdx.x] = part[(bz * kRedBlocks + threadIdx.x) * 2 + 1];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s_off[threadIdx.x] += s_off[threadIdx.x + w];
            s_all[threadIdx.x] += s_all[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * bz] = s_off[0];
        out[2 * bz + 1] = s_all[0];
    }
}

__global__ __launch_bounds__(256) void gather_cols_batched_kernel(
    const double2* __restrict__ in, double2* __restrict__ out, int rows, int n_in, int n_out,
    const int* __restrict__ perm) {
    const int64_t bz = blockIdx.z;
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(rows) * n_out) return;
    const int64_t i = t / n_out;
    const int j = static_cast<int>(t % n_out);
    out[bz * rows * n_out + t] = in[bz * rows * n_in + i * n_in + perm[bz * n_out + j]];
}

}  // namespace

void launch_gather_cols(const double2* in, double2* out, int rows, int n_in, int n_out,
                        const int* perm, int batch, hipStream_t s) {
    const int64_t n = static_cast<int64_t>(rows) * n_out;
    if (n <= 0 || batch <= 0) return;
    hipLaunchKernelGGL(gather_cols_batched_kernel,
                       dim3(static_cast<unsigned>(ceil_div64(n, 256)), 1, batch), dim3(256), 0, s,
                       in, out, rows, n_in, n_out, perm);
    GW_HIP_TRY(hipGetLastError());
}

void launch_zgemm(ZOp opa, ZOp opb, const ZGemm& g, hipStream_t s) {
    if (g.m <= 0 || g.n <= 0 || g.batch <= 0) return;
    switch (opa * 3 + opb) {
        case 0: zgemm_launch<kOpN, kOpN>(g, s); break;
        case 1: zgemm_launch<kOpN, kOpT>(g, s); break;
        case 2: zgemm_launch<kOpN, kOpC>(g, s); break;
        case 3: zgemm_launch<kOpT, kOpN>(g, s); break;
        case 4: zgemm_launch<kOpT, kOpT>(g, s); break;
        case 5: zgemm_launch<kOpT, kOpC>(g, s); break;
        case 6: zgemm_launch<kOpC, kOpN>(g, s); break;
        case 7: zgemm_launch<kOpC, kOpT>(g, s); break;
        default: zgemm_launch<kOpC, kOpC>(g, s); break;
    }
}

void launch_zaxpby(int64_t n, double2 a, const double2* x, double2 b, const double2* y,
                   double2* z, hipStream_t s) {
    if (n <= 0) return;
    const int64_t blocks = std::min<int64_t>(ceil_div64(n, 256), 8192);
    hipLaunchKernelGGL(zaxpby_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, n, a,
                       x, b, y, z);
    GW_HIP_TRY(hipGetLastError());
}

void launch_diag_re(const double2* a, int n, int batch, double* out, hipStream_t s) {
    if (n <= 0 || batch <= 0) return;
    hipLaunchKernelGGL(diag_re_kernel, dim3(ceil_div(n, 256), batch), dim3(256), 0, s, a, n, out);
    GW_HIP_TRY(hipGetLastError());
}

void launch_scale_rows(const double2* in, double2* out, const double* w, int64_t rows,
                       int64_t cols, hipStream_t s) {
    const int64_t n = rows * cols;
    if (n <= 0) return;
    const int64_t blocks = std::min<int64_t>(ceil_div64(n, 256), 8192);
    hipLaunchKernelGGL(scale_rows_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                       in, out, w, n, cols);
    GW_HIP_TRY(hipGetLastError());
}

size_t chol_work_bytes(int n) {
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    // x (kCB x kCB), panel t (kCB x n), column block u (n x kCB), gmax
    return al(sizeof(double2) * kCB * kCB) + 2 * al(sizeof(double2) * kCB * static_cast<size_t>(n)) + 256;
}

void chol_inverse(double2* g, double2* rinv, int n, void* work, hipStream_t s) {
    if (n <= 0) return;
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    char* w = static_cast<char*>(work);
    double2* x = reinterpret_cast<double2*>(w);
    double2* t = reinterpret_cast<double2*>(w + al(sizeof(double2) * kCB * kCB));
    double2* u = reinterpret_cast<double2*>(w + al(sizeof(double2) * kCB * kCB) +
                                            al(sizeof(double2) * kCB * static_cast<size_t>(n)));
    double* gmax = reinterpret_cast<double*>(w + al(sizeof(double2) * kCB * kCB) +
                                             2 * al(sizeof(double2) * kCB * static_cast<size_t>(n)));
    const int64_t nn = static_cast<int64_t>(n) * n;
    hipLaunchKernelGGL(zero_fill_kernel, dim3(static_cast<unsigned>(std::min<int64_t>(ceil_div64(nn, 256), 4096))),
                       dim3(256), 0, s, rinv, nn);
    hipLaunchKernelGGL(diag_max_kernel, dim3(1), dim3(256), 0, s, g, n, gmax);
    GW_HIP_TRY(hipGetLastError());
    const double2 one = make_double2(1.0, 0.0), mone = make_double2(-1.0, 0.0);
    for (int k0 = 0; k0 < n; k0 += kCB) {
        const int kb = std::min(kCB, n - k0), rest = n - k0 - kb;
        hipLaunchKernelGGL(chol_block_kernel, dim3(1), dim3(256), 0, s, g, n, k0, kb, gmax, x);
        GW_HIP_TRY(hipGetLastError());
        if (rest > 0) {
            // panel of R: T = X^H g[K][K+], then g[K][K+] = T
            ZGemm p;
            p.m = kb;
            p.n = rest;
            p.k = kb;
            p.a = x;
            p.lda = kCB;
            p.b = g + static_cast<int64_t>(k0) * n + k0 + kb;
            p.ldb = n;
            p.c = t;
            p.ldc = n;
            launch_zgemm(kOpC, kOpN, p, s);
            hipLaunchKernelGGL(copy_block_kernel, dim3(static_cast<unsigned>(ceil_div64(static_cast<int64_t>(kb) * rest, 256))),
                               dim3(256), 0, s, t, static_cast<int64_t>(n),
                               g + static_cast<int64_t>(k0) * n + k0 + kb, static_cast<int64_t>(n), kb, rest);
            GW_HIP_TRY(hipGetLastError());
            // trailing update g[K+][K+] -= T^H T
            ZGemm q;
            q.m = rest;
            q.n = rest;
            q.k = kb;
            q.a = t;
            q.lda = n;
            q.b = t;
            q.ldb = n;
            q.c = g + static_cast<int64_t>(k0 + kb) * n + k0 + kb;
            q.ldc = n;
            q.alpha = mone;
            q.beta = one;
            launch_zgemm(kOpC, kOpN, q, s);
        }
        // R^-1 column block K: diagonal block X, above it -R^-1[<K][<K] R[<K][K] X
        hipLaunchKernelGGL(copy_block_kernel, dim3(static_cast<unsigned>(ceil_div64(static_cast<int64_t>(kb) * kb, 256))),
                           dim3(256), 0, s, x, static_cast<int64_t>(kCB),
                           rinv + static_cast<int64_t>(k0) * n + k0, static_cast<int64_t>(n), kb, kb);
        GW_HIP_TRY(hipGetLastError());
        if (k0 > 0) {
            ZGemm a;  // U = R^-1[<K][<K] R[<K][K]
            a.m = k0;
            a.n = kb;
            a.k = k0;
            a.a = rinv;
            a.lda = n;
            a.b = g + k0;
            a.ldb = n;
            a.c = u;
            a.ldc = kCB;
            launch_zgemm(kOpN, kOpN, a, s);
            ZGemm b;  // R^-1[<K][K] = -U X
            b.m = k0;
            b.n = kb;
            b.k = kb;
            b.a = u;
            b.lda = kCB;
            b.b = x;
            b.ldb = kCB;
            b.c = rinv + k0;
            b.ldc = n;
            b.alpha = mone;
            launch_zgemm(kOpN, kOpN, b, s);
        }
    }
}

size_t jacobi_work_bytes(int n, int batch) {
    // reduction partials and the two results per entry
    const size_t red = static_cast<size_t>(batch) * kRedBlocks * 2 * 8 +
                       static_cast<size_t>(batch) * 2 * 8 + 512;
    if (n >= kBJMin) {  // one Q per pair of blocks
        const int nblk = ceil_div(n, kBJ), nbp = nblk + (nblk & 1);
        const size_t qb = static_cast<size_t>(nbp / 2) * kBP * kBP * sizeof(double2) * batch;
        return ((qb + 255) & ~size_t(255)) + red;
    }
    // second A and V buffers
    const size_t nn = static_cast<size_t>(n) * n * batch * sizeof(double2);
    return 2 * ((nn + 255) & ~size_t(255)) + red;
}

int jacobi_eigh(double2* a, double2* v, int n, int batch, double tol, int max_sweeps, void* work,
                hipStream_t s) {
    if (n <= 0 || batch <= 0) return 0;
    const int64_t nn = static_cast<int64_t>(n) * n;
    const bool blocked = n >= kBJMin;
    const int nblk = ceil_div(n, kBJ), nbp = nblk + (nblk & 1), npair = nbp / 2;
    const int64_t q_stride = static_cast<int64_t>(npair) * kBP * kBP;
    const size_t first =
        blocked ? ((static_cast<size_t>(q_stride) * batch * sizeof(double2) + 255) & ~size_t(255))
                : 2 * ((static_cast<size_t>(nn) * batch * sizeof(double2) + 255) & ~size_t(255));
    char* w = static_cast<char*>(work);
    double* part = reinterpret_cast<double*>(w + first);
    double* res = part + static_cast<size_t>(batch) * kRedBlocks * 2;
    const unsigned eb = static_cast<unsigned>(std::min<int64_t>(ceil_div64(nn, 256), 4096));
    hipLaunchKernelGGL(eye_kernel, dim3(eb, 1, batch), dim3(256), 0, s, v, n, nn);
    GW_HIP_TRY(hipGetLastError());
    if (n == 1) return 0;
    // element sweeps: A and V ping-pong between the caller's buffers and the work area
    const int np = n + (n & 1), half = np / 2;
    const int64_t na_el = static_cast<int64_t>(half) * half;
    const dim3 grid_el(static_cast<unsigned>(ceil_div64(na_el + static_cast<int64_t>(n) * half, 256)),
                       1, batch);
    const size_t nnb = (static_cast<size_t>(nn) * batch * sizeof(double2) + 255) & ~size_t(255);
    double2 *ac = a, *an = reinterpret_cast<double2*>(w), *vc = v,
            *vn = reinterpret_cast<double2*>(w + nnb);
    // block sweeps: in place, Q's in the work area
    double2* qs = reinterpret_cast<double2*>(w);
    const int na_bl = npair * (npair + 1) / 2;
    const int nv_bl = ceil_div(n, kBP) * npair;
    std::vector<double> h(2 * static_cast<size_t>(batch));
    std::vector<double> prev(batch, -1.0);
    int sweeps = 0;
    for (; sweeps < max_sweeps; ++sweeps) {
        hipLaunchKernelGGL(offnorm_partial_kernel, dim3(kRedBlocks, 1, batch), dim3(256), 0, s, ac,
                           n, nn, part);
        hipLaunchKernelGGL(offnorm_final_kernel, dim3(batch), dim3(256), 0, s, part, res);
        GW_HIP_TRY(hipGetLastError());
        GW_HIP_TRY(hipMemcpyAsync(h.data(), res, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        GW_HIP_TRY(hipStreamSynchronize(s));
        // done when the off-diagonal norm is below tol of the norm, or when it
        // has stopped falling (the convergence is quadratic until rounding
        // re-creates off-diagonal entries at the level of the unit roundoff)
        bool done = true;
        for (int b = 0; b < batch; ++b) {
            const double off = std::sqrt(h[2 * b]), all = std::sqrt(h[2 * b + 1]);
            const bool small = off <= tol * all;
            const bool stalled = sweeps >= 3 && prev[b] >= 0.0 && off >= 0.25 * prev[b] &&
                                 off <= 1e-12 * all;
            if (!small && !stalled) done = false;
            prev[b] = off;
        }
        if (done) break;
        ProfScope ps("jacobi_sweep", s);
        if (blocked) {
            for (int r = 0; r < nbp - 1; ++r) {
                hipLaunchKernelGGL(bj_inner_kernel, dim3(npair, 1, batch), dim3(256), 0, s, ac, n,
                                   nbp, r, qs, nn, q_stride);
                hipLaunchKernelGGL(bj_update_kernel, dim3(na_bl + nv_bl, 1, batch), dim3(256), 0,
                                   s, ac, vc, n, nbp, r, qs, nn, q_stride, na_bl);
            }
        } else {
            for (int r = 0; r < np - 1; ++r) {
                hipLaunchKernelGGL(jacobi_step_kernel, grid_el, dim3(256), 0, s, ac, an, vc, vn, n,
                                   np, r, na_el, nn);
                std::swap(ac, an);
                std::swap(vc, vn);
            }
        }
        GW_HIP_TRY(hipGetLastError());
    }
    if (ac != a) {  // results back into the caller's buffers
        GW_HIP_TRY(hipMemcpyAsync(a, ac, static_cast<size_t>(nn) * batch * sizeof(double2),
                                  hipMemcpyDeviceToDevice, s));
        GW_HIP_TRY(hipMemcpyAsync(v, vc, static_cast<size_t>(nn) * batch * sizeof(double2),
                                  hipMemcpyDeviceToDevice, s));
    }
    return sweeps;
}

}  // namespace gw
