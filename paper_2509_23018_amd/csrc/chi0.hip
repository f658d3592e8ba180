// CHI0 on gfx950: chi_w += M^H diag(s*Delta_w) M over one streamed chunk of
// pairs (Eq. (4) of the paper), FP64 MFMA 16x16x4 tiles, plus the energy
// factor, the Hermitian mirror and the zero fill.
#include <algorithm>

#include "chi0.hpp"
#include "common.hpp"
#include "prof.hpp"

namespace gw {

namespace {

// ---------------------------------------------------------------- energy factor

__global__ __launch_bounds__(256) void delta_kernel(const double* __restrict__ e_v,
                                                    const double* __restrict__ e_c, PairMap pm,
                                                    int64_t npairs, ZArgs za, int w0,
                                                    double2* __restrict__ delta) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= npairs) return;
    const int64_t lin = pm.k_off + k;
    const double de = e_v[pm.v0 + lin / pm.cw] - e_c[pm.c0 + lin % pm.cw];
    for (int w = 0; w < za.nz; ++w) {
        const double zr = za.re[w], zi = za.im[w];
        // 1/(de + z) + 1/(de - z), each as conj(d)/|d|^2
        const double ar = de + zr, br = de - zr;
        const double n1 = ar * ar + zi * zi, n2 = br * br + zi * zi;
        double re = ar / n1 + br / n2;
        double im = -zi / n1 + zi / n2;
        if (zr == 0.0) im = 0.0;  // imaginary axis / static: Delta is real
        delta[static_cast<int64_t>(w0 + w) * npairs + k] = make_double2(za.spin * re, za.spin * im);
    }
}

// ---------------------------------------------------------------- FP64 contraction

constexpr int kTile = 64;   // output tile edge per workgroup
constexpr int kKt = 16;     // pairs per LDS stage

// Work item of workgroup b.  Items are frequency-major: first every
// Hermitian frequency over the nh tiles on or above the diagonal, then every
// other frequency over all nb*nb tiles.  The 8 XCDs take workgroups
// round-robin, so blocks are renumbered to give each XCD a contiguous range
// of items (consecutive tiles of one frequency share M rows in its L2).
__device__ __forceinline__ void item_of_block(int b, const WList& wl, int nb, int& w, int& bi,
                                              int& bj) {
    const int nh = nb * (nb + 1) / 2, nf = nb * nb;
    const int nitems = wl.nh * nh + wl.nf * nf;
    const int q = nitems >> 3, r = nitems & 7;
    const int x = b & 7, i = b >> 3;
    int t = x * q + (x < r ? x : r) + i;
    if (t < wl.nh * nh) {
        w = wl.w[t / nh];
        t %= nh;
        bi = 0;
        while (t >= nb - bi) {
            t -= nb - bi;
            ++bi;
        }
        bj = bi + t;
    } else {
        t -= wl.nh * nh;
        w = wl.w[wl.nh + t / nf];
        t %= nf;
        bi = t / nb;
        bj = t - bi * nb;
    }
}

// One workgroup = one 64x64 tile of chi_w; 4 waves in a 2x2 layout, each a
// 32x32 sub-tile of 2x2 MFMA blocks.  Per stage of 16 pairs the rows of M
// for the tile's G and G' are staged in LDS (double-buffered), the G' side
// already multiplied by s*Delta_w(k); the MFMAs then accumulate
// conj(M_i) (Delta M_j).  Loads are unconditional: pair rows past the chunk
// end are clamped and carry Delta = 0, columns past N_G are clamped and only
// feed outputs that are not stored.  mode: 0 overwrite, 1 accumulate.
__global__ __launch_bounds__(256) void chi0_f64_kernel(const double2* __restrict__ m, int64_t kc,
                                                       int ng, const double2* __restrict__ delta,
                                                       WList wl, double2* __restrict__ chi,
                                                       int mode, int nb) {
    int w, bi, bj;
    item_of_block(blockIdx.x, wl, nb, w, bi, bj);
    __shared__ double2 s_a[2][kKt][kTile];
    __shared__ double2 s_b[2][kKt][kTile];
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63, row = lane & 15, kq = lane >> 4;
    const int wi = wave >> 1, wj = wave & 1;
    const int i0 = bi * kTile, j0 = bj * kTile;
    const double2* dw = delta + static_cast<int64_t>(w) * kc;

    // this thread's staging slots: rows kk = (tid >> 6) + 4u, column cc = tid & 63
    const int cc = tid & 63, kk0 = tid >> 6;
    const int64_t ci = min(i0 + cc, ng - 1), cj = min(j0 + cc, ng - 1);

    dbl4 accr[2][2], acci[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) accr[a][b] = acci[a][b] = zero4();

    double2 ra[4], rb[4], rd[4];
    auto gload = [&](int64_t k0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t k = k0 + kk0 + 4 * u;
            const int64_t kr = k < kc ? k : kc - 1;
            const double2* mr = m + kr * ng;
            ra[u] = mr[ci];
            rb[u] = mr[cj];
            rd[u] = dw[kr];
            if (k >= kc) rd[u] = make_double2(0.0, 0.0);
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            s_a[buf][kk0 + 4 * u][cc] = ra[u];
            s_b[buf][kk0 + 4 * u][cc] = cmul(rd[u], rb[u]);
        }
    };

    gload(0);
    sstore(0);
    __syncthreads();
    int buf = 0;
    const int nsteps = static_cast<int>((kc + kKt - 1) / kKt);
    for (int st = 0; st < nsteps; ++st) {
        // unconditional (clamped) prefetch keeps the loop free of branches, so
        // the compiler cannot merge the LDS stores into the load block
        gload(static_cast<int64_t>(st + 1) * kKt);
#pragma unroll
        for (int s = 0; s < kKt / 4; ++s) {
            double2 a[2], b[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                a[x] = s_a[buf][s * 4 + kq][wi * 32 + x * 16 + row];
                b[x] = s_b[buf][s * 4 + kq][wj * 32 + x * 16 + row];
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y)
                    cmfma_conj_a(accr[x][y], acci[x][y], a[x].x, a[x].y, b[y].x, b[y].y);
        }
        // keep the LDS stores of the next stage after this stage's MFMAs, so
        // the global loads issued above stay in flight during the compute
        __builtin_amdgcn_sched_barrier(0);
        sstore(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
    double2* cw = chi + static_cast<int64_t>(w) * ng * ng;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int gi = i0 + wi * 32 + x * 16 + 4 * t + kq;
                const int gj = j0 + wj * 32 + y * 16 + row;
                if (gi < ng && gj < ng) {
                    double2* p = cw + static_cast<int64_t>(gi) * ng + gj;
                    double2 v = make_double2(accr[x][y][t], acci[x][y][t]);
                    if (mode) {
                        const double2 o = *p;
                        v.x += o.x;
                        v.y += o.y;
                    }
                    *p = v;
                }
            }
}

// chi[i][j] = conj(chi[j][i]) for every (i, j) in a tile strictly below the
// diagonal of 64x64 tiles (those the Hermitian contraction skipped).
__global__ __launch_bounds__(256) void mirror_kernel(double2* __restrict__ chi, int ng) {
    const int j = blockIdx.x * 16 + (threadIdx.x & 15);
    const int i = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (i >= ng || j >= ng) return;
    if (i / kTile <= j / kTile) return;
    const double2 u = chi[static_cast<int64_t>(j) * ng + i];
    chi[static_cast<int64_t>(i) * ng + j] = make_double2(u.x, -u.y);
}

__global__ __launch_bounds__(256) void fill_zero_kernel(double2* __restrict__ p, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = make_double2(0.0, 0.0);
}

}  // namespace

void launch_delta(const double* e_v, const double* e_c, PairMap pm, int64_t npairs,
                  const double2* z, int nz, double spin, double2* delta, hipStream_t s) {
    if (npairs <= 0) return;
    for (int w0 = 0; w0 < nz; w0 += kMaxZ) {
        ZArgs za{};
        za.nz = std::min(kMaxZ, nz - w0);
        za.spin = spin;
        for (int w = 0; w < za.nz; ++w) {
            za.re[w] = z[w0 + w].x;
            za.im[w] = z[w0 + w].y;
        }
        ProfScope ps("delta", s);
        hipLaunchKernelGGL(delta_kernel, dim3(static_cast<unsigned>(ceil_div64(npairs, 256))),
                           dim3(256), 0, s, e_v, e_c, pm, npairs, za, w0, delta);
        GW_HIP_TRY(hipGetLastError());
    }
}

void launch_chi0_f64(const double2* m, int64_t kc, int ng, const double2* delta,
                     const WList& wl, double2* chi, bool accumulate, hipStream_t s) {
    if (kc <= 0 || wl.nh + wl.nf == 0) return;
    const int nb = ceil_div(ng, kTile);
    const int64_t nitems = static_cast<int64_t>(wl.nh) * (nb * (nb + 1) / 2) +
                           static_cast<int64_t>(wl.nf) * nb * nb;
    if (nitems >= (int64_t(1) << 31)) throw Error{-4, "too many chi tiles for one launch"};
    ProfScope ps("chi0_f64", s);
    hipLaunchKernelGGL(chi0_f64_kernel, dim3(static_cast<unsigned>(nitems)), dim3(256), 0, s, m,
                       kc, ng, delta, wl, chi, accumulate ? 1 : 0, nb);
    GW_HIP_TRY(hipGetLastError());
}

void launch_mirror(double2* chi, int ng, hipStream_t s) {
    ProfScope ps("mirror", s);
    hipLaunchKernelGGL(mirror_kernel, dim3(ceil_div(ng, 16), ceil_div(ng, 16)), dim3(256), 0, s,
                       chi, ng);
    GW_HIP_TRY(hipGetLastError());
}

void launch_fill_zero(double2* p, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    const int64_t blocks = std::min<int64_t>(ceil_div64(n, 256), 65536);
    hipLaunchKernelGGL(fill_zero_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, p, n);
    GW_HIP_TRY(hipGetLastError());
}

int chi0_tile() { return kTile; }



}  // namespace gw
