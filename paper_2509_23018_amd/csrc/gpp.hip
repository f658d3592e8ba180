// The GPP off-diagonal self-energy kernel (Optimized GPP Kernel for
// Off-Diagonal Self-Energy Matrix Elements section of the paper): the full
// matrix Sigma_lm(E) on a grid of energies,
//     Sigma_lm(E) = sum_n sum_GG' conj(M_ln(G)) P^{nE}_GG' M_mn(G'),
// as the paper casts it, two complex GEMMs per (band n, energy E):
//   T = conj(M_n) P^{nE}        (N_Sigma x N_G x N_G)
//   Sigma(E) += T M_n^T         (N_Sigma x N_G x N_Sigma).
// The plasmon-pole inner matrix is
//     P_GG' = Omega2_GG' v_G' / (2 wt_GG' (E - E_n - s_n wt_GG')),
// s_n = -1 (occupied) or +1 (empty).  Here it is never stored: the first
// GEMM forms each 16 x 64 stage of P from Omega2, wt and v as it writes the
// stage to LDS (a complex division per element, for every energy of the
// launch), so P costs no HBM traffic; that GEMM runs over all energies of a
// batch in one launch (one workgroup grid per energy), and the second is one
// batched GEMM over the same energies.
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "gpp.hpp"
#include "linalg.hpp"
#include "prof.hpp"

namespace gw {
namespace {

// T[e][l][G'] = sum_G conj(M[l][G]) P_e[G][G'] for one band: 64 (l) x 64 (G')
// tiles, 4 waves of 32 x 32 on the 16x16x4 FP64 MFMA, G staged 16 at a time
// through registers and LDS, three real products per complex multiply-add.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void gpp_t_kernel(
    const double2* __restrict__ m, int ns, int ng, const double2* __restrict__ omega2,
    const double* __restrict__ wt, const double* __restrict__ v,
    const double2* __restrict__ energies, double en, double sn, double2* __restrict__ t) {
    __shared__ double2 s_a[64][17];  // [l][G]
    __shared__ double2 s_b[16][65];  // [G][G']
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63, row = lane & 15, kq = lane >> 4;
    const int wi = wave >> 1, wj = wave & 1;
    const int64_t e = blockIdx.z;
    const double2 ee = energies[e];
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    const int llast = ns - 1, glast = ng - 1;

    dbl4 p1[2][2], p2[2][2], p3[2][2];
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) p1[x][y] = p2[x][y] = p3[x][y] = zero4();

    double2 ra[4], ro[4];
    double rw[4], rv[4];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int q = tid + 256 * u;
            const double2* sa = m + static_cast<int64_t>(min(i0 + (q >> 4), llast)) * ng +
                                min(k0 + (q & 15), glast);
            ra[u].x = sa->x;
            ra[u].y = sa->y;
            const int64_t o = static_cast<int64_t>(min(k0 + (q >> 6), glast)) * ng +
                              min(j0 + (q & 63), glast);
            ro[u].x = omega2[o].x;
            ro[u].y = omega2[o].y;
            rw[u] = wt[o];
            rv[u] = v[min(j0 + (q & 63), glast)];
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < ng; k0 += 16) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int q = tid + 256 * u;
            const int ll = q >> 4, ka = q & 15;
            const bool oka = i0 + ll < ns && k0 + ka < ng;
            s_a[ll][ka] = oka ? make_double2(ra[u].x, -ra[u].y) : make_double2(0.0, 0.0);
            const int kb = q >> 6, gg = q & 63;
            double2 pv = make_double2(0.0, 0.0);
            if (k0 + kb < ng && j0 + gg < ng) {
                // P = Omega2 v / (2 wt (E - E_n - s wt)), E complex
                const double w2 = 2.0 * rw[u];
                const double dr = w2 * (ee.x - en - sn * rw[u]), di = w2 * ee.y;
                const double inv = rv[u] / (dr * dr + di * di);
                pv = make_double2((ro[u].x * dr + ro[u].y * di) * inv,
                                  (ro[u].y * dr - ro[u].x * di) * inv);
            }
            s_b[kb][gg] = pv;
        }
        __syncthreads();
        __builtin_amdgcn_s_setprio(1);
        if (k0 + 16 < ng) fetch(k0 + 16);
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
    double2* te = t + e * static_cast<int64_t>(ns) * ng;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int r = i0 + wi * 32 + x * 16 + 4 * q + kq;
                const int c = j0 + wj * 32 + y * 16 + row;
                if (r < ns && c < ng)
                    te[static_cast<int64_t>(r) * ng + c] =
                        make_double2(p1[x][y][q] - p2[x][y][q], p3[x][y][q] - p1[x][y][q] - p2[x][y][q]);
            }
}

__global__ __launch_bounds__(256) void zero_kernel(double2* __restrict__ p, int64_t n) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = make_double2(0.0, 0.0);
}

}  // namespace

int gpp_energy_batch(int ns, int ng, int ne) {
    // T of a batch within 1 GiB, at least one energy
    const size_t per = static_cast<size_t>(ns) * ng * sizeof(double2);
    return std::max(1, std::min<int>(ne, static_cast<int>((size_t(1) << 30) / std::max<size_t>(per, 1))));
}

size_t gpp_bytes(int ns, int ng, int ne) {
    const int eb = gpp_energy_batch(ns, ng, ne);
    const size_t t = static_cast<size_t>(eb) * ns * ng * sizeof(double2);
    return ((t + 255) & ~size_t(255)) + ((static_cast<size_t>(ne) * sizeof(double2) + 255) & ~size_t(255));
}

void run_gpp_sigma(const double2* m, int nb, int ns, int ng, const double* e_n,
                   const int32_t* occupied, const double2* energies_dev, int ne,
                   const double2* omega2, const double* wt, const double* v, double2* sigma,
                   char* base, hipStream_t s) {
    const int eb = gpp_energy_batch(ns, ng, ne);
    double2* t = reinterpret_cast<double2*>(base);
    const int64_t sig = static_cast<int64_t>(ns) * ns;
    {
        const int64_t n = sig * ne;
        hipLaunchKernelGGL(zero_kernel, dim3(static_cast<unsigned>(std::min<int64_t>(ceil_div64(n, 256), 4096))),
                           dim3(256), 0, s, sigma, n);
        GW_HIP_TRY(hipGetLastError());
    }
    if (nb == 0 || ns == 0 || ng == 0) return;
    for (int e0 = 0; e0 < ne; e0 += eb) {
        const int ec = std::min(eb, ne - e0);
        for (int n = 0; n < nb; ++n) {
            const double2* mn = m + static_cast<int64_t>(n) * ns * ng;
            {
                ProfScope ps("gpp_t", s);
                hipLaunchKernelGGL(gpp_t_kernel,
                                   dim3(static_cast<unsigned>(ceil_div(ng, 64)),
                                        static_cast<unsigned>(ceil_div(ns, 64)), ec),
                                   dim3(256), 0, s, mn, ns, ng, omega2, wt, v, energies_dev + e0,
                                   e_n[n], occupied[n] ? -1.0 : 1.0, t);
                GW_HIP_TRY(hipGetLastError());
            }
            ZGemm g;  // Sigma(E) += T M_n^T for the batch's energies
            g.m = ns;
            g.n = ns;
            g.k = ng;
            g.a = t;
            g.lda = ng;
            g.stride_a = static_cast<int64_t>(ns) * ng;
            g.b = mn;
            g.ldb = ng;
            g.stride_b = 0;
            g.c = sigma + e0 * sig;
            g.ldc = ns;
            g.stride_c = sig;
            g.beta = make_double2(1.0, 0.0);
            g.batch = ec;
            launch_zgemm(kOpN, kOpT, g, s);
        }
    }
}

}  // namespace gw
