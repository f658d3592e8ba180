// Stochastic pseudobands on gfx950 (the Reduced Cost and Scaling section of
// the paper): the bands of each energy slice S are replaced by n_xi
// random-phase combinations
//     xi_j^S(r) = (1/sqrt(n_xi)) sum_{n in S} exp(2 pi i theta_n^j) psi_n(r),
// each with the mean energy of the slice; protected bands are copied as they
// are.  The mixing reads every band of a slice once and writes n_xi rows:
// it is bound by HBM bandwidth, so one thread owns one grid point r of one
// slice (coalesced rows) and keeps the n_xi sums in registers; the phases of
// the slice are formed once per workgroup in LDS, a chunk of bands at a time.
#include <algorithm>

#include "common.hpp"
#include "prof.hpp"
#include "pseudobands.hpp"

namespace gw {

namespace {

constexpr int kPbThreads = 256;
constexpr int kPbChunk = 256;  // bands whose phases are staged in LDS at once

template <int NX>
__global__ __launch_bounds__(kPbThreads) void pseudo_mix_kernel(
    const double2* __restrict__ psi, int64_t nr, const int* __restrict__ idx,
    const int* __restrict__ off, const double* __restrict__ theta,
    const int64_t* __restrict__ theta_off, double2* __restrict__ out, int out_row0) {
    __shared__ double2 s_ph[NX][kPbChunk];
    const int sl = blockIdx.y;
    const int b0 = off[sl], nbs = off[sl + 1] - b0;
    const double* th = theta + theta_off[sl];  // [NX][nbs]
    const int64_t r = static_cast<int64_t>(blockIdx.x) * kPbThreads + threadIdx.x;
    double2 acc[NX];
#pragma unroll
    for (int j = 0; j < NX; ++j) acc[j] = make_double2(0.0, 0.0);
    for (int c0 = 0; c0 < nbs; c0 += kPbChunk) {
        const int cn = min(kPbChunk, nbs - c0);
        __syncthreads();  // the previous chunk's phases are no longer read
        for (int t = threadIdx.x; t < NX * cn; t += kPbThreads) {
            const int j = t / cn, n = t - j * cn;
            double sn, cs;
            sincospi(2.0 * th[static_cast<int64_t>(j) * nbs + c0 + n], &sn, &cs);
            s_ph[j][n] = make_double2(cs, sn);
        }
        __syncthreads();
        if (r < nr) {
#pragma unroll 4
            for (int n = 0; n < cn; ++n) {
                const double2 p = psi[static_cast<int64_t>(idx[b0 + c0 + n]) * nr + r];
#pragma unroll
                for (int j = 0; j < NX; ++j) {
                    const double2 w = s_ph[j][n];
                    acc[j].x += w.x * p.x - w.y * p.y;
                    acc[j].y += w.x * p.y + w.y * p.x;
                }
            }
        }
    }
    if (r >= nr) return;
    const double sc = 1.0 / sqrt(static_cast<double>(NX));
#pragma unroll
    for (int j = 0; j < NX; ++j)
        out[(static_cast<int64_t>(out_row0) + static_cast<int64_t>(sl) * NX + j) * nr + r] =
            make_double2(sc * acc[j].x, sc * acc[j].y);
}

// Protected bands: row i of the output is band keep[i].
__global__ __launch_bounds__(kPbThreads) void pseudo_keep_kernel(
    const double2* __restrict__ psi, int64_t nr, const int* __restrict__ keep,
    double2* __restrict__ out) {
    const int i = blockIdx.y;
    const int64_t src = static_cast<int64_t>(keep[i]) * nr;
    for (int64_t r = static_cast<int64_t>(blockIdx.x) * kPbThreads + threadIdx.x; r < nr;
         r += static_cast<int64_t>(gridDim.x) * kPbThreads)
        out[static_cast<int64_t>(i) * nr + r] = psi[src + r];
}

// Energies: the protected ones copied, each slice's mean (summed in band order)
// written to its n_xi rows.
__global__ __launch_bounds__(kPbThreads) void pseudo_energy_kernel(
    const double* __restrict__ e, const int* __restrict__ keep, int nkeep,
    const int* __restrict__ idx, const int* __restrict__ off, int nslices, int n_xi,
    double* __restrict__ out_e) {
    const int t = blockIdx.x * kPbThreads + threadIdx.x;
    if (t < nkeep) {
        out_e[t] = e[keep[t]];
    } else if (t < nkeep + nslices) {
        const int sl = t - nkeep, b0 = off[sl], b1 = off[sl + 1];
        double sum = 0.0;
        for (int b = b0; b < b1; ++b) sum += e[idx[b]];
        const double mean = sum / static_cast<double>(b1 - b0);
        for (int j = 0; j < n_xi; ++j) out_e[nkeep + sl * n_xi + j] = mean;
    }
}

using MixKernel = void (*)(const double2*, int64_t, const int*, const int*, const double*,
                           const int64_t*, double2*, int);

MixKernel select_mix(int n_xi) {
    static const MixKernel table[kMaxPseudoXi] = {
        &pseudo_mix_kernel<1>, &pseudo_mix_kernel<2>, &pseudo_mix_kernel<3>,
        &pseudo_mix_kernel<4>, &pseudo_mix_kernel<5>, &pseudo_mix_kernel<6>,
        &pseudo_mix_kernel<7>, &pseudo_mix_kernel<8>};
    return table[n_xi - 1];
}

}  // namespace

void launch_pseudobands(const double2* psi, const double* e, int64_t nr, const PseudoTables& t,
                        int nkeep, int nslices, int n_xi, double2* out_psi, double* out_e,
                        hipStream_t s) {
    if (nkeep + nslices == 0) return;
    const unsigned gr = static_cast<unsigned>(ceil_div64(nr, kPbThreads));
    {
        ProfScope ps("pseudo_energy", s);
        hipLaunchKernelGGL(pseudo_energy_kernel, dim3(ceil_div(nkeep + nslices, kPbThreads)),
                           dim3(kPbThreads), 0, s, e, t.keep, nkeep, t.idx, t.off, nslices, n_xi,
                           out_e);
        GW_HIP_TRY(hipGetLastError());
    }
    if (nkeep > 0) {
        ProfScope ps("pseudo_keep", s);
        hipLaunchKernelGGL(pseudo_keep_kernel, dim3(std::min(gr, 4096u), nkeep), dim3(kPbThreads),
                           0, s, psi, nr, t.keep, out_psi);
        GW_HIP_TRY(hipGetLastError());
    }
    if (nslices > 0) {
        ProfScope ps("pseudo_mix", s);
        hipLaunchKernelGGL(select_mix(n_xi), dim3(gr, nslices), dim3(kPbThreads), 0, s, psi, nr,
                           t.idx, t.off, t.theta, t.theta_off, out_psi, nkeep);
        GW_HIP_TRY(hipGetLastError());
    }
}

}  // namespace gw
