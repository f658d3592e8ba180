// Stochastic pseudobands on gfx950 (the Reduced Cost and Scaling section of
// the paper): the bands of each energy slice S are replaced by n_xi
// random-phase combinations
//     xi_j^S(r) = (1/sqrt(n_xi)) sum_{n in S} exp(2 pi i theta_n^j) psi_n(r),
// each with the mean energy of the slice; protected bands are copied as they
// are.  A prep kernel turns the phases into a table of unit complex numbers
// and writes the energies.  The mixing reads every band of a slice once and
// writes n_xi rows: it is bound by HBM bandwidth.  A workgroup owns 64
// consecutive grid points of one slice (one per lane, so each band row is
// read as 1 KiB runs) and its four waves take every fourth band of the
// slice, which keeps many loads in flight even for the largest slice.  The
// band rows are read with non-temporal loads; the band index and phases of a
// step are the same across a wave (scalar loads of adjacent words); the
// waves' n_xi sums meet in LDS at the end; the slices are launched largest
// first.
#include <algorithm>

#include "common.hpp"
#include "prof.hpp"
#include "pseudobands.hpp"

namespace gw {

namespace {

constexpr int kPbThreads = 256;
constexpr int kPbPoints = 64;                      // grid points of one workgroup
constexpr int kPbGroups = kPbThreads / kPbPoints;  // waves splitting the bands of a slice

template <int NX>
__global__ __launch_bounds__(kPbThreads) void pseudo_mix_kernel(
    const double2* __restrict__ psi, int64_t nr, const int* __restrict__ idx,
    const int* __restrict__ off, const int* __restrict__ order,
    const double2* __restrict__ phase, const int64_t* __restrict__ theta_off,
    double2* __restrict__ out, int out_row0) {
    __shared__ double2 s_part[kPbGroups - 1][NX][kPbPoints];
    const int sl = order[blockIdx.y];
    const int b0 = off[sl], nbs = off[sl + 1] - b0;
    const double2* ph = phase + theta_off[sl];  // [nbs][NX]
    const int* ix = idx + b0;
    const int lane = threadIdx.x % kPbPoints;
    const int grp = __builtin_amdgcn_readfirstlane(threadIdx.x / kPbPoints);
    const int64_t r = static_cast<int64_t>(blockIdx.x) * kPbPoints + lane;
    const bool live = r < nr;
    double2 acc[NX];
#pragma unroll
    for (int j = 0; j < NX; ++j) acc[j] = make_double2(0.0, 0.0);
    if (live) {
#pragma unroll 8
        for (int n = grp; n < nbs; n += kPbGroups) {
            // each band row is read once: non-temporal loads keep it from
            // displacing reusable lines in the caches
            const double* q =
                reinterpret_cast<const double*>(psi + static_cast<int64_t>(ix[n]) * nr + r);
            const double2 p = make_double2(__builtin_nontemporal_load(q),
                                           __builtin_nontemporal_load(q + 1));
            const double2* w = ph + static_cast<int64_t>(n) * NX;  // the NX phases of band n
#pragma unroll
            for (int j = 0; j < NX; ++j) {
                acc[j].x += w[j].x * p.x - w[j].y * p.y;
                acc[j].y += w[j].x * p.y + w[j].y * p.x;
            }
        }
    }
    if (grp > 0) {
#pragma unroll
        for (int j = 0; j < NX; ++j) s_part[grp - 1][j][lane] = acc[j];
    }
    __syncthreads();
    if (grp > 0 || !live) return;
#pragma unroll
    for (int g = 0; g < kPbGroups - 1; ++g)
#pragma unroll
        for (int j = 0; j < NX; ++j) {
            const double2 v = s_part[g][j][lane];
            acc[j].x += v.x;
            acc[j].y += v.y;
        }
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

// Workgroup sl < nslices: slice sl's phase table exp(2 pi i theta), band-major
// ([|S|][n_xi], so the phases a mixing step needs are adjacent), and the mean
// of its energies, written to its n_xi rows; the
// workgroups after those copy the energies of the protected bands.
__global__ __launch_bounds__(kPbThreads) void pseudo_prep_kernel(
    const double* __restrict__ e, const int* __restrict__ keep, int nkeep,
    const int* __restrict__ idx, const int* __restrict__ off, const double* __restrict__ theta,
    const int64_t* __restrict__ theta_off, int nslices, int n_xi, double2* __restrict__ phase,
    double* __restrict__ out_e) {
    __shared__ double s_sum[kPbThreads / 64];
    const int b = blockIdx.x;
    if (b >= nslices) {
        const int t = (b - nslices) * kPbThreads + threadIdx.x;
        if (t < nkeep) out_e[t] = e[keep[t]];
        return;
    }
    const int b0 = off[b], nbs = off[b + 1] - b0;
    const int64_t t0 = theta_off[b];
    for (int t = threadIdx.x; t < n_xi * nbs; t += kPbThreads) {
        const int j = t / nbs, n = t - j * nbs;
        double sn, cs;
        sincospi(2.0 * theta[t0 + t], &sn, &cs);
        phase[t0 + static_cast<int64_t>(n) * n_xi + j] = make_double2(cs, sn);
    }
    double sum = 0.0;
    for (int n = threadIdx.x; n < nbs; n += kPbThreads) sum += e[idx[b0 + n]];
    for (int d = 32; d > 0; d /= 2) sum += __shfl_xor(sum, d, 64);
    if (threadIdx.x % 64 == 0) s_sum[threadIdx.x / 64] = sum;
    __syncthreads();
    if (threadIdx.x < n_xi) {
        double tot = 0.0;
        for (int w = 0; w < kPbThreads / 64; ++w) tot += s_sum[w];
        out_e[nkeep + b * n_xi + threadIdx.x] = tot / static_cast<double>(nbs);
    }
}

using MixKernel = void (*)(const double2*, int64_t, const int*, const int*, const int*,
                           const double2*, const int64_t*, double2*, int);

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
    {
        ProfScope ps("pseudo_prep", s);
        hipLaunchKernelGGL(pseudo_prep_kernel, dim3(nslices + ceil_div(nkeep, kPbThreads)),
                           dim3(kPbThreads), 0, s, e, t.keep, nkeep, t.idx, t.off, t.theta,
                           t.theta_off, nslices, n_xi, t.phase, out_e);
        GW_HIP_TRY(hipGetLastError());
    }
    if (nkeep > 0) {
        ProfScope ps("pseudo_keep", s);
        const unsigned gr = static_cast<unsigned>(ceil_div64(nr, kPbThreads));
        hipLaunchKernelGGL(pseudo_keep_kernel, dim3(std::min(gr, 4096u), nkeep), dim3(kPbThreads),
                           0, s, psi, nr, t.keep, out_psi);
        GW_HIP_TRY(hipGetLastError());
    }
    if (nslices > 0) {
        ProfScope ps("pseudo_mix", s);
        const unsigned gm = static_cast<unsigned>(ceil_div64(nr, kPbPoints));
        hipLaunchKernelGGL(select_mix(n_xi), dim3(gm, nslices), dim3(kPbThreads), 0, s, psi, nr,
                           t.idx, t.off, t.order, t.phase, t.theta_off, out_psi, nkeep);
        GW_HIP_TRY(hipGetLastError());
    }
}

}  // namespace gw
