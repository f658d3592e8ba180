// Host entry of the pseudoband kernels (internal to libgw).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gw {

constexpr int kMaxPseudoXi = 8;  // pseudobands per slice

// Device copies of the caller's host tables.
struct PseudoTables {
    const int* keep;          // [nkeep] protected band indices
    const int* idx;           // [off[nslices]] band indices of the slices, slice by slice
    const int* off;           // [nslices + 1] slice s is idx[off[s] .. off[s+1])
    const int* order;         // [nslices] the slices in launch order (largest first)
    const double* theta;      // per slice [n_xi][|S|] phases in turns
    const int64_t* theta_off; // [nslices] start of slice s in theta and phase
    double2* phase;           // per slice [|S|][n_xi] exp(2 pi i theta), written by the prep kernel
};

void launch_pseudobands(const double2* psi, const double* e, int64_t nr, const PseudoTables& t,
                        int nkeep, int nslices, int n_xi, double2* out_psi, double* out_e,
                        hipStream_t s);

}  // namespace gw
