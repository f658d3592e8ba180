// The GPP off-diagonal self-energy kernel (internal to libgw).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace gw {

// Energies per launch (the first GEMM's output for a batch stays within 1 GiB).
int gpp_energy_batch(int ns, int ng, int ne);
// Device scratch of run_gpp_sigma.
size_t gpp_bytes(int ns, int ng, int ne);

// sigma[e] (device [ne][ns][ns], overwritten) = sum_n conj(M_n) P^{n e} M_n^T
// with M device [nb][ns][ng], e_n and occupied host [nb], energies_dev device
// [ne] (complex), omega2 device [ng][ng], wt device [ng][ng], v device [ng].
void run_gpp_sigma(const double2* m, int nb, int ns, int ng, const double* e_n,
                   const int32_t* occupied, const double2* energies_dev, int ne,
                   const double2* omega2, const double* wt, const double* v, double2* sigma,
                   char* base, hipStream_t s);

}  // namespace gw
