// Inverse dielectric matrix of Eq. (3) (internal to libgw).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace gw {

// Device scratch of run_epsinv.
size_t epsinv_bytes(int ng, int nz);

// out[w] = [I - diag(v) chi[w]]^-1 for w < nz; chi and out device [nz][ng][ng]
// (distinct), v device [ng].  Asynchronous.
void run_epsinv(const double2* chi, int ng, int nz, const double* v, double2* out, char* base,
                hipStream_t s);

}  // namespace gw
