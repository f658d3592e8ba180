// Adjoint of the chi0 build (internal to libgw).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <functional>

#include "gw.h"
#include "plan.hpp"

namespace gw {

// Gradients of a real loss with respect to psi_v, psi_c, E_v and E_c given
// grad_chi = dL/dchi (PyTorch complex convention).  Outputs are overwritten;
// any may be NULL.  `get_scratch(bytes)` returns device scratch valid on s.
void run_chi0_backward(const MtxelPlan& plan, const gw_problem_t& p, const double2* grad_chi,
                       double2* grad_psi_v, double2* grad_psi_c, double* grad_e_v,
                       double* grad_e_c, double spin, int pair_chunk, hipStream_t s,
                       const std::function<void*(size_t)>& get_scratch);

}  // namespace gw
