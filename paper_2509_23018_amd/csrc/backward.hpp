// Adjoint of the chi0 build (internal to libgw).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "gw.h"
#include "plan.hpp"

namespace gw {

// Gradients of a real loss with respect to psi_v, psi_c, E_v and E_c given
// grad_chi = dL/dchi (PyTorch complex convention).  Outputs are overwritten;
// any may be NULL.  `base` is device scratch of chi0_backward_bytes(...)
// bytes for the same problem, outputs wanted and pair_chunk, valid on s.
// `aux` is a companion stream (MTXEL of the next chunk runs there) and ev[0..4]
// five events for the hand-over between the two; s waits for all of aux's work.
// With m_keep (M kept by gw_chi0_keep_m for the same problem and pair_chunk)
// no MTXEL runs and scratch is chi0_backward_bytes(..., kept = true); a chunk
// shape other than the forward's is an Error with GW_EINVAL.
void run_chi0_backward(const MtxelPlan& plan, const gw_problem_t& p, const double2* grad_chi,
                       double2* grad_psi_v, double2* grad_psi_c, double* grad_e_v,
                       double* grad_e_c, double spin, int pair_chunk, hipStream_t s, char* base,
                       hipStream_t aux, hipEvent_t* ev, const double2* m_keep = nullptr);
size_t chi0_backward_bytes(const MtxelPlan& plan, const gw_problem_t& p, bool want_psi_v,
                           bool want_psi_c, bool want_e, int pair_chunk, bool kept = false);

}  // namespace gw
