// Exchange-correlation step on the grid (xc.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace aims {

constexpr int kXcBlocks = 256;   // blocks per system of the pointwise kernels

// v_out[q] = v_xc(n[q]) (caller order) of the spin-unpolarised LDA (Slater + PW92); with
// sums_or_null, sums[s] = (E_xc = sum w n eps_xc, sum w n v_xc) per system.  part: 2 kXcBlocks
// n_sys doubles of scratch.
hipError_t launch_lda(const DeviceView& dv, const double* n, double* v_out, double* part,
                      double* sums_or_null, hipStream_t st);

// PBE: v_out = df/dn, u_out = 4 (df/dsigma) grad n (3 per point, caller order); sums[s] =
// (E_xc = sum w f, sum w (n v_n + 2 sigma v_sigma))
hipError_t launch_pbe(const DeviceView& dv, const double* n, const double* grad, double* v_out,
                      double* u_out, double* part, double* sums_or_null, hipStream_t st);

// grad_out[q] (caller order, 3 per point) = 2 sum_j X_pj grad phi_j(p) for the batches
// [b0, b0 + nbatch) of dv, X^T being the function-major slab of the X pass (FP64)
hipError_t launch_gradn(const DeviceView& dv, int b0, int nbatch, const double* X, double* grad_out,
                        hipStream_t st);

// slab2 += w_p u_p . grad phi_j(p) (the gradient term of the H integrand) for the batches
// [b0, b0 + nbatch) of dv; u: [n_points][3] caller order
template <typename T>
hipError_t launch_vector_term(const DeviceView& dv, int b0, int nbatch, const double* u, T* slab2,
                              hipStream_t st);

}  // namespace aims
