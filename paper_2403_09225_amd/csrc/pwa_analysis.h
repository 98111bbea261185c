// Launchers of the kernels used at a minimum (Hessian columns, fit
// fractions).  Internal to the library; not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pwa {

// v = e_j, P entries.
hipError_t launch_unit(double* v, int P, int j, hipStream_t st);
// H <- (H + H^T) / 2, P x P row-major.
hipError_t launch_symmetrise(double* H, int P, hipStream_t st);
// out = theta with every coupling but resonance k's set to zero.
hipError_t launch_mask(const double* theta, double* out, int K, int k, hipStream_t st);
// num[k], row k of dnum (may be null) from a masked pass's partial vector.
hipError_t launch_ff_take(const double* dd, int P, int k, double* num, double* dnum,
                          hipStream_t st);
// Fraction matrix (fit fractions and interference terms) from the MC Gram
// matrix and the couplings in theta.
hipError_t launch_phi(const double* gram, const double* theta, int K, double* phi, hipStream_t st);
// num <- num / G, dnum <- d(num / G) with G, dG from the full model's
// partial vector.
hipError_t launch_ff_finish(const double* dd, int K, int P, double* num, double* dnum,
                            hipStream_t st);

}  // namespace pwa
