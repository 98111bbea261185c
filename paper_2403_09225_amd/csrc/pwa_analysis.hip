// Small kernels for the quantities read off at a minimum: the full Hessian
// (from forward-over-reverse passes along unit directions) and the fit
// fractions with their gradients (from MC-only passes with all but one
// coupling switched off).  The event passes themselves are the likelihood
// kernels; these kernels only prepare directions and masked parameter
// vectors and rearrange the per-pass results.

#include "pwa_analysis.h"

namespace pwa {

// v = e_j (P entries).
__global__ __launch_bounds__(256) void unit_kernel(double* __restrict__ v, int P, int j) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < P) v[i] = (i == j) ? 1.0 : 0.0;
}

// H <- (H + H^T) / 2 for a P x P row-major matrix; the thread of (i, j) with
// i < j owns both mirror entries.
__global__ __launch_bounds__(256) void symmetrise_kernel(double* __restrict__ H, int P) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)P * P) return;
  const int i = (int)(t / P), j = (int)(t % P);
  if (i >= j) return;
  const double a = 0.5 * (H[(int64_t)i * P + j] + H[(int64_t)j * P + i]);
  H[(int64_t)i * P + j] = a;
  H[(int64_t)j * P + i] = a;
}

// out = theta with the couplings of every resonance but k set to zero
// (masses and widths kept), so that z = c_k a_k.
__global__ __launch_bounds__(256) void mask_kernel(const double* __restrict__ theta,
                                                   double* __restrict__ out, int K, int k) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 4 * K) return;
  const bool coupling = (i & 3) < 2;
  out[i] = (coupling && (i >> 2) != k) ? 0.0 : theta[i];
}

// From the partial vector of a masked pass (layout [F, G, dF(P), dG(P), ...]
// as (hi, lo) pairs): num[k] = G_k = sum_MC |c_k a_k|^2 and row k of dnum =
// dG_k/dtheta, whose only non-zero entries are resonance k's four.
__global__ __launch_bounds__(256) void ff_take_kernel(const double* __restrict__ dd, int P, int k,
                                                      double* __restrict__ num,
                                                      double* __restrict__ dnum) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) num[k] = dd[2] + dd[3];
  if (dnum && i < P) {
    const int q = 2 + P + i;  // dG/dtheta_i
    dnum[(int64_t)k * P + i] = ((i >> 2) == k) ? dd[2 * q] + dd[2 * q + 1] : 0.0;
  }
}

// F_k = G_k / G and dF_k = dG_k / G - G_k dG / G^2, in place over num and
// dnum; dd is the partial vector of the full model.  One block: every
// thread reads before any writes (a barrier separates them).
__global__ __launch_bounds__(1024) void ff_finish_kernel(const double* __restrict__ dd, int K,
                                                         int P, double* num, double* dnum) {
  const double G = dd[2] + dd[3];
  const double rG = 1.0 / G;
  if (dnum) {
    for (int t = threadIdx.x; t < K * P; t += blockDim.x) {
      const int k = t / P, p = t % P;
      const int q = 2 + P + p;
      const double dG = dd[2 * q] + dd[2 * q + 1];
      dnum[t] = (dnum[t] - num[k] * rG * dG) * rG;
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < K; k += blockDim.x) num[k] = num[k] * rG;
}

static inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

hipError_t launch_unit(double* v, int P, int j, hipStream_t st) {
  hipLaunchKernelGGL(unit_kernel, dim3(blocks_for(P, 256)), dim3(256), 0, st, v, P, j);
  return hipGetLastError();
}

hipError_t launch_symmetrise(double* H, int P, hipStream_t st) {
  hipLaunchKernelGGL(symmetrise_kernel, dim3(blocks_for((int64_t)P * P, 256)), dim3(256), 0, st,
                     H, P);
  return hipGetLastError();
}

hipError_t launch_mask(const double* theta, double* out, int K, int k, hipStream_t st) {
  hipLaunchKernelGGL(mask_kernel, dim3(blocks_for(4 * K, 256)), dim3(256), 0, st, theta, out, K,
                     k);
  return hipGetLastError();
}

hipError_t launch_ff_take(const double* dd, int P, int k, double* num, double* dnum,
                          hipStream_t st) {
  hipLaunchKernelGGL(ff_take_kernel, dim3(blocks_for(P, 256)), dim3(256), 0, st, dd, P, k, num,
                     dnum);
  return hipGetLastError();
}

hipError_t launch_ff_finish(const double* dd, int K, int P, double* num, double* dnum,
                            hipStream_t st) {
  hipLaunchKernelGGL(ff_finish_kernel, dim3(1), dim3(1024), 0, st, dd, K, P, num, dnum);
  return hipGetLastError();
}

}  // namespace pwa
