// Small kernels for the quantities read off at a minimum: the full Hessian
// (from forward-over-reverse passes along unit directions), the fit
// fractions with their gradients (from MC-only passes with all but one
// coupling switched off) and the fraction matrix with the interference
// terms (from the MC Gram matrix).  The event passes themselves are the
// likelihood and Gram kernels; these kernels only prepare directions and
// masked parameter vectors and rearrange the per-pass results.

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

// Fraction matrix from the MC Gram matrix Gm[k][l] = sum_MC conj(a_k) a_l
// ((re, im) pairs, row-major) and the couplings in theta: with
// y_k = c_k a_k, sum_MC conj(y_k) y_l = conj(c_k) c_l Gm[k][l], so
//   D = sum_kl Re(conj(c_k) c_l Gm[k][l]) = sum_MC |z|^2,
//   phi[k][k] = |c_k|^2 Re Gm[k][k] / D,
//   phi[k][l] = 2 Re(conj(c_k) c_l Gm[k][l]) / D  (k < l),  0 below.
// One block; D is summed in a fixed order by thread 0.
__global__ __launch_bounds__(1024) void phi_kernel(const double* __restrict__ gram,
                                                   const double* __restrict__ theta, int K,
                                                   double* __restrict__ phi) {
  __shared__ double sD;
  auto term = [&](int k, int l) {
    const double ckr = theta[4 * k], cki = theta[4 * k + 1];
    const double clr = theta[4 * l], cli = theta[4 * l + 1];
    // conj(c_k) c_l
    const double pr = ckr * clr + cki * cli, pi = ckr * cli - cki * clr;
    const double gr = gram[2 * (k * K + l)], gi = gram[2 * (k * K + l) + 1];
    return pr * gr - pi * gi;
  };
  if (threadIdx.x == 0) {
    double D = 0.0;
    for (int k = 0; k < K; ++k)
      for (int l = 0; l < K; ++l) D += term(k, l);
    sD = D;
  }
  __syncthreads();
  const double rD = 1.0 / sD;
  for (int i = threadIdx.x; i < K * K; i += blockDim.x) {
    const int k = i / K, l = i % K;
    phi[i] = (l < k) ? 0.0 : (l == k ? term(k, k) : 2.0 * term(k, l)) * rD;
  }
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

hipError_t launch_phi(const double* gram, const double* theta, int K, double* phi, hipStream_t st) {
  hipLaunchKernelGGL(phi_kernel, dim3(1), dim3(1024), 0, st, gram, theta, K, phi);
  return hipGetLastError();
}

hipError_t launch_ff_finish(const double* dd, int K, int P, double* num, double* dnum,
                            hipStream_t st) {
  hipLaunchKernelGGL(ff_finish_kernel, dim3(1), dim3(1024), 0, st, dd, K, P, num, dnum);
  return hipGetLastError();
}

}  // namespace pwa
