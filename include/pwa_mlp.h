/* Learned start-point proposal: binned Dalitz histograms and a small MLP
 * (n_in -> n_h1 -> n_h2 -> n_out, GELU on the hidden layers) trained in
 * bfloat16 with FP32 master weights, all on the GPU.
 *
 * The network maps the binned data of a fit to a start point for Newton-CG
 * and is trained on fits that the likelihood library itself performs on toy
 * data.  It adds to the paper's method, whose fits start from random points
 * (Sec. 3, fit-success study); random multi-start remains the fallback.
 *
 * Conventions (as in pwa.h): every array argument is a device pointer unless
 * marked host; the caller owns all memory; calls are asynchronous on
 * `stream`; the library allocates nothing.  Return values are pwa_status
 * codes (0 = PWA_OK; PWA_E_INVALID for bad arguments, PWA_E_WORKSPACE for a
 * short or misaligned workspace, PWA_E_HIP for a failed launch).
 *
 * Parameter packing (FP32 master, gradient, Adam moments): the vector
 *   [W1 (n_h1 x n_in), b1 (n_h1), W2 (n_h2 x n_h1), b2 (n_h2),
 *    W3 (n_out x n_h2), b3 (n_out)]
 * with each W row-major, W[out][in].  Layers: h1 = GELU(W1 x + b1),
 * h2 = GELU(W2 h1 + b2), y = W3 h2 + b3, GELU(x) = x Phi(x) (exact form).
 * Loss: L = sum over batch and outputs of (y - t)^2 / (batch n_out).
 */
#ifndef PWA_MLP_H
#define PWA_MLP_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pwa_mlp_dims {
  int32_t n_in;   /* multiple of 16 */
  int32_t n_h1;   /* multiple of 16 */
  int32_t n_h2;   /* multiple of 16 */
  int32_t n_out;  /* >= 1 */
} pwa_mlp_dims;

/* Normalised 2-D histograms of n_sets event sets over the Dalitz bounding
 * box [(m1+m2)^2, (M-m3)^2] x [(m1+m3)^2, (M-m2)^2] (s12 along rows, s13
 * along columns, nbins x nbins, nbins = 32): set i is events
 * d_offsets[i] .. d_offsets[i+1]-1 of d_s12/d_s13 (FP64); d_offsets holds
 * n_sets + 1 non-decreasing int64 values (device).  d_out: n_sets x 1024
 * floats, bin count / events in the set (0 for an empty set).  Counting is
 * exact (integer), so the result does not depend on scheduling.  An event on
 * an upper edge falls in the last bin; events outside the box are clamped
 * to the border bins.  h_masses: host, 3 doubles.  n_sets <= 65535. */
int pwa_hist2d(const double* d_s12, const double* d_s13, const int64_t* d_offsets,
               int32_t n_sets, double parent_mass, const double* h_masses, float* d_out,
               hipStream_t stream);

/* Number of parameters of the packed vector; 0 for invalid dims. */
int64_t pwa_mlp_n_params(const pwa_mlp_dims* dims);

/* Elements (uint16 bfloat16) of the transposed weight copy: W2^T
 * (n_h1 x n_h2) then W3^T (n_h2 x n_out padded to a multiple of 16, the
 * padding zero), the operands of the backward products; 0 for invalid dims. */
int64_t pwa_mlp_n_transposed(const pwa_mlp_dims* dims);

/* Workspace bytes for batch size `batch` (rounded up to a multiple of 16
 * internally): rounded inputs, pre-activations, activations and the
 * back-propagated signals, in row and column layouts. */
size_t pwa_mlp_workspace_bytes(const pwa_mlp_dims* dims, int32_t batch);

/* Refresh the bfloat16 copies from the FP32 master: d_wbf (n_params
 * uint16, packed like the master) and d_wtbf (pwa_mlp_n_transposed uint16).
 * Round to nearest even. */
int pwa_mlp_cast(const pwa_mlp_dims* dims, const float* d_master, uint16_t* d_wbf,
                 uint16_t* d_wtbf, hipStream_t stream);

/* Forward pass on `batch` inputs d_x (batch x n_in FP32, row-major; rounded
 * to bfloat16 on entry): matrix cores in bfloat16 with FP32 accumulation,
 * biases (FP32, from d_master) and GELU fused into the products' epilogues,
 * hidden activations kept in bfloat16.  Writes d_y (batch x n_out FP32) and
 * keeps what the backward pass needs in d_ws (256-byte aligned,
 * >= pwa_mlp_workspace_bytes). */
int pwa_mlp_forward(const pwa_mlp_dims* dims, const float* d_master, const uint16_t* d_wbf,
                    const float* d_x, int32_t batch, float* d_y, void* d_ws, size_t ws_bytes,
                    hipStream_t stream);

/* pwa_mlp_forward without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops that
 * propose start points, harnesses that forbid hipMalloc).  Same kernels and
 * the same results as pwa_mlp_forward; what that call keeps in d_ws lives
 * instead in a fixed 4 MiB device array inside the library (one copy per GPU,
 * held until the process ends; the call allocates nothing).  The forward
 * buffers must fit in it: with the batch rounded up to 16 rows, 4 n_in +
 * 8 n_h1 + 8 n_h2 bytes per row (each of the 8 buffers rounded up to 256
 * bytes), e.g. batch <= 336 for 1024 -> 512 -> 512 -> 48; larger batches
 * return PWA_E_WORKSPACE.  Every call on one GPU shares that GPU's array, so
 * calls that overlap on one GPU (concurrent streams or threads) race; the
 * array keeps the last call's contents, and nothing in it needs to start at
 * zero.  No backward pass can follow this call (use pwa_mlp_forward for
 * training).  Errors: PWA_E_INVALID, PWA_E_WORKSPACE, PWA_E_HIP. */
int pwa_mlp_forward_noalloc(const pwa_mlp_dims* dims, const float* d_master,
                            const uint16_t* d_wbf, const float* d_x, int32_t batch, float* d_y,
                            hipStream_t stream);

/* Backward pass of the loss against d_target (batch x n_out FP32) for the
 * forward pass last run on d_ws with the same batch: d_grad (n_params FP32,
 * packed like the master) receives dL/dparams, d_loss (1 double) the loss.
 * Back-propagated signals are rounded to bfloat16 before each product;
 * products accumulate in FP32; bias gradients are fixed-order FP32 sums. */
int pwa_mlp_backward(const pwa_mlp_dims* dims, const uint16_t* d_wtbf, const float* d_y,
                     const float* d_target, int32_t batch, void* d_ws, size_t ws_bytes,
                     float* d_grad, double* d_loss, hipStream_t stream);

/* One Adam step (Kingma and Ba, bias-corrected, step >= 1) with decoupled
 * weight decay wd >= 0 (Loshchilov and Hutter):
 *   w <- w - lr (m_hat / (sqrt(v_hat) + eps) + wd w)
 * on the FP32 master with FP32 moments d_m, d_v (n_params each, zero
 * before step 1), then refresh of both bfloat16 copies (as pwa_mlp_cast). */
int pwa_mlp_adam(const pwa_mlp_dims* dims, float* d_master, float* d_m, float* d_v,
                 const float* d_grad, int32_t step, float lr, float beta1, float beta2,
                 float eps, float weight_decay, uint16_t* d_wbf, uint16_t* d_wtbf,
                 hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* PWA_MLP_H */
