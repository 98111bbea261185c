/*
 * pwa.h -- C ABI of the MI355X partial-wave-analysis likelihood library.
 *
 * The library evaluates the unbinned negative log-likelihood of a
 * three-body Dalitz-plot model, its gradient and its Hessian-vector product
 * (arXiv:2403.09225, Sec. 2.2 eq. (1)-(3) and Sec. 2.3 eq. (4)-(7)), and
 * drives a Newton-conjugate-gradient fit with them (Sec. 3, the
 * "NTCG+AutoDiff" method).  Every step of the evaluation runs in HIP kernels
 * written for gfx950.
 *
 * Conventions for every entry point:
 *   - Plain C: no C++ types or exceptions cross this boundary.
 *   - Array arguments named d_* are DEVICE pointers; everything else
 *     (pwa_model, pwa_fit_opts, pwa_fit_report) lives in host memory.
 *   - The caller owns all device memory.  The library never allocates device
 *     memory; the workspace is the caller's buffer of pwa_workspace_bytes().
 *   - Calls taking a hipStream_t only enqueue work on that stream and return
 *     at once (the exception is pwa_fit, which synchronises).  Outputs are
 *     valid once the stream reaches the enqueued work.
 *   - A context is not thread-safe; several contexts may coexist.
 *   - Return value: PWA_OK (0) or a negative pwa_status.  Arguments are
 *     validated on the host before any HIP call, so bad arguments are
 *     reported without touching the device.
 *
 * Physics conventions (the paper is silent on them; these are the readings):
 *   - Parent of spin 0 (or 1, see pwa_bind_oriented) decaying to three
 *     distinguishable pseudoscalars with masses m[0..2]; an event is
 *     x = (s12, s13), s_ij = (p_i + p_j)^2 in GeV^2;
 *     s23 = M^2 + sum m_i^2 - s12 - s13.
 *   - Channel c: 0 = (12) with bachelor 3, 1 = (13) with bachelor 2,
 *     2 = (23) with bachelor 1.  The helicity angle of channel (ab) is the
 *     angle, in the (ab) rest frame, between a and the direction opposite to
 *     the bachelor.
 *   - Amplitude of resonance k (channel c, spin J in {0,1,2}):
 *       a_k = P_J(cos th) [F_J(z)/F_J(z0)] / (M_k^2 - s - i M_k Gamma_k(s)),
 *       Gamma_k(s) = Gamma_k (q/q0)^(2J+1) (M_k/sqrt s) [F_J(z)/F_J(z0)]^2,
 *     with q the breakup momentum, q0 = q(s = M_k^2), z = (q r)^2, and
 *     Blatt-Weisskopf F_0 = 1, F_1 = (1+z)^-1/2, F_2 = (z^2+3z+9)^-1/2.
 *     PWA_WIDTH_CONSTANT sets Gamma_k(s) = Gamma_k.  A scalar resonance may
 *     instead take the Flatte form (pwa_lineshape).
 *   - Intensity (eq. (1)): w(x) = |sum_k c_k a_k(x)|^2 for a spin-0 parent
 *     (one helicity term), sum over mu = +-1 of |sum_k c_k a_k^mu(x)|^2 for a
 *     spin-1 parent.
 *   - NLL = -ln L = -sum_data ln w + N_D ln( (1/N_MC) sum_MC w )  (eq. (3)).
 *   - Parameter vector theta (P = 4K doubles), k-major:
 *       theta[4k+0] = Re c_k, theta[4k+1] = Im c_k,
 *       theta[4k+2] = M_k,    theta[4k+3] = Gamma_k (g_1 for a Flatte
 *       resonance).
 *   - A resonance mass at or below its pair threshold, or a non-positive
 *     intensity sum, is not an error: the NLL is +inf and a device status
 *     bit is set (read it with pwa_device_status).
 */
#ifndef PWA_H
#define PWA_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PWA_MAX_RES 64

typedef enum pwa_status {
  PWA_OK = 0,
  PWA_E_INVALID = -1,   /* null pointer, bad size, bad channel/spin, ...     */
  PWA_E_WORKSPACE = -2, /* workspace missing, too small or misaligned        */
  PWA_E_HIP = -3,       /* a HIP runtime call failed (e.g. no device)        */
  PWA_E_DOMAIN = -4,    /* fit start point outside the model's domain        */
  PWA_E_NOCONV = -5,    /* fit stopped without meeting xtol; theta = best    */
  PWA_E_STATE = -6      /* context not bound to events yet                   */
} pwa_status;

/* Arithmetic of the per-event evaluation.  Event sums are always FP64. */
typedef enum pwa_precision {
  PWA_PREC_F64 = 0, /* FP64 event stream and FP64 per-event arithmetic       */
  PWA_PREC_F32 = 1  /* FP32 event stream and arithmetic, FP64 accumulation   */
} pwa_precision;

/* Which event streams pwa_bind materialises (bit mask). */
#define PWA_STREAM_F64 1
#define PWA_STREAM_F32 2

typedef enum pwa_width_mode {
  PWA_WIDTH_MASS_DEPENDENT = 0,
  PWA_WIDTH_CONSTANT = 1
} pwa_width_mode;

/* Lineshape of a resonance.  The paper's test model includes f0(980) in the
 * Flatte form (Sec. 3, Table 1); the form is not written out there, and this
 * is the reading: for a scalar (J = 0) resonance of channel (ab) with a
 * coupled second channel of masses flatte_masses and coupling ratio
 * r = flatte_ratio = g_2 / g_1,
 *   a_k = 1 / (M_k^2 - s - i g_1 [rho_ab(s) + r rho_2(s)]),
 *   rho(s) = sqrt(lambda(s, m_1^2, m_2^2)) / s  (= 2 q / sqrt s),
 * continued below the second threshold on the physical sheet,
 * rho_2 = +i sqrt(-lambda) / s.  theta[4k+3] is then g_1 (GeV^2) instead of
 * Gamma_k; no barrier or angular factor (J = 0). */
typedef enum pwa_lineshape {
  PWA_LINESHAPE_BREIT_WIGNER = 0,
  PWA_LINESHAPE_FLATTE = 1
} pwa_lineshape;

/* Model description (host memory, copied by pwa_create).  Zero-initialise
 * it: the fields after `spin` default to a spin-0 parent and Breit-Wigner
 * resonances. */
typedef struct pwa_model {
  double parent_mass;          /* GeV                                          */
  double masses[3];            /* daughter masses m1, m2, m3 (GeV)             */
  double r;                    /* Blatt-Weisskopf radius (GeV^-1)              */
  int32_t n_res;               /* K, 1 <= K <= PWA_MAX_RES                      */
  int32_t width_mode;          /* pwa_width_mode (Breit-Wigner resonances)     */
  int32_t channel[PWA_MAX_RES];/* channel of resonance k: 0, 1 or 2            */
  int32_t spin[PWA_MAX_RES];   /* spin J of resonance k: 0, 1 or 2             */
  int32_t lineshape[PWA_MAX_RES]; /* pwa_lineshape of resonance k             */
  double flatte_masses[2];     /* second channel of the Flatte resonances (GeV) */
  double flatte_ratio;         /* r = g_2 / g_1 of the Flatte resonances (>= 0) */
  int32_t parent_spin;         /* 0, or 1: a vector parent polarised along z
                                  with mu = +1, -1 (see pwa_bind_oriented)    */
  int32_t reserved;
} pwa_model;

typedef struct pwa_ctx pwa_ctx;

/* Create a context for `model` (host memory, copied).  Models with a
 * Flatte resonance or a spin-1 parent (the general physics path) take at
 * most 16 resonances.
 * streams: PWA_STREAM_F64 and/or PWA_STREAM_F32 -- the event streams pwa_bind
 * will build (both are needed for mixed-precision fits).
 * Errors: PWA_E_INVALID for a null pointer, K out of range, a channel or spin
 * out of range, non-positive masses, r <= 0, an empty stream mask, or a
 * parent mass not above the sum of the daughter masses. */
int pwa_create(const pwa_model* model, int32_t streams, pwa_ctx** out);

/* Destroy a context (null is accepted).  Owns no device memory. */
void pwa_destroy(pwa_ctx* ctx);

/* Device workspace (bytes) needed to bind n_data data and n_mc MC events:
 * the parameter-free event stream (the paper's precomputed U, Sec. 2.2:
 * per channel s, per (channel, J) the width factor and, for J >= 1, the
 * angular factor, for each event), the resonance table, the per-block
 * partial sums and the status words.  0 on invalid arguments. */
size_t pwa_workspace_bytes(const pwa_ctx* ctx, int64_t n_data, int64_t n_mc);

/* Bind events and build the parameter-free event stream in the workspace
 * (Sec. 2.2: the parameter-free factors are computed once and kept on the
 * GPU).  d_s12/d_s13: n_data data events; d_mc_s12/d_mc_s13: n_mc MC events
 * (phase-space distributed, efficiency 1); FP64, contiguous.  The event
 * arrays are read on `stream` during this call and not retained.
 * d_ws: caller-owned device buffer of ws_bytes >= pwa_workspace_bytes(),
 * 256-byte aligned; it must stay allocated while the context is used.
 * n_data >= 0, n_mc >= 1, n_data + n_mc <= 2^29 - 256 (536 870 656) events
 * per context, or 357 000 000 with an FP32 stream (32-bit offsets within
 * the stream planes); larger samples are sharded over contexts and combined
 * with pwa_partials / pwa_combine.
 * Errors: PWA_E_INVALID (null pointers, sizes), PWA_E_WORKSPACE, PWA_E_HIP. */
int pwa_bind(pwa_ctx* ctx, const double* d_s12, const double* d_s13, int64_t n_data,
             const double* d_mc_s12, const double* d_mc_s13, int64_t n_mc,
             void* d_ws, size_t ws_bytes, hipStream_t stream);

/* pwa_bind for a spin-1 parent (pwa_model.parent_spin = 1), whose events
 * carry the orientation of the decay besides (s12, s13).  The paper's
 * intensity sums the squared amplitude over the parent's helicity index mu
 * (eq. (1): w = 1/2 sum_mu |A^mu|^2, with U_m^mu the parameter-free part);
 * here mu = +1, -1 for a vector parent polarised along the z axis of its rest
 * frame, and the constant 1/2 is dropped (it cancels in eq. (3)).  Reading
 * (the paper's covariant tensors are not given): in the parent rest frame
 * the daughters' momenta p_i lie in the plane reached from the reference
 * plane (p_1 along x, p_2 in the upper x-y half plane) by the rotation
 * R_y(beta) R_z(gamma); for channel (ab) with bachelor c, with p^_c the unit
 * bachelor momentum and q^ the unit momentum of a in the (ab) rest frame
 * (boosted along the pair's momentum), and the polarisation vectors
 * e_+ = -(1, i, 0)/sqrt2, e_- = (1, -i, 0)/sqrt2,
 *   U^mu = F_J(z) Y_J^mu:  Y_0 = e.p^_c,  Y_1 = e.(p^_c x q^),
 *   Y_2 = (e.q^)(q^.p^_c) - (e.p^_c)/3,
 * times the lineshape (parity is not imposed: the workload is synthetic).
 * d_cosb, d_gamma: cos(beta) in [-1, 1] and gamma (radians) per event, FP64,
 * beside the (s12, s13) arrays of each set.  Other arguments and errors as
 * pwa_bind; pwa_bind rejects a spin-1 parent model with PWA_E_INVALID and
 * this call a spin-0 one. */
int pwa_bind_oriented(pwa_ctx* ctx, const double* d_s12, const double* d_s13,
                      const double* d_cosb, const double* d_gamma, int64_t n_data,
                      const double* d_mc_s12, const double* d_mc_s13, const double* d_mc_cosb,
                      const double* d_mc_gamma, int64_t n_mc, void* d_ws, size_t ws_bytes,
                      hipStream_t stream);

/* Precision of subsequent pwa_nll/pwa_grad/pwa_hvp/pwa_partials calls.
 * PWA_E_INVALID if that stream was not requested at pwa_create. */
int pwa_set_precision(pwa_ctx* ctx, int32_t precision);

/* NLL(theta) of eq. (3).  d_theta: P = 4K doubles; d_nll: 1 double. */
int pwa_nll(pwa_ctx* ctx, const double* d_theta, double* d_nll, hipStream_t stream);

/* NLL and its gradient (eq. (6) with NLL = -ln L) in one pass over the
 * events.  d_grad: P doubles. */
int pwa_grad(pwa_ctx* ctx, const double* d_theta, double* d_nll, double* d_grad,
             hipStream_t stream);

/* Hessian-vector product H v of the NLL (eq. (7) with NLL = -ln L, the
 * middle term summed over shards), with NLL and gradient from the same pass
 * (forward-over-reverse: one pass over the events, nothing stored per
 * event).  d_v, d_hv: P doubles; d_nll and d_grad may be null. */
int pwa_hvp(pwa_ctx* ctx, const double* d_theta, const double* d_v, double* d_hv,
            double* d_nll, double* d_grad, hipStream_t stream);

/* Hessian-vector product at the theta of the last pwa_hvp call (or
 * pwa_partials call with a direction) on this context, for a new direction
 * d_v (P doubles): Newton-CG evaluates many
 * products at one theta.  Of the per-resonance event moments that the
 * eq. (7) product is contracted from, only the three weighted by the
 * direction (the derivative of z along v) depend on v; this pass
 * accumulates those alone and reuses the theta-only totals of that call, so
 * it issues about 60 % of the per-event instructions of a full pass.
 * Results equal pwa_hvp at that theta up to rounding.  d_nll, d_grad (may
 * be null) receive the NLL and gradient at that theta.  Any other
 * evaluation on the context (pwa_nll, pwa_grad, pwa_partials, pwa_fit,
 * pwa_hessian, pwa_fit_fractions, pwa_fraction_matrix, pwa_bind) ends the
 * reuse: PWA_E_STATE until the next pwa_hvp (or pwa_partials with a
 * direction).  Uses the current
 * precision (a full pass if the cached totals are of the other one).
 * Errors: PWA_E_INVALID, PWA_E_STATE, PWA_E_HIP. */
int pwa_hvp_reuse(pwa_ctx* ctx, const double* d_v, double* d_hv, double* d_nll, double* d_grad,
                  hipStream_t stream);

/* Per-event intensity omega(x) = |sum_k c_k a_k(x)|^2 of eq. (1) at theta
 * for the bound data events (which = 0; n_data outputs) or MC events
 * (which = 1; n_mc outputs), in the event order given to pwa_bind, using the
 * event stream of the current precision and FP64 arithmetic.  d_out: device,
 * caller-owned, one double per event.  Used to draw events from the model by
 * accept-reject (toy data).  A mass at or below its threshold sets the device
 * status (pwa_device_status) and leaves the outputs unspecified.
 * Errors: PWA_E_INVALID, PWA_E_STATE (unbound), PWA_E_HIP. */
int pwa_intensity(pwa_ctx* ctx, const double* d_theta, int32_t which, double* d_out,
                  hipStream_t stream);

/* Un-combined per-shard sums of eq. (5) and their derivatives for the bound
 * events (one GPU's share in the paper's multi-GPU scheme, Sec. 2.3).
 * d_part receives 2*(2+4P) doubles: (hi, lo) double-double pairs of
 *   [F, G, dF/dtheta (P), dG/dtheta (P), H_F v (P), H_G v (P)]
 * with F = sum_data ln w, G = sum_MC w.  With d_v null the H v entries are
 * written as zero. */
int pwa_partials(pwa_ctx* ctx, const double* d_theta, const double* d_v, double* d_part,
                 hipStream_t stream);

/* pwa_partials with a new direction d_v at the theta of the last pwa_hvp or
 * pwa_partials-with-direction call on this context, by the direction-only
 * pass of pwa_hvp_reuse (same rules; PWA_E_STATE without such totals).  On
 * each rank of a sharded fit this gives the per-shard vector of the CG
 * products after the first at a Newton iterate. */
int pwa_partials_reuse(pwa_ctx* ctx, const double* d_v, double* d_part, hipStream_t stream);

/* Combine n_shards partial vectors (layout of pwa_partials, consecutive in
 * d_parts) with eq. (4), (6), (7): NLL, gradient and (if d_hv is non-null)
 * H v.  The shards are summed in index order in double-double arithmetic,
 * so the result does not depend on how events were split beyond rounding.
 * n_data_total, n_mc_total: event counts over all shards.  d_v is needed
 * when d_hv is non-null. */
int pwa_combine(int32_t n_par, int32_t n_shards, const double* d_parts,
                int64_t n_data_total, int64_t n_mc_total, const double* d_v,
                double* d_nll, double* d_grad, double* d_hv, hipStream_t stream);

/* Newton-CG fit options (host memory). */
typedef struct pwa_fit_opts {
  double xtol;            /* stop when mean |step| <= xtol (scipy's rule); a
                             Newton step within it ends the fit before its
                             line search (the NLL is flat to rounding there) */
  int32_t maxiter;        /* outer Newton iterations (<= 0: 200)              */
  int32_t cg_maxiter;     /* CG iterations per Newton step (<= 0: 20 P)        */
  double time_cap_s;      /* wall-clock cap, seconds (<= 0: none); Sec. 3 uses 500 */
  int32_t hvp_precision;  /* pwa_precision of the HVPs inside CG; with
                             PWA_PREC_F32, Newton steps whose CG forcing term
                             (see `forcing`) is below 1e-3 use FP64 HVPs
                             (FP32 ones cannot resolve that tolerance)      */
  int32_t free_mask_set;  /* 0: all parameters free; 1: use free_mask         */
  uint8_t free_mask[4 * PWA_MAX_RES]; /* 1 = free, 0 = fixed                   */
  int32_t forcing;        /* CG forcing term: 0 = scipy's eta = min(1/2,
                             sqrt(sum |g|)) (absolute: with many events it
                             stays 1/2 and Newton-CG converges linearly);
                             1 = relative eta = min(1/2, sqrt(sum |g| /
                             sum |g_0|)), superlinear (Eisenstat-Walker)   */
  int32_t precondition;   /* 0: plain CG (scipy's Newton-CG); 1: CG
                             preconditioned with the inverse of |H| (H from
                             HVPs along the free unit vectors at the first
                             iterate, eigenvalues floored at 1e-6 of the
                             largest), rebuilt when a solve needs more than
                             max(8, P/4) CG steps; those HVPs are counted
                             in n_hvp                                     */
  int32_t reconjugate;    /* 0: CG's three-term recurrence only; 1: each new
                             search direction is also made H-conjugate to
                             every earlier one of the same solve (Gram-Schmidt
                             with the stored H p_j: no extra HVPs), with the
                             exact line minimum -(r.p)/(p.Hp) as step.  The
                             recurrence loses conjugacy on an ill-conditioned
                             H, so that plain CG can take several times P
                             steps; with FP32 HVPs more so                */
} pwa_fit_opts;

/* Fit report (host memory, written by pwa_fit). */
typedef struct pwa_fit_report {
  double nll;             /* NLL at the returned theta                         */
  double grad_max;        /* max |gradient| over free parameters               */
  double seconds;         /* wall time of the fit                              */
  int32_t iterations;     /* Newton iterations                                  */
  int32_t n_nll;          /* NLL-only evaluations (line search)                */
  int32_t n_grad;         /* NLL+gradient evaluations                          */
  int32_t n_hvp;          /* Hessian-vector products                           */
  int32_t status;         /* pwa_status of the fit                             */
  int32_t converged;      /* 1 if the xtol test was met                        */
} pwa_fit_report;

/* Minimise the NLL from d_theta_inout with line-search Newton-CG (truncated
 * CG on H p = -g using pwa_hvp, strong-Wolfe line search on the FP64 NLL and
 * gradient) and write the best point back.  The paper fits with scipy's
 * Newton-CG (Sec. 3); the xtol test follows scipy's (mean absolute step).
 * Synchronous: returns when the fit ends.  h_rep may be null.
 * Errors: PWA_E_STATE (unbound), PWA_E_INVALID (options), PWA_E_DOMAIN (NLL
 * not finite at the start), PWA_E_NOCONV (maxiter/time cap/line-search
 * failure; theta holds the best point), PWA_E_HIP. */
int pwa_fit(pwa_ctx* ctx, double* d_theta_inout, const pwa_fit_opts* h_opts,
            pwa_fit_report* h_rep, hipStream_t stream);

/* Gradient-only comparator of pwa_fit: BFGS on the inverse Hessian (first
 * inverse scaled by y's / y'y after the first step; no Hessian-vector
 * products) with the same strong-Wolfe line search on the FP64 NLL and
 * gradient; it stops when the full quasi-Newton step p, or a line-search
 * step of at least p/2, is within the tolerance (mean |step| <= xtol).  The
 * paper
 * compares Newton-CG with gradient-only quasi-Newton minimisation (Migrad
 * with AD and with finite-difference gradients, Sec. 3); this is the
 * gradient-only arm.  Of h_opts it reads xtol, maxiter, time_cap_s and the
 * free mask (cg_maxiter, hvp_precision, forcing, precondition are ignored);
 * h_rep->iterations counts BFGS steps and n_hvp is 0.  Synchronous.  Errors
 * as pwa_fit. */
int pwa_fit_bfgs(pwa_ctx* ctx, double* d_theta_inout, const pwa_fit_opts* h_opts,
                 pwa_fit_report* h_rep, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * At a minimum: error matrix and fit fractions.  The paper quotes a fit
 * fraction per resonance (Table 1, column F_i) without defining it; here it
 * is the usual phase-space integral ratio, estimated with the bound MC
 * events (efficiency 1):
 *   F_k = sum_MC |c_k a_k|^2 / sum_MC |sum_l c_l a_l|^2,
 * so the F_k need not add up to 1 (interference).  Parameter errors are the
 * inverse Hessian of NLL = -ln L (eq. (3)).
 * ------------------------------------------------------------------------- */

/* Hessian d^2 NLL / dtheta^2 at theta: P forward-over-reverse passes (the
 * Hessian-vector product of eq. (7)) along the unit vectors, symmetrised as
 * (H + H^T)/2.  d_H: device, caller-owned, P*P doubles, row-major.  Uses the
 * event stream of the current precision; stream-ordered.
 * Errors: PWA_E_INVALID, PWA_E_STATE (unbound), PWA_E_HIP. */
int pwa_hessian(pwa_ctx* ctx, const double* d_theta, double* d_H, hipStream_t stream);

/* Fit fractions F_k (definition above; d_ff: K doubles) and, if d_dff is not
 * null, their gradients dF_k/dtheta (d_dff: K x P doubles, row-major), from
 * K + 1 gradient passes over the MC events only: one per resonance with the
 * other couplings set to zero (G_k = sum_MC |c_k a_k|^2 and its gradient)
 * and one with all of them (G).  Device buffers, caller-owned; uses the
 * current precision's stream; stream-ordered.  If G = 0 (all couplings zero)
 * the outputs are not finite.  Errors: PWA_E_INVALID, PWA_E_STATE, PWA_E_HIP. */
int pwa_fit_fractions(pwa_ctx* ctx, const double* d_theta, double* d_ff, double* d_dff,
                      hipStream_t stream);

/* Fraction matrix Phi (K x K, row-major, device, caller-owned): Phi[k][k] =
 * F_k as above, Phi[k][l] = I_kl = sum_MC 2 Re(conj(c_k a_k) c_l a_l) /
 * sum_MC |z|^2 for k < l (interference), 0 for k > l; all entries add up
 * to 1.  Computed from the MC Gram matrix sum_MC conj(a_k) a_l at theta's
 * masses and widths (FP64 matrix cores, FP64 event stream, K <= 24).
 * d_ws: caller-owned device scratch of pwa_fraction_matrix_workspace_bytes()
 * bytes, 256-byte aligned.  Errors: PWA_E_INVALID (K > 24, no FP64 stream,
 * null), PWA_E_STATE, PWA_E_WORKSPACE, PWA_E_HIP. */
size_t pwa_fraction_matrix_workspace_bytes(const pwa_ctx* ctx);
int pwa_fraction_matrix(pwa_ctx* ctx, const double* d_theta, void* d_ws, size_t ws_bytes,
                        double* d_phi, hipStream_t stream);

/* Covariance matrix of the free parameters (host arrays, P x P row-major):
 * the inverse of H restricted to the rows and columns i with h_free[i] != 0
 * (all of them if h_free is null), by a Cholesky factorisation of that
 * block; rows and columns of fixed parameters are zero.  The NLL does not
 * change when every coupling is multiplied by one complex number, so with
 * all parameters free H is singular: fix one coupling (its real and
 * imaginary parts).  Errors: PWA_E_INVALID (sizes, null, non-finite H),
 * PWA_E_DOMAIN (the free block is not positive definite, or numerically
 * singular: a Cholesky pivot at or below 1e-12 n H_jj, n the number of free
 * parameters, is a direction the Hessian does not resolve above rounding). */
int pwa_covariance(int32_t P, const double* h_H, const uint8_t* h_free, double* h_cov);

/* Linear error propagation (host arrays): sigma_r = sqrt(J_r C J_r^T) for the
 * n rows of J (n x P, row-major), e.g. the fit-fraction gradients, with the
 * covariance C (P x P).  A negative quadratic form gives NaN.
 * Errors: PWA_E_INVALID. */
int pwa_propagate(int32_t P, int32_t n, const double* h_J, const double* h_cov, double* h_sigma);

/* Reads and clears the context's sticky device status word (synchronises
 * the stream).  Bits: 1 = a resonance mass at or below threshold was seen,
 * 2 = a non-finite NLL was produced.  Negative on error. */
int pwa_device_status(pwa_ctx* ctx, hipStream_t stream);

/* Static description of a status code. */
const char* pwa_status_str(int status);

/* Number of parameters P = 4K of a context (or -1 for null). */
int32_t pwa_n_par(const pwa_ctx* ctx);

/* Number of per-event planes of the context's parameter-free event stream
 * (Sec. 2.2: the precomputed per-event factors), or -1 for null.  Each pass
 * reads every plane once per event: 8 bytes per plane and event on the FP64
 * stream, 4 on the FP32 one.  Fixed by the model at pwa_create. */
int32_t pwa_stream_fields(const pwa_ctx* ctx);

/* Launch shape of the NLL/gradient/HVP pass kernels (for tuning; the
 * default is an automatic choice by K).  layout 1: `groups` lanes of one
 * wavefront cooperate on each event; layout 2: `groups` wavefronts of one
 * block cooperate on each batch of 64 events; layout 3: the same for models
 * with a Flatte resonance or a spin-1 parent (the only layout those use;
 * groups in {1, 2, 4, 8} with res_per_group 2, or 4 groups of 3, so
 * K <= 16 there).  Each lane
 * owns `res_per_group` resonances; groups * res_per_group >= K.  layout 0
 * restores the automatic choice.  PWA_E_INVALID for a shape that is not
 * built or does not fit the model. */
int pwa_set_launch_shape(pwa_ctx* ctx, int32_t layout, int32_t groups, int32_t res_per_group);

/* Number of thread blocks the NLL/gradient/HVP kernels launch (after
 * pwa_bind), or -1. */
int32_t pwa_grid_blocks(const pwa_ctx* ctx);

/* Kernel timing for measurement: while enabled (enable != 0), every
 * evaluation records a pair of HIP events on the caller's stream around its
 * per-event pass kernel (the dominant kernel; not the table or finaliser
 * launches).  pwa_kernel_time synchronises on the last recorded event,
 * returns the summed duration (ms) and the number of timed launches since
 * the previous call, and resets them.  Events are created by the library on
 * first use (no device memory is allocated).  Errors: PWA_E_INVALID,
 * PWA_E_HIP. */
int pwa_set_kernel_timing(pwa_ctx* ctx, int32_t enable);
int pwa_kernel_time(pwa_ctx* ctx, double* total_ms, int64_t* n_launches);

/* ---------------------------------------------------------------------------
 * Fixed-lineshape batched path.  With the masses and widths frozen, the
 * amplitudes a_k(x) of eq. (1) are fixed and the couplings enter linearly:
 * for a batch of coupling vectors c_b the data term is
 * F_b = sum_data ln |sum_k c_kb a_k(x)|^2 (a complex matrix product of the
 * N_D x K amplitude matrix with the K x B coupling block, then a log), and the
 * normalisation is G_b = c_b^H Gm c_b with the K x K Gram matrix
 * Gm = sum_MC conj(a_k) a_l.  NLL_b = -F_b + N_D ln(G_b / N_MC) (eq. (3)).
 * ------------------------------------------------------------------------- */
/* Operand formats.  A rounding of a coupling shifts every event's log the
 * same way (the NLL error grows like N_D times the gradient in c), while a
 * rounding of an amplitude is independent from event to event (its error
 * grows like sqrt(N_D)).  BF16 and FP16 round both operands once and are the
 * fast, low-precision formats.
 *
 * The sliced FP16 format runs on the FP16 matrix cores with fixed-point
 * operands.  Each event's amplitude row is scaled by a power of two, 2^(9-E)
 * with |largest component| < 2^E, and cut into four integer slices
 * x = 2^(E-9) (q0 + 2^-9 q1 + 2^-18 q2 + 2^-27 q3) + r with |q0| <= 512,
 * |q1..q3| <= 256 and |r| <= 2^(E-37); each start's couplings are cut the
 * same way with the exponent of its largest real or imaginary component.
 * Z = sum over slice pairs (i, j) with i + j <= 3 of 2^(-9 (i + j)) q^A_i . q^C_j
 * (ten products) times the two powers of two.  Every slice product is an
 * integer, so the leading dot product (at most 48 terms below 2^18) is formed
 * exactly in FP32 and the next two levels are too; the levels are combined in
 * FP64 and the logs are FP64.  Representation error: 2^-28 of the row's
 * largest amplitude (random over events) and 2^-37 of the start's largest
 * coupling (the same for every event). */
typedef enum pwa_operand {
  PWA_OP_F64 = 0,   /* FP64 operands, FP64 matrix-core accumulation          */
  PWA_OP_F32 = 1,   /* FP32 amplitudes; couplings as FP32 hi + lo (two
                       products); FP32 accumulation                          */
  PWA_OP_BF16 = 2,  /* BF16 operands, FP32 accumulation                      */
  PWA_OP_F16 = 3,   /* FP16 operands, FP32 accumulation                      */
  PWA_OP_F16S = 4   /* sliced FP16 (above): four 9-bit fixed-point slices of
                       each operand, ten exact integer products              */
} pwa_operand;

/* Device workspace (bytes) of the batched path for n_data data events,
 * operand format `operand` and up to max_batch coupling vectors per call.
 * 0 on invalid arguments (K > 24 is not supported on this path). */
size_t pwa_batched_workspace_bytes(const pwa_ctx* ctx, int64_t n_data, int32_t operand,
                                   int32_t max_batch);

/* Freeze M and Gamma at d_theta (P doubles; the couplings in it are ignored):
 * builds the data amplitude matrix in the operand format and the FP64 Gram
 * matrix of the MC amplitudes (matrix cores, FP64) in d_bws, a caller-owned
 * 256-byte aligned device buffer of bws_bytes >= pwa_batched_workspace_bytes.
 * Needs a bound context with the FP64 event stream.
 * Errors: PWA_E_STATE, PWA_E_INVALID, PWA_E_WORKSPACE, PWA_E_HIP. */
int pwa_freeze(pwa_ctx* ctx, const double* d_theta, int32_t operand, int32_t max_batch,
               void* d_bws, size_t bws_bytes, hipStream_t stream);

/* NLL of B coupling vectors at the frozen masses and widths.  d_C: K x B
 * complex couplings as (re, im) FP64 pairs, start-major: coupling k of
 * start b at d_C[2 (b K + k)], d_C[2 (b K + k) + 1].  d_nll: B doubles
 * (+inf where G_b <= 0).  B <= max_batch of pwa_freeze. */
int pwa_nll_batched(pwa_ctx* ctx, const double* d_C, int32_t B, double* d_nll,
                    hipStream_t stream);

/* Copy the frozen Gram matrix Gm[k][l] = sum_MC conj(a_k) a_l (K x K complex,
 * (re, im) pairs, row-major) to d_gram (2 K^2 doubles). */
int pwa_gram(pwa_ctx* ctx, double* d_gram, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* PWA_H */
