// Internal declarations shared by the kernel and host translation units of
// the PWA likelihood library.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pwa.h"

namespace pwa {

// ---------------------------------------------------------------- table --
// Per-resonance constants built on the device from (theta, v) before every
// evaluation.  Factorised Breit-Wigner: with the per-event stream values
//   s (pair mass^2), u = F_J(z) P_J(cos), g = q^(2J+1) F_J(z)^2 / sqrt(s)
// and the per-resonance functions of M only
//   eta(M) = M^2 / (q0^(2J+1) F_J(z0)^2),  beta(M) = 1/F_J(z0),
// one has M Gamma(s) = Gamma eta g, and the amplitude is
//   a = beta u w,  w = 1/D,  D = (M^2 - s) - i Gamma eta g.
// The first slots are read per event by the pass kernels; the rest only by
// the finaliser, which contracts the event moments with them.
enum TableSlot : int {
  TB_M2 = 0,      // M^2
  TB_NGE = 1,     // -Gamma eta           (Im D = TB_NGE * g)
  TB_UMUL = 2,    // u = u_plane * UMUL + UADD (J = 0: u = 1)
  TB_UADD = 3,
  TB_CBR = 4,     // c beta               (z = sum c beta u w)
  TB_CBI = 5,
  TB_K1R = 6,     // zdot = sum K1 u w + K2 u w^2 + K3 u g w^2
  TB_K1I = 7,
  TB_K2R = 8,
  TB_K2I = 9,
  TB_K3R = 10,
  TB_K3I = 11,
  TB_HOT = 12,    // slots read by the pass kernels
  TB_BETA = 12,   // beta, beta'
  TB_BETA1 = 13,
  TB_BDOT = 14,   // v_M beta', v_M beta''
  TB_BDOT1 = 15,
  TB_CR = 16,     // c
  TB_CI = 17,
  TB_VR = 18,     // v on Re c, Im c, M
  TB_VI = 19,
  TB_VM = 20,
  TB_2M = 21,     // dD/dM = (2M, NGE1 g)
  TB_NGE1 = 22,
  TB_NETA = 23,   // dD/dGamma = (0, NETA g), NETA = -eta
  TB_DDR = 24,    // directional derivative of D along v: (DDR, DDIG g)
  TB_DDIG = 25,
  TB_DMDDIG = 26, // its M-derivative: (2 v_M, DMDDIG g)
  TB_DGDDIG = 27, // its Gamma-derivative: (0, DGDDIG g)
  TB_USED = 28
};
// Event moments accumulated per resonance (complex, re/im interleaved):
//   C1..C3 = sum gamma u {w, w^2, g w^2}           (gradient and HVP)
//   B1..B3 = sum alpha u {w, w^2, g w^2}           (HVP)
//   C4..C6 = sum gamma u {w^3, g w^3, g^2 w^3}     (HVP)
constexpr int NMOM_GRAD = 6;
constexpr int NMOM_HVP = 18;
constexpr int TS = 32;        // table stride (reals) per resonance
// Int table per resonance: plane indices of s, u, g, the spin J, and for the
// general physics path the imaginary width factor h (Flatte) and the complex
// angular factors of the parent's helicity amplitudes (u is the real part of
// mu = 0; the rest are the zero plane where a model has no such factor).
enum ITableSlot : int { IT_S = 0, IT_U = 1, IT_G = 2, IT_J = 3, IT_H = 4, IT_UI = 5, IT_U1R = 6, IT_U1I = 7 };
constexpr int ITS = 8;
constexpr int KPAD = 64;      // table rows (resonance slots incl. padding)
constexpr int BLOCK = 256;    // threads per block of the evaluation kernels
constexpr int MAX_BLOCKS = 4096;

// Evaluation modes.
// MODE_HVPB: a Hessian-vector product at the theta of the previous full
// HVP pass; the pass accumulates the direction moments B1..B3 only and the
// finaliser reuses that pass's theta-only totals (S, C1..C6).
enum Mode : int { MODE_NLL = 0, MODE_GRAD = 1, MODE_HVP = 2, MODE_HVPB = 3 };

// Output kinds of the finaliser.
enum OutKind : int { OUT_COMBINED = 0, OUT_PARTIALS = 1 };

// Physical constants of the model, passed by value to kernels.
struct ModelDev {
  double M2;                 // parent mass^2
  double msq[3];             // daughter masses^2
  double m[3];
  double r2;                 // Blatt-Weisskopf radius^2
  int K;
  int width_mode;
  int parent_spin;           // 0, or 1 (helicity amplitudes mu = +1, -1)
  int gen;                   // 1: general physics path (Flatte or spin-1 parent)
  double fl_msq[2];          // Flatte second channel: masses^2
  double fl_ratio;           //   and coupling ratio g_2 / g_1
  int ch[PWA_MAX_RES];
  int spin[PWA_MAX_RES];
  int lineshape[PWA_MAX_RES];
  int fidx[PWA_MAX_RES][ITS];  // int table row of each resonance (ITableSlot)
};

// Which planes the event stream holds.
struct FieldSpec {
  int s_field[3];            // -1: channel unused
  int u_field[3][3];         // [channel][J], -1: absent (always -1 for J = 0)
  int g_field[3][3];
  int fg_field[3];           // Flatte width factor per channel: real part
  int fh_field[3];           //   and imaginary part
  int uc_field[3][3][4];     // spin-1 parent: u^mu per (channel, J): re, im of mu = +1, -1
  int zero_field;            // a plane of zeros (general path), -1: none
  int n_fields;
};

constexpr int MAX_FIELDS = 18;   // 3 s + 6 u + 9 g planes at most
// general path: 3 s + 6 Flatte (g, h) + 9 g + 36 spin-1 u^mu (re, im of
// mu = +1, -1 per (channel, J)) + 1 zero plane at most
constexpr int MAX_GEN_FIELDS = 55;

// Stream staging geometry (wave-group layout): one 16-byte load per lane
// brings 64 events of stage_ppi planes; the LDS stage buffers hold the
// planes rounded up to whole groups of them.
__host__ __device__ constexpr int stage_ppi(int bytes) { return 16 / bytes; }
__host__ __device__ constexpr int stage_planes(int n_fields, int bytes) {
  return (n_fields + stage_ppi(bytes) - 1) / stage_ppi(bytes) * stage_ppi(bytes);
}

struct EvalArgs {
  const void* planes;        // n_fields planes of `stride` reals
  int64_t stride;            // a multiple of 64
  int n_fields;
  const double* tbl64;
  const float* tbl32;
  const int* itbl;
  int64_t n_data, n_mc;      // data events [0, n_data), MC [mc_base, mc_base + n_mc)
  int64_t mc_base;           // n_data rounded up to 64
  int gen;                   // general physics path (wgx_kernel)
  int nmu;                   // helicity amplitudes per event (1 or 2)
  int nb_data, nb_mc;
  int K;
  double* part;              // per-block (hi, lo) partial sums
};

struct FinalArgs {
  const double* part;
  double* tot;               // reduced totals: 2 V (hi, lo) pairs
  const double* tbl;         // resonance table (finaliser slots)
  int nb_data, nb_mc;
  int V;                     // values per block: 1 + NMOM * K
  int K, mode, out_kind;
  double n_data, n_mc;
  const double* v;           // direction (HVP), may be null
  double* nll;
  double* grad;
  double* hv;
  double* dd_out;            // partials output (out_kind == OUT_PARTIALS)
  int* status;               // [0] this evaluation, [1] sticky
};

// Launchers (pwa_kernels.hip).  All return hipError_t of the launch.
hipError_t launch_precompute(const double* s12, const double* s13, const double* cosb,
                             const double* gam, int64_t n, int64_t offset, void* planes,
                             int64_t stride, int is_f32, const ModelDev& md, const FieldSpec& fs,
                             hipStream_t st);
hipError_t launch_intensity(bool f32, const void* planes, int64_t stride, int64_t base, int64_t n,
                            const double* tbl, const int* itbl, int K, int gen, int nmu,
                            double* out, hipStream_t st);
hipError_t launch_table(const double* theta, const double* v, const ModelDev& md, int kslots,
                        double* tbl64, float* tbl32, int* itbl, int* status, hipStream_t st);
// layout 1: T lanes of one wave share an event; layout 2: T waves of one
// block share each batch of 64 events.  R resonances per lane.
hipError_t launch_eval(int is_f32, int mode, int layout, int T, int R, const EvalArgs& a,
                       int nblocks, hipStream_t st);
hipError_t launch_final(const FinalArgs& f, hipStream_t st);
hipError_t launch_combine(int n_par, int n_shards, const double* parts, double n_data,
                          double n_mc, const double* v, double* nll, double* grad, double* hv,
                          int* status, hipStream_t st);
// Maximum resident blocks per CU of an evaluation kernel variant.
int eval_occupancy(int is_f32, int mode, int layout, int T, int R, int n_fields);
// Is (T, R) an instantiated launch shape of layout 1 / layout 2?
bool shape_built(int T, int R);
bool wg_shape_built(int G, int R);
bool gen_shape_built(int G, int R);
bool nll_shape_built(int R);

}  // namespace pwa
