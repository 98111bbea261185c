// HIP kernels of the PWA likelihood library (gfx950 / CDNA4).
//
// What the kernels compute (arXiv:2403.09225):
//   intensity  w = |z|^2, z = sum_k c_k a_k               Sec. 2.2, eq. (1)
//   per-shard  F = sum_data ln w, G = sum_MC w              Sec. 2.3, eq. (5)
//   NLL = -F + N_D ln(G / N_MC)                             eq. (3)/(4), NLL = -ln L
//   gradient and Hessian-vector product combine             eq. (6)/(7)
// The parameter-free part of every amplitude is precomputed once per event
// (Sec. 2.2: "pre-computed and stored on the GPU") into a structure-of-arrays
// stream; each evaluation then makes one pass over that stream.
//
// Kernel structure (one evaluation = 3 launches on the caller's stream):
//   1. table_kernel: per-resonance constants from (theta, v), including the
//      first and second M-derivatives of the mass-only factors, by
//      second-order Taylor arithmetic in one thread per resonance.
//   2. eval_kernel / nll_kernel: one pass over the events.  A team of T lanes
//      shares an event; each lane owns R resonances and keeps their gradient
//      and HVP sums in FP64 registers over all the events it visits.  Event
//      sums are reduced per wave with a double-double butterfly and per block
//      in a fixed order into per-block (hi, lo) partials: no atomics, so the
//      result is bitwise reproducible for a given grid.
//   3. final_kernel: fixed-order double-double sum of the block partials and
//      the eq. (4)/(6)/(7) combine (or the raw eq. (5) partials).

#include <math.h>

#include "pwa_internal.h"

namespace pwa {

typedef __attribute__((address_space(4))) const double c_double;
typedef __attribute__((address_space(4))) const float c_float;
typedef __attribute__((address_space(4))) const int c_int;

template <typename Real> struct CPtr;
template <> struct CPtr<double> { typedef c_double type; };
template <> struct CPtr<float> { typedef c_float type; };

// Re-materialise a wave-uniform constant pointer every loop trip: keeps the
// per-resonance table in scalar loads (SGPR operands) instead of letting the
// compiler hoist hundreds of table values into vector registers.
template <typename P>
__device__ __forceinline__ P* opaque_s(P* p) {
  asm volatile("" : "+s"(p));
  return p;
}
__device__ __forceinline__ int opaque_v(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Reciprocal: hardware estimate refined by two Newton steps (FP64), or the
// single-precision hardware reciprocal (FP32 path).
__device__ __forceinline__ double rcp_r(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float rcp_r(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double log_r(double x) { return log(x); }
__device__ __forceinline__ float log_r(float x) { return __logf(x); }

// Double-double accumulation (TwoSum then renormalise).  Symmetric in its
// operands, so a butterfly leaves identical values in both lanes.
__device__ __forceinline__ void dd_add(double& hi, double& lo, double bhi, double blo) {
  const double s = hi + bhi;
  const double bb = s - hi;
  double e = (hi - (s - bb)) + (bhi - bb);
  e += lo + blo;
  hi = s + e;
  lo = e - (hi - s);
}

__device__ __forceinline__ void dd_wave_reduce(double& hi, double& lo, int first_offset) {
  for (int off = first_offset; off < 64; off <<= 1) {
    const double oh = __shfl_xor(hi, off);
    const double ol = __shfl_xor(lo, off);
    dd_add(hi, lo, oh, ol);
  }
}

__device__ __forceinline__ double kallen(double x, double y, double z) {
  return x * x + y * y + z * z - 2.0 * (x * y + x * z + y * z);
}

// ------------------------------------------------------------------------
// 1. Parameter-free event stream.
// For each channel in use: s of the pair; for each (channel, J) in use:
// g = q^(2J+1) F_J(z)^2 / sqrt(s) (1 for constant width) and, for J >= 1,
// u = F_J(z) P_J(cos th).  Computed in FP64, stored as Real.
// ------------------------------------------------------------------------
template <typename Real>
__global__ __launch_bounds__(256) void precompute_kernel(const double* __restrict__ s12,
                                                         const double* __restrict__ s13,
                                                         int64_t n, int64_t offset,
                                                         Real* __restrict__ planes,
                                                         int64_t stride, ModelDev md,
                                                         FieldSpec fs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x12 = s12[i], x13 = s13[i];
  const double x23 = md.M2 + md.msq[0] + md.msq[1] + md.msq[2] - x12 - x13;
  const int64_t o = offset + i;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (fs.s_field[c] < 0) continue;
    // channel c = (a b) with bachelor cc; s_ab and s_ac
    const int a = (c == 2) ? 1 : 0;
    const int b = (c == 0) ? 1 : 2;
    const int cc = (c == 0) ? 2 : (c == 1 ? 1 : 0);
    const double sab = (c == 0) ? x12 : (c == 1 ? x13 : x23);
    const double sac = (c == 0) ? x13 : x12;
    const double ma2 = md.msq[a], mb2 = md.msq[b], mc2 = md.msq[cc];
    const double rs = sqrt(sab);
    const double h = 0.5 / rs;
    const double q = sqrt(fmax(kallen(sab, ma2, mb2), 0.0)) * h;
    const double p = sqrt(fmax(kallen(md.M2, sab, mc2), 0.0)) * h;
    const double ea = (sab + ma2 - mb2) * h;
    const double ec = (md.M2 - sab - mc2) * h;
    const double cs = (sac - ma2 - mc2 - 2.0 * ea * ec) / (2.0 * q * p);
    const double z = q * q * md.r2;
    planes[fs.s_field[c] * stride + o] = (Real)sab;
#pragma unroll
    for (int J = 0; J < 3; ++J) {
      const int gf = fs.g_field[c][J];
      if (gf < 0) continue;
      const double F2 = (J == 0) ? 1.0 : (J == 1 ? 1.0 / (1.0 + z) : 1.0 / (z * z + 3.0 * z + 9.0));
      const double q2 = q * q;
      const double qp = (J == 0) ? q : (J == 1 ? q * q2 : q * q2 * q2);   // q^(2J+1)
      const double g = (md.width_mode == PWA_WIDTH_MASS_DEPENDENT) ? qp * F2 / rs : 1.0;
      planes[gf * stride + o] = (Real)g;
      if (J >= 1) {
        const double PJ = (J == 1) ? cs : 1.5 * cs * cs - 0.5;
        planes[fs.u_field[c][J] * stride + o] = (Real)(sqrt(F2) * PJ);
      }
    }
  }
}

// ------------------------------------------------------------------------
// 2. Resonance table.  Second-order Taylor arithmetic in M gives the mass-only
// factors eta, beta and their first two M-derivatives exactly (to rounding).
// ------------------------------------------------------------------------
struct Jet {
  double v, d, dd;  // f, f', f'' with respect to M
};
__device__ __forceinline__ Jet jmul(Jet a, Jet b) {
  return {a.v * b.v, a.v * b.d + a.d * b.v, a.v * b.dd + 2.0 * a.d * b.d + a.dd * b.v};
}
__device__ __forceinline__ Jet jaddc(Jet a, double c) { return {a.v + c, a.d, a.dd}; }
__device__ __forceinline__ Jet jscale(Jet a, double c) { return {a.v * c, a.d * c, a.dd * c}; }
__device__ __forceinline__ Jet jadd(Jet a, Jet b) { return {a.v + b.v, a.d + b.d, a.dd + b.dd}; }
__device__ __forceinline__ Jet jrcp(Jet a) {
  const double r = 1.0 / a.v;
  return {r, -a.d * r * r, (2.0 * a.d * a.d * r - a.dd) * r * r};
}
__device__ __forceinline__ Jet jsqrt(Jet a) {
  const double s = sqrt(a.v);
  return {s, a.d / (2.0 * s), a.dd / (2.0 * s) - a.d * a.d / (4.0 * s * s * s)};
}

__global__ __launch_bounds__(64) void table_kernel(const double* __restrict__ theta,
                                                   const double* __restrict__ v, ModelDev md,
                                                   int kslots, double* __restrict__ tbl64,
                                                   float* __restrict__ tbl32,
                                                   int* __restrict__ itbl, int* status) {
  __shared__ int bad;
  const int k = threadIdx.x;
  if (k == 0) bad = 0;
  __syncthreads();
  if (k < kslots) {
    double e[TS];
    int f[ITS];
#pragma unroll
    for (int j = 0; j < TS; ++j) e[j] = 0.0;
    if (k < md.K) {
      const double cr = theta[4 * k], ci = theta[4 * k + 1];
      const double M = theta[4 * k + 2], G = theta[4 * k + 3];
      double vr = 0, vi = 0, vM = 0, vG = 0;
      if (v) {
        vr = v[4 * k];
        vi = v[4 * k + 1];
        vM = v[4 * k + 2];
        vG = v[4 * k + 3];
      }
      const int c = md.ch[k], J = md.spin[k];
      const int a = (c == 2) ? 1 : 0, b = (c == 0) ? 1 : 2;
      const double sig = (md.m[a] + md.m[b]) * (md.m[a] + md.m[b]);
      const double del = (md.m[a] - md.m[b]) * (md.m[a] - md.m[b]);
      const Jet Mj = {M, 1.0, 0.0};
      const Jet M2 = jmul(Mj, Mj);
      // q0^2 = (M^2 - (ma+mb)^2)(M^2 - (ma-mb)^2) / (4 M^2)
      Jet Q = jmul(jmul(jaddc(M2, -sig), jaddc(M2, -del)), jrcp(jscale(M2, 4.0)));
      if (!(Q.v > 0.0) || !(M > 0.0) || !isfinite(Q.v)) {
        atomicOr(&bad, 1);
        Q = {1.0, 0.0, 0.0};
      }
      const Jet z0 = jscale(Q, md.r2);
      Jet Finv2 = {1.0, 0.0, 0.0};  // 1 / F_J(z0)^2
      if (J == 1) Finv2 = jaddc(z0, 1.0);
      if (J == 2) Finv2 = jaddc(jadd(jmul(z0, z0), jscale(z0, 3.0)), 9.0);
      const Jet beta = (J == 0) ? Jet{1.0, 0.0, 0.0} : jsqrt(Finv2);
      Jet eta;
      if (md.width_mode == PWA_WIDTH_MASS_DEPENDENT) {
        Jet qp = jsqrt(Q);  // q0^(2J+1)
        for (int j = 0; j < J; ++j) qp = jmul(qp, Q);
        eta = jmul(jmul(M2, Finv2), jrcp(qp));
      } else {
        eta = Mj;
      }
      e[TB_M2] = M * M;
      e[TB_NGE] = -G * eta.v;
      e[TB_BETA] = beta.v;
      e[TB_CR] = cr;
      e[TB_CI] = ci;
      e[TB_UMUL] = (J == 0) ? 0.0 : 1.0;
      e[TB_UADD] = (J == 0) ? 1.0 : 0.0;
      e[TB_DDR] = 2.0 * M * vM;
      e[TB_DDIG] = -(vM * G * eta.d + vG * eta.v);
      e[TB_BDOT] = vM * beta.d;
      e[TB_VR] = vr;
      e[TB_VI] = vi;
      e[TB_2M] = 2.0 * M;
      e[TB_NGE1] = -G * eta.d;
      e[TB_NETA] = -eta.v;
      e[TB_BETA1] = beta.d;
      e[TB_DMDDR] = 2.0 * vM;
      e[TB_DMDDIG] = -(vM * G * eta.dd + vG * eta.d);
      e[TB_DGDDIG] = -vM * eta.d;
      e[TB_BDOT1] = vM * beta.dd;
      f[0] = md.fidx[k][0];
      f[1] = md.fidx[k][1];
      f[2] = md.fidx[k][2];
      f[3] = J;
    } else {
      // inert padding slot: a = 0 and every derivative 0, D = -1 - s != 0
      e[TB_M2] = -1.0;
      e[TB_UADD] = 1.0;
      f[0] = f[1] = f[2] = f[3] = 0;
    }
#pragma unroll
    for (int j = 0; j < TS; ++j) {
      tbl64[k * TS + j] = e[j];
      tbl32[k * TS + j] = (float)e[j];
    }
#pragma unroll
    for (int j = 0; j < ITS; ++j) itbl[k * ITS + j] = f[j];
  }
  __syncthreads();
  if (k == 0) {
    status[0] = bad;
    if (bad) atomicOr(&status[1], 1);
  }
}

// ------------------------------------------------------------------------
// Block-range helper: blocks [0, nb_data) take data events, the rest MC.
// ------------------------------------------------------------------------
struct Range {
  bool is_data;
  int64_t base, begin, end;
};
__device__ __forceinline__ Range block_range(const EvalArgs& a) {
  Range rg;
  rg.is_data = (int)blockIdx.x < a.nb_data;
  const int64_t n_set = rg.is_data ? a.n_data : a.n_mc;
  const int nb_set = rg.is_data ? a.nb_data : a.nb_mc;
  const int bi = rg.is_data ? (int)blockIdx.x : (int)blockIdx.x - a.nb_data;
  rg.base = rg.is_data ? 0 : a.n_data;
  const int64_t chunk = (n_set + nb_set - 1) / nb_set;
  rg.begin = min(n_set, (int64_t)bi * chunk);
  rg.end = min(n_set, rg.begin + chunk);
  return rg;
}

// ------------------------------------------------------------------------
// NLL-only pass: one lane per event, runtime resonance loop, table in SGPRs.
// ------------------------------------------------------------------------
template <typename Real>
__global__ __launch_bounds__(BLOCK) void nll_kernel(EvalArgs a) {
  typedef typename CPtr<Real>::type CReal;
  const Range rg = block_range(a);
  const Real* __restrict__ planes = (const Real*)a.planes;
  const int64_t stride = a.stride;
  const Real* tsrc = (sizeof(Real) == 8) ? (const Real*)a.tbl64 : (const Real*)a.tbl32;
  double acc = 0.0;
  for (int64_t e0 = rg.begin; e0 < rg.end; e0 += BLOCK) {
    const int64_t e = e0 + threadIdx.x;
    const bool valid = e < rg.end;
    const int64_t ev = rg.base + (valid ? e : rg.begin);
    CReal* tb = opaque_s((CReal*)tsrc);
    c_int* it = opaque_s((c_int*)a.itbl);
    Real zr = 0, zi = 0;
    for (int k = 0; k < a.K; ++k) {
      CReal* t = tb + k * TS;
      const Real s = planes[it[k * ITS + 0] * stride + ev];
      const Real u = planes[it[k * ITS + 1] * stride + ev] * t[TB_UMUL] + t[TB_UADD];
      const Real g = planes[it[k * ITS + 2] * stride + ev];
      const Real Dr = t[TB_M2] - s;
      const Real Di = t[TB_NGE] * g;
      const Real inv = rcp_r(Dr * Dr + Di * Di);
      const Real bu = t[TB_BETA] * u * inv;
      const Real ar = bu * Dr, ai = -bu * Di;
      zr += t[TB_CR] * ar - t[TB_CI] * ai;
      zi += t[TB_CR] * ai + t[TB_CI] * ar;
    }
    const Real om = zr * zr + zi * zi;
    const double term = rg.is_data ? (double)log_r(om) : (double)om;
    acc += valid ? term : 0.0;
  }
  double hi = acc, lo = 0.0;
  dd_wave_reduce(hi, lo, 1);
  __shared__ double red[BLOCK / 64][2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[wave][0] = hi;
    red[wave][1] = lo;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double h = red[0][0], l = red[0][1];
    for (int w = 1; w < BLOCK / 64; ++w) dd_add(h, l, red[w][0], red[w][1]);
    a.part[blockIdx.x * 2 + 0] = h;
    a.part[blockIdx.x * 2 + 1] = l;
  }
}

// ------------------------------------------------------------------------
// Gradient / HVP pass.
//
// Per event, with w = 1/D, w2 = w^2 and the directional derivative
// Ddot = v_M dD/dM + v_Gamma dD/dGamma:
//   a     = beta u w,            adot = u (beta' v_M w + beta wdot),  wdot = -Ddot w2
//   da/dM = u (beta' w + beta wM),  wM = -(dD/dM) w2
//   da/dG = beta u wG,              wG = -(dD/dGamma) w2
//   z = sum c a,  zdot = sum (cdot a + c adot)           (zdot = dz along v)
// The gradient of w = |z|^2 along theta_p is 2 Re(conj(z) dz/dtheta_p) and its
// Hessian times v is 2 Re(conj(zdot) dz/dtheta_p + conj(z) dzdot/dtheta_p).
// For ln w (data) and w (MC) both are 2 Re(alpha dz/dtheta_p + gamma
// dzdot/dtheta_p) with per-event weights
//   data: gamma = conj(z)/w, alpha = (conj(zdot) - (wdot/w) conj(z))/w
//   MC:   gamma = conj(z),   alpha = conj(zdot)
// (the gradient uses gamma only).  The factor 2 is applied by the finaliser.
// ------------------------------------------------------------------------
template <typename Real, int MODE, int T, int R>
__global__ __launch_bounds__(BLOCK) void eval_kernel(EvalArgs a) {
  static_assert(64 % T == 0, "team size must divide the wavefront");
  typedef typename CPtr<Real>::type CReal;
  constexpr int TEAMS = BLOCK / T;
  constexpr int NG = 4 * R;
  constexpr int NH = (MODE == MODE_HVP) ? 4 * R : 0;
  constexpr int NA = NG + NH;
  constexpr int NV = 1 + NA;
  constexpr int NSLOT = T * R;
  constexpr int NWAVE = BLOCK / 64;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int team = tid / T;
  const int pos = tid % T;
  const Range rg = block_range(a);
  const Real* __restrict__ planes = (const Real*)a.planes;
  const int64_t stride = a.stride;
  const Real* tsrc = (sizeof(Real) == 8) ? (const Real*)a.tbl64 : (const Real*)a.tbl32;

  __shared__ Real s_tb[(T > 1) ? NSLOT * TS : 1];
  __shared__ int s_it[(T > 1) ? NSLOT * ITS : 1];
  if constexpr (T > 1) {
    for (int i = tid; i < NSLOT * TS; i += BLOCK) s_tb[i] = tsrc[i];
    for (int i = tid; i < NSLOT * ITS; i += BLOCK) s_it[i] = a.itbl[i];
    __syncthreads();
  }

  double accS = 0.0;
  double acc[NA];
#pragma unroll
  for (int j = 0; j < NA; ++j) acc[j] = 0.0;

  for (int64_t e0 = rg.begin; e0 < rg.end; e0 += TEAMS) {
    const int64_t e = e0 + team;
    const bool valid = e < rg.end;
    const int64_t ev = rg.base + (valid ? e : rg.begin);

    // Table access: scalar loads for T == 1, LDS rows of this lane otherwise.
    CReal* tb = opaque_s((CReal*)tsrc);
    c_int* it = opaque_s((c_int*)a.itbl);
    const int row0 = (T > 1) ? opaque_v(pos * R) : 0;
    auto TB = [&](int r, int slot) -> Real {
      if constexpr (T == 1) return tb[r * TS + slot];
      else return s_tb[(row0 + r) * TS + slot];
    };
    auto IT = [&](int r, int j) -> int {
      if constexpr (T == 1) return it[r * ITS + j];
      else return s_it[(row0 + r) * ITS + j];
    };

    // ---- pass 1: z (and zdot)
    Real zr = 0, zi = 0, zdr = 0, zdi = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const Real s = planes[IT(r, 0) * stride + ev];
      const Real u = planes[IT(r, 1) * stride + ev] * TB(r, TB_UMUL) + TB(r, TB_UADD);
      const Real g = planes[IT(r, 2) * stride + ev];
      const Real Dr = TB(r, TB_M2) - s;
      const Real Di = TB(r, TB_NGE) * g;
      const Real inv = rcp_r(Dr * Dr + Di * Di);
      const Real wr = Dr * inv, wi = -Di * inv;
      const Real beta = TB(r, TB_BETA);
      const Real bu = beta * u;
      const Real ar = bu * wr, ai = bu * wi;
      const Real cr = TB(r, TB_CR), ci = TB(r, TB_CI);
      zr += cr * ar - ci * ai;
      zi += cr * ai + ci * ar;
      if constexpr (MODE == MODE_HVP) {
        const Real w2r = wr * wr - wi * wi, w2i = 2 * wr * wi;
        const Real Ddr = TB(r, TB_DDR), Ddi = TB(r, TB_DDIG) * g;
        const Real wdr = -(Ddr * w2r - Ddi * w2i), wdi = -(Ddr * w2i + Ddi * w2r);
        const Real bdot = TB(r, TB_BDOT);
        const Real adr = u * (bdot * wr + beta * wdr), adi = u * (bdot * wi + beta * wdi);
        const Real vr = TB(r, TB_VR), vi = TB(r, TB_VI);
        zdr += vr * ar - vi * ai + cr * adr - ci * adi;
        zdi += vr * ai + vi * ar + cr * adi + ci * adr;
      }
    }
    if constexpr (T > 1) {
#pragma unroll
      for (int off = 1; off < T; off <<= 1) {
        zr += __shfl_xor(zr, off);
        zi += __shfl_xor(zi, off);
        if constexpr (MODE == MODE_HVP) {
          zdr += __shfl_xor(zdr, off);
          zdi += __shfl_xor(zdi, off);
        }
      }
    }

    // ---- per-event weights
    const Real om = zr * zr + zi * zi;
    Real gr, gi, alr = 0, ali = 0;
    double sterm;
    if (rg.is_data) {
      sterm = (double)log_r(om);
      const Real io = rcp_r(om);
      gr = zr * io;
      gi = -zi * io;
      if constexpr (MODE == MODE_HVP) {
        const Real t = 2 * (zr * zdr + zi * zdi) * io;
        alr = (zdr - t * zr) * io;
        ali = (t * zi - zdi) * io;
      }
    } else {
      sterm = (double)om;
      gr = zr;
      gi = -zi;
      alr = zdr;
      ali = -zdi;
    }
    if (!valid) {
      sterm = 0.0;
      gr = gi = alr = ali = 0;
    }
    if (pos == 0) accS += sterm;

    // ---- pass 2: per-parameter sums
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const Real s = planes[IT(r, 0) * stride + ev];
      const Real u = planes[IT(r, 1) * stride + ev] * TB(r, TB_UMUL) + TB(r, TB_UADD);
      const Real g = planes[IT(r, 2) * stride + ev];
      const Real Dr = TB(r, TB_M2) - s;
      const Real Di = TB(r, TB_NGE) * g;
      const Real inv = rcp_r(Dr * Dr + Di * Di);
      const Real wr = Dr * inv, wi = -Di * inv;
      const Real w2r = wr * wr - wi * wi, w2i = 2 * wr * wi;
      const Real beta = TB(r, TB_BETA), beta1 = TB(r, TB_BETA1);
      const Real bu = beta * u;
      const Real ar = bu * wr, ai = bu * wi;
      const Real cr = TB(r, TB_CR), ci = TB(r, TB_CI);
      const Real dmr = TB(r, TB_2M), dmi = TB(r, TB_NGE1) * g;
      const Real wMr = -(dmr * w2r - dmi * w2i), wMi = -(dmr * w2i + dmi * w2r);
      const Real dgi = TB(r, TB_NETA) * g;
      const Real wGr = dgi * w2i, wGi = -dgi * w2r;
      const Real aMr = u * (beta1 * wr + beta * wMr), aMi = u * (beta1 * wi + beta * wMi);
      const Real aGr = bu * wGr, aGi = bu * wGi;
      const Real cMr = cr * aMr - ci * aMi, cMi = cr * aMi + ci * aMr;
      const Real cGr = cr * aGr - ci * aGi, cGi = cr * aGi + ci * aGr;
      acc[4 * r + 0] += (double)(gr * ar - gi * ai);
      acc[4 * r + 1] += (double)(-(gr * ai + gi * ar));
      acc[4 * r + 2] += (double)(gr * cMr - gi * cMi);
      acc[4 * r + 3] += (double)(gr * cGr - gi * cGi);
      if constexpr (MODE == MODE_HVP) {
        const Real Ddr = TB(r, TB_DDR), Ddi = TB(r, TB_DDIG) * g;
        const Real wdr = -(Ddr * w2r - Ddi * w2i), wdi = -(Ddr * w2i + Ddi * w2r);
        const Real bdot = TB(r, TB_BDOT), bdot1 = TB(r, TB_BDOT1);
        const Real adr = u * (bdot * wr + beta * wdr), adi = u * (bdot * wi + beta * wdi);
        const Real wwMr = wr * wMr - wi * wMi, wwMi = wr * wMi + wi * wMr;
        const Real e1r = TB(r, TB_DMDDR), e1i = TB(r, TB_DMDDIG) * g;
        const Real wdMr = -(e1r * w2r - e1i * w2i) - 2 * (Ddr * wwMr - Ddi * wwMi);
        const Real wdMi = -(e1r * w2i + e1i * w2r) - 2 * (Ddr * wwMi + Ddi * wwMr);
        const Real wwGr = wr * wGr - wi * wGi, wwGi = wr * wGi + wi * wGr;
        const Real e2i = TB(r, TB_DGDDIG) * g;
        const Real wdGr = e2i * w2i - 2 * (Ddr * wwGr - Ddi * wwGi);
        const Real wdGi = -e2i * w2r - 2 * (Ddr * wwGi + Ddi * wwGr);
        const Real adMr = u * (bdot1 * wr + bdot * wMr + beta1 * wdr + beta * wdMr);
        const Real adMi = u * (bdot1 * wi + bdot * wMi + beta1 * wdi + beta * wdMi);
        const Real adGr = u * (bdot * wGr + beta * wdGr), adGi = u * (bdot * wGi + beta * wdGi);
        const Real vr = TB(r, TB_VR), vi = TB(r, TB_VI);
        const Real zMr = vr * aMr - vi * aMi + cr * adMr - ci * adMi;
        const Real zMi = vr * aMi + vi * aMr + cr * adMi + ci * adMr;
        const Real zGr = vr * aGr - vi * aGi + cr * adGr - ci * adGi;
        const Real zGi = vr * aGi + vi * aGr + cr * adGi + ci * adGr;
        acc[NG + 4 * r + 0] += (double)((alr * ar - ali * ai) + (gr * adr - gi * adi));
        acc[NG + 4 * r + 1] += (double)(-(alr * ai + ali * ar) - (gr * adi + gi * adr));
        acc[NG + 4 * r + 2] += (double)((alr * cMr - ali * cMi) + (gr * zMr - gi * zMi));
        acc[NG + 4 * r + 3] += (double)((alr * cGr - ali * cGi) + (gr * zGr - gi * zGi));
      }
    }
  }

  // ---- reduction: wave butterfly over teams, then waves in fixed order
  __shared__ double red[NWAVE][T][NV][2];
  {
    double hi = accS, lo = 0.0;
    dd_wave_reduce(hi, lo, T);
    if (lane < T) {
      red[wave][lane][0][0] = hi;
      red[wave][lane][0][1] = lo;
    }
  }
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    double hi = acc[j], lo = 0.0;
    dd_wave_reduce(hi, lo, T);
    if (lane < T) {
      red[wave][lane][1 + j][0] = hi;
      red[wave][lane][1 + j][1] = lo;
    }
  }
  __syncthreads();
  const int K = a.K;
  const int V = 1 + 4 * K + ((MODE == MODE_HVP) ? 4 * K : 0);
  double* out = a.part + (int64_t)blockIdx.x * V * 2;
  for (int idx = tid; idx < T * NV; idx += BLOCK) {
    const int p = idx / NV, j = idx % NV;
    int vi = -1;
    if (j == 0) {
      if (p == 0) vi = 0;
    } else {
      const int q = (j - 1) % NG;
      const int k = p * R + q / 4;
      if (k < K) vi = 1 + ((j - 1) >= NG ? 4 * K : 0) + 4 * k + (q % 4);
    }
    if (vi < 0) continue;
    double h = red[0][p][j][0], l = red[0][p][j][1];
    for (int w = 1; w < NWAVE; ++w) dd_add(h, l, red[w][p][j][0], red[w][p][j][1]);
    out[vi * 2 + 0] = h;
    out[vi * 2 + 1] = l;
  }
}

// ------------------------------------------------------------------------
// 3. Finaliser and combine (eq. (4), (6), (7) for NLL = -ln L).
// Inputs are double-double totals; derivative totals still lack the factor 2
// of d|z|^2 = 2 Re(conj(z) dz) when `halved` is set.
// ------------------------------------------------------------------------
struct Totals {
  const double* F;   // dd pair
  const double* G;   // dd pair
  const double* dF;  // P dd pairs
  const double* dG;
  const double* HF;
  const double* HG;
  double scale;      // factor applied to derivative totals
};

__device__ void combine_block(const Totals& t, int P, int mode, double nd, double nm,
                              const double* v, double* nll, double* grad, double* hv,
                              int* status) {
  __shared__ double sc[3];
  const int tid = threadIdx.x;
  if (tid == 0) {
    const double F = t.F[0] + t.F[1];
    const double G = t.G[0] + t.G[1];
    double val = -F + nd * log(G / nm);
    int flags = status ? status[0] : 0;
    if (!(G > 0.0) || !isfinite(val)) flags |= 2;
    if (flags) val = INFINITY;
    double dh = 0.0, dl = 0.0;
    if (mode == MODE_HVP && v) {
      for (int p = 0; p < P; ++p) {
        const double gp = t.scale * (t.dG[2 * p] + t.dG[2 * p + 1]);
        const double prod = gp * v[p];
        dd_add(dh, dl, prod, fma(gp, v[p], -prod));
      }
    }
    sc[0] = G;
    sc[1] = dh + dl;
    sc[2] = val;
    if (nll) *nll = val;
    if (status) {
      status[0] = flags;
      if (flags) atomicOr(&status[1], flags);
    }
  }
  __syncthreads();
  if (mode == MODE_NLL) return;
  const double G = sc[0], dGv = sc[1];
  const double wG = nd / G;
  for (int p = tid; p < P; p += blockDim.x) {
    const double gF = t.scale * (t.dF[2 * p] + t.dF[2 * p + 1]);
    const double gG = t.scale * (t.dG[2 * p] + t.dG[2 * p + 1]);
    if (grad) grad[p] = -gF + wG * gG;
    if (mode == MODE_HVP && hv) {
      const double hF = t.scale * (t.HF[2 * p] + t.HF[2 * p + 1]);
      const double hG = t.scale * (t.HG[2 * p] + t.HG[2 * p + 1]);
      hv[p] = -hF + wG * hG - (wG / G) * gG * dGv;
    }
  }
}

__global__ __launch_bounds__(1024) void final_kernel(FinalArgs f) {
  __shared__ double tot[2 * (1 + 8 * PWA_MAX_RES) * 2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nw = blockDim.x >> 6;
  for (int vv = wave; vv < 2 * f.V; vv += nw) {
    const int set = vv >= f.V;
    const int vi = vv - set * f.V;
    const int b0 = set ? f.nb_data : 0;
    const int nb = set ? f.nb_mc : f.nb_data;
    double hi = 0.0, lo = 0.0;
    for (int b = lane; b < nb; b += 64)
      dd_add(hi, lo, f.part[((int64_t)(b0 + b) * f.V + vi) * 2], f.part[((int64_t)(b0 + b) * f.V + vi) * 2 + 1]);
    dd_wave_reduce(hi, lo, 1);
    if (lane == 0) {
      tot[vv * 2] = hi;
      tot[vv * 2 + 1] = lo;
    }
  }
  __syncthreads();
  const int K = f.K, P = 4 * K;
  const double* D = tot;                 // data set values
  const double* M = tot + 2 * f.V;       // MC set values
  if (f.out_kind == OUT_PARTIALS) {
    // [F, G, dF(P), dG(P), HFv(P), HGv(P)] as (hi, lo), derivatives x 2
    const int NOUT = 2 + 4 * P;
    for (int i = tid; i < NOUT; i += blockDim.x) {
      double h = 0.0, l = 0.0;
      if (i == 0) {
        h = D[0];
        l = D[1];
      } else if (i == 1) {
        h = M[0];
        l = M[1];
      } else {
        const int q = i - 2, grp = q / P, p = q % P;
        const double* src = (grp % 2 == 0) ? D : M;
        const int off = 1 + (grp >= 2 ? P : 0) + p;
        const bool have = (grp < 2) ? (f.mode >= MODE_GRAD) : (f.mode == MODE_HVP);
        if (have) {
          h = 2.0 * src[2 * off];
          l = 2.0 * src[2 * off + 1];
        }
      }
      f.dd_out[2 * i] = h;
      f.dd_out[2 * i + 1] = l;
    }
    if (tid == 0 && f.status && f.status[0]) atomicOr(&f.status[1], f.status[0]);
    return;
  }
  Totals t;
  t.F = D;
  t.G = M;
  t.dF = D + 2;
  t.dG = M + 2;
  t.HF = D + 2 + 2 * P;
  t.HG = M + 2 + 2 * P;
  t.scale = 2.0;
  combine_block(t, P, f.mode, f.n_data, f.n_mc, f.v, f.nll, f.grad, f.hv, f.status);
}

// pwa_combine: shard partials [F, G, dF, dG, HF, HG] (dd pairs, already
// including the factor 2), summed over shards in index order.
__global__ __launch_bounds__(1024) void combine_kernel(int P, int n_shards,
                                                       const double* __restrict__ parts,
                                                       double nd, double nm,
                                                       const double* __restrict__ v,
                                                       double* nll, double* grad, double* hv,
                                                       int* status) {
  __shared__ double tot[(2 + 4 * 4 * PWA_MAX_RES) * 2];
  const int NOUT = 2 + 4 * P;
  for (int i = threadIdx.x; i < NOUT; i += blockDim.x) {
    double h = 0.0, l = 0.0;
    for (int s = 0; s < n_shards; ++s)
      dd_add(h, l, parts[((int64_t)s * NOUT + i) * 2], parts[((int64_t)s * NOUT + i) * 2 + 1]);
    tot[2 * i] = h;
    tot[2 * i + 1] = l;
  }
  __syncthreads();
  Totals t;
  t.F = tot;
  t.G = tot + 2;
  t.dF = tot + 4;
  t.dG = tot + 4 + 2 * P;
  t.HF = tot + 4 + 4 * P;
  t.HG = tot + 4 + 6 * P;
  t.scale = 1.0;
  if (threadIdx.x == 0 && status) status[0] = 0;
  __syncthreads();
  combine_block(t, P, hv ? MODE_HVP : (grad ? MODE_GRAD : MODE_NLL), nd, nm, v, nll, grad, hv,
                status);
}

// ------------------------------------------------------------------------
// Launchers and the table of built launch shapes.
// ------------------------------------------------------------------------
hipError_t launch_precompute(const double* s12, const double* s13, int64_t n, int64_t offset,
                             void* planes, int64_t stride, int is_f32, const ModelDev& md,
                             const FieldSpec& fs, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((n + 255) / 256);
  if (is_f32)
    hipLaunchKernelGGL(precompute_kernel<float>, dim3(grid), dim3(256), 0, st, s12, s13, n,
                       offset, (float*)planes, stride, md, fs);
  else
    hipLaunchKernelGGL(precompute_kernel<double>, dim3(grid), dim3(256), 0, st, s12, s13, n,
                       offset, (double*)planes, stride, md, fs);
  return hipGetLastError();
}

hipError_t launch_table(const double* theta, const double* v, const ModelDev& md, int kslots,
                        double* tbl64, float* tbl32, int* itbl, int* status, hipStream_t st) {
  hipLaunchKernelGGL(table_kernel, dim3(1), dim3(64), 0, st, theta, v, md, kslots, tbl64, tbl32,
                     itbl, status);
  return hipGetLastError();
}

// Launch shapes (lanes per event T, resonances per lane R) that are built.
#define PWA_SHAPES(X) \
  X(1, 2) X(1, 4) X(1, 8) X(1, 12) X(2, 4) X(2, 6) X(4, 2) X(4, 3) X(4, 4) X(8, 2) X(8, 4) X(8, 8) X(16, 4)

bool shape_built(int T, int R) {
#define PWA_IS(TT, RR) if (T == TT && R == RR) return true;
  PWA_SHAPES(PWA_IS)
#undef PWA_IS
  return false;
}

typedef void (*EvalFn)(EvalArgs);

static EvalFn eval_fn(int is_f32, int mode, int T, int R) {
  if (mode == MODE_NLL) return is_f32 ? nll_kernel<float> : nll_kernel<double>;
#define PWA_PICK(TT, RR)                                                              \
  if (T == TT && R == RR) {                                                           \
    if (mode == MODE_GRAD)                                                            \
      return is_f32 ? eval_kernel<float, MODE_GRAD, TT, RR> : eval_kernel<double, MODE_GRAD, TT, RR>; \
    return is_f32 ? eval_kernel<float, MODE_HVP, TT, RR> : eval_kernel<double, MODE_HVP, TT, RR>;     \
  }
  PWA_SHAPES(PWA_PICK)
#undef PWA_PICK
  return nullptr;
}

hipError_t launch_eval(int is_f32, int mode, int T, int R, const EvalArgs& a, int nblocks,
                       hipStream_t st) {
  EvalFn fn = eval_fn(is_f32, mode, T, R);
  if (!fn) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fn, dim3(nblocks), dim3(BLOCK), 0, st, a);
  return hipGetLastError();
}

int eval_occupancy(int is_f32, int mode, int T, int R) {
  EvalFn fn = eval_fn(is_f32, mode, T, R);
  if (!fn) return 0;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)fn, BLOCK, 0) != hipSuccess)
    return 0;
  return nb;
}

hipError_t launch_final(const FinalArgs& f, hipStream_t st) {
  hipLaunchKernelGGL(final_kernel, dim3(1), dim3(1024), 0, st, f);
  return hipGetLastError();
}

hipError_t launch_combine(int n_par, int n_shards, const double* parts, double n_data,
                          double n_mc, const double* v, double* nll, double* grad, double* hv,
                          int* status, hipStream_t st) {
  hipLaunchKernelGGL(combine_kernel, dim3(1), dim3(1024), 0, st, n_par, n_shards, parts, n_data,
                     n_mc, v, nll, grad, hv, status);
  return hipGetLastError();
}

}  // namespace pwa
