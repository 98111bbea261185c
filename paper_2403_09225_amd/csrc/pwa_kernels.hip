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
// Kernel structure (one evaluation = 4 launches on the caller's stream):
//   1. table_kernel: per-resonance constants from (theta, v), including the
//      first and second M-derivatives of the mass-only factors, by
//      second-order Taylor arithmetic in one thread per resonance.
//   2. eval_kernel: one pass over the events.  A team of T lanes shares an
//      event; each lane owns R resonances and keeps their event moments in
//      FP64 registers over all the events it visits.  Event
//      sums are reduced per wave with a double-double butterfly and per block
//      in a fixed order into per-block (hi, lo) partials: no atomics, so the
//      result is bitwise reproducible for a given grid.
//   3. reduce_kernel + final_kernel: fixed-order double-double sum of the
//      block partials, contraction of the moments with the table, and the
//      eq. (4)/(6)/(7) combine (or the raw eq. (5) partials).

#include <math.h>

#include <type_traits>

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
__device__ __forceinline__ double sconst(double c) {
  asm volatile("" : "+s"(c));
  return c;
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
// Natural logarithm for x > 0 (finite, normal): x = m 2^e with m in
// [sqrt(1/2), sqrt(2)), ln m = 2 atanh(y), y = (m - 1)/(m + 1), |y| <= 0.1716,
// by its odd series through y^21 (truncation < 1e-19 relative), plus e ln 2
// with ln 2 split as hi + lo (hi = ln 2 with its 21 low mantissa bits
// cleared, so e * hi is exact).  Absolute error ~2e-16 max(1, |ln x|),
// about a third of the instructions of the library routine.
__device__ __forceinline__ double log_r(double x) {
  int e;
  double m = frexp(x, &e);
  const bool lo = m < 0.70710678118654752440;
  m = lo ? 2.0 * m : m;
  e = lo ? e - 1 : e;
  const double y = (m - 1.0) * rcp_r(m + 1.0);
  const double y2 = y * y;
  // the series coefficients are materialised in scalar registers at each
  // use: hoisted out of the event loop they would occupy vector registers
  double p = sconst(1.0 / 21.0);
  p = fma(p, y2, sconst(1.0 / 19.0));
  p = fma(p, y2, sconst(1.0 / 17.0));
  p = fma(p, y2, sconst(1.0 / 15.0));
  p = fma(p, y2, sconst(1.0 / 13.0));
  p = fma(p, y2, sconst(1.0 / 11.0));
  p = fma(p, y2, sconst(1.0 / 9.0));
  p = fma(p, y2, sconst(1.0 / 7.0));
  p = fma(p, y2, sconst(1.0 / 5.0));
  p = fma(p, y2, sconst(1.0 / 3.0));
  const double t = 2.0 * y;
  const double r = fma(t * y2, p, t);
  const double de = (double)e;
  return fma(de, 6.93147180369123816490e-01, fma(de, 1.90821492927058770002e-10, r));
}
// a * b + c as a multiply and an add (no contraction): when a and c are both
// wave-uniform scalars, a fused form would need one of them copied to a
// vector register first (one scalar operand per VALU instruction).
__device__ __forceinline__ double mad_nc(double a, double b, double c) {
#pragma clang fp contract(off)
  return a * b + c;
}
__device__ __forceinline__ float mad_nc(float a, float b, float c) {
#pragma clang fp contract(off)
  return a * b + c;
}
__device__ __forceinline__ double fma_r(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float fma_r(float a, float b, float c) { return fmaf(a, b, c); }
// FP64 accumulation of per-event terms (converted once for the FP32 path).
__device__ __forceinline__ void acc_add(double& acc, double x) { acc += x; }
__device__ __forceinline__ void acc_add(double& acc, float x) { acc += (double)x; }
__device__ __forceinline__ void acc_fma(double& acc, double a, double b) { acc = fma(a, b, acc); }
__device__ __forceinline__ void acc_fma(double& acc, float a, float b) { acc += (double)(a * b); }
// FP32 run accumulators (FP32 stream, wave-group pass): a few batches of
// per-event terms summed in FP32, then flushed into the FP64 accumulators.
__device__ __forceinline__ void acc_add(float& acc, float x) { acc += x; }
__device__ __forceinline__ void acc_fma(float& acc, float a, float b) { acc = fmaf(a, b, acc); }
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
// General physics path: per channel with a Flatte resonance the width
// factor rho_ab + r rho_2 (real and imaginary planes); for a spin-1 parent
// the complex angular factors u^mu = F_J(z) Y_J^mu of mu = +1, -1 (from the
// event's orientation: daughter momenta in the parent frame, the bachelor
// direction and the direction of a in the pair's rest frame); a zero plane.
// ------------------------------------------------------------------------
struct V3 {
  double x, y, z;
};
__device__ __forceinline__ V3 v3(double x, double y, double z) { return {x, y, z}; }
__device__ __forceinline__ double dot3(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross3(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ V3 scale3(V3 a, double k) { return {a.x * k, a.y * k, a.z * k}; }
__device__ __forceinline__ V3 unit3(V3 a) {
  const double n = sqrt(dot3(a, a));
  return n > 0.0 ? scale3(a, 1.0 / n) : v3(0.0, 0.0, 0.0);
}

template <typename Real>
__global__ __launch_bounds__(256) void precompute_kernel(const double* __restrict__ s12,
                                                         const double* __restrict__ s13,
                                                         const double* __restrict__ cosb,
                                                         const double* __restrict__ gam,
                                                         int64_t n, int64_t offset,
                                                         Real* __restrict__ planes,
                                                         int64_t stride, ModelDev md,
                                                         FieldSpec fs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x12 = s12[i], x13 = s13[i];
  const double x23 = md.M2 + md.msq[0] + md.msq[1] + md.msq[2] - x12 - x13;
  const int64_t o = offset + i;
  if (fs.zero_field >= 0) planes[fs.zero_field * stride + o] = (Real)0;
  // spin-1 parent: daughter momenta in the parent rest frame, the decay
  // plane rotated from the reference plane (p_1 along x, p_2 in the upper
  // x-y half plane) by R_y(beta) R_z(gamma)
  V3 pl[3] = {};
  double En[3] = {};
  if (md.parent_spin == 1) {
    const double M = sqrt(md.M2);
    const double sjk[3] = {x23, x13, x12};
    double pm[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      En[d] = (md.M2 + md.msq[d] - sjk[d]) / (2.0 * M);
      pm[d] = sqrt(fmax(En[d] * En[d] - md.msq[d], 0.0));
    }
    double c12 = (En[0] * En[1] - 0.5 * (x12 - md.msq[0] - md.msq[1])) / (pm[0] * pm[1]);
    c12 = fmin(1.0, fmax(-1.0, c12));
    const double s12n = sqrt(fmax(1.0 - c12 * c12, 0.0));
    const V3 body[3] = {v3(pm[0], 0.0, 0.0), v3(pm[1] * c12, pm[1] * s12n, 0.0),
                        v3(-pm[0] - pm[1] * c12, -pm[1] * s12n, 0.0)};
    const double cb = cosb[i], sb = sqrt(fmax(1.0 - cb * cb, 0.0));
    const double cg = cos(gam[i]), sg = sin(gam[i]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double xr = body[d].x * cg - body[d].y * sg, yr = body[d].x * sg + body[d].y * cg;
      pl[d] = v3(xr * cb, yr, -xr * sb);
    }
  }
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
    if (fs.fg_field[c] >= 0) {
      // Flatte width factor rho_ab + r rho_2, rho = sqrt(lambda) / s, the
      // second channel continued below threshold to +i sqrt(-lambda) / s
      const double lam2 = kallen(sab, md.fl_msq[0], md.fl_msq[1]);
      const double r2re = lam2 >= 0.0 ? sqrt(lam2) / sab : 0.0;
      const double r2im = lam2 < 0.0 ? sqrt(-lam2) / sab : 0.0;
      planes[fs.fg_field[c] * stride + o] = (Real)(2.0 * q / rs + md.fl_ratio * r2re);
      planes[fs.fh_field[c] * stride + o] = (Real)(md.fl_ratio * r2im);
    }
    // spin-1 parent: unit bachelor momentum and unit momentum of a in the
    // (ab) rest frame (boost along the pair momentum P = -p_c)
    V3 pc = {}, qa = {};
    if (md.parent_spin == 1) {
      pc = unit3(pl[cc]);
      const V3 P = scale3(pl[cc], -1.0);
      const double Eab = En[a] + En[b];
      const double Pm = sqrt(dot3(P, P));
      V3 pa = pl[a];
      if (Pm > 0.0) {
        const V3 Ph = scale3(P, 1.0 / Pm);
        const double gb = Eab / rs, bb = Pm / Eab;
        const double k = (gb - 1.0) * dot3(pa, Ph) - gb * bb * En[a];
        pa = v3(pa.x + k * Ph.x, pa.y + k * Ph.y, pa.z + k * Ph.z);
      }
      qa = unit3(pa);
    }
#pragma unroll
    for (int J = 0; J < 3; ++J) {
      const int gf = fs.g_field[c][J];
      if (gf < 0) continue;
      const double F2 = (J == 0) ? 1.0 : (J == 1 ? 1.0 / (1.0 + z) : 1.0 / (z * z + 3.0 * z + 9.0));
      const double q2 = q * q;
      const double qp = (J == 0) ? q : (J == 1 ? q * q2 : q * q2 * q2);   // q^(2J+1)
      const double g = (md.width_mode == PWA_WIDTH_MASS_DEPENDENT) ? qp * F2 / rs : 1.0;
      planes[gf * stride + o] = (Real)g;
      if (J >= 1 && fs.u_field[c][J] >= 0) {
        const double PJ = (J == 1) ? cs : 1.5 * cs * cs - 0.5;
        planes[fs.u_field[c][J] * stride + o] = (Real)(sqrt(F2) * PJ);
      }
      if (md.parent_spin == 1 && fs.uc_field[c][J][0] >= 0) {
        // Y_J^mu with e_+ = -(1, i, 0)/sqrt2, e_- = (1, -i, 0)/sqrt2:
        // e_pm . v = -+(v_x +- i v_y) / sqrt2
        V3 yv;   // Y_J = e . yv
        if (J == 0) yv = pc;
        else if (J == 1) yv = cross3(pc, qa);
        else {
          const double qp_ = dot3(qa, pc);
          yv = v3(qa.x * qp_ - pc.x / 3.0, qa.y * qp_ - pc.y / 3.0, qa.z * qp_ - pc.z / 3.0);
        }
        const double f = sqrt(F2) * 0.70710678118654752440;
        planes[fs.uc_field[c][J][0] * stride + o] = (Real)(-f * yv.x);
        planes[fs.uc_field[c][J][1] * stride + o] = (Real)(-f * yv.y);
        planes[fs.uc_field[c][J][2] * stride + o] = (Real)(f * yv.x);
        planes[fs.uc_field[c][J][3] * stride + o] = (Real)(-f * yv.y);
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
      Jet beta = {1.0, 0.0, 0.0}, eta = {1.0, 0.0, 0.0};
      if (md.lineshape[k] == PWA_LINESHAPE_FLATTE) {
        // D = M^2 - s - i g_1 (g + i h): eta = 1, no barrier (J = 0)
        if (!isfinite(M)) atomicOr(&bad, 1);
      } else {
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
        if (J > 0) beta = jsqrt(Finv2);
        if (md.width_mode == PWA_WIDTH_MASS_DEPENDENT) {
          Jet qp = jsqrt(Q);  // q0^(2J+1)
          for (int j = 0; j < J; ++j) qp = jmul(qp, Q);
          eta = jmul(jmul(M2, Finv2), jrcp(qp));
        } else {
          eta = Mj;
        }
      }
      const double Ddr = 2.0 * M * vM;
      const double Ddig = -(vM * G * eta.d + vG * eta.v);
      const double bdot = vM * beta.d;
      const double cbr = cr * beta.v, cbi = ci * beta.v;
      e[TB_M2] = M * M;
      e[TB_NGE] = -G * eta.v;
      // u = u_plane UMUL + UADD: J = 0 of a spin-0 parent has u = 1
      const bool u_one = (J == 0 && md.parent_spin == 0);
      e[TB_UMUL] = u_one ? 0.0 : 1.0;
      e[TB_UADD] = u_one ? 1.0 : 0.0;
      e[TB_CBR] = cbr;
      e[TB_CBI] = cbi;
      e[TB_K1R] = vr * beta.v + cr * bdot;   // cdot beta + c beta'v_M
      e[TB_K1I] = vi * beta.v + ci * bdot;
      e[TB_K2R] = -cbr * Ddr;                // -c beta Ddr
      e[TB_K2I] = -cbi * Ddr;
      e[TB_K3R] = cbi * Ddig;                // -i c beta Ddig
      e[TB_K3I] = -cbr * Ddig;
      e[TB_BETA] = beta.v;
      e[TB_BETA1] = beta.d;
      e[TB_BDOT] = bdot;
      e[TB_BDOT1] = vM * beta.dd;
      e[TB_CR] = cr;
      e[TB_CI] = ci;
      e[TB_VR] = vr;
      e[TB_VI] = vi;
      e[TB_VM] = vM;
      e[TB_2M] = 2.0 * M;
      e[TB_NGE1] = -G * eta.d;
      e[TB_NETA] = -eta.v;
      e[TB_DDR] = Ddr;
      e[TB_DDIG] = Ddig;
      e[TB_DMDDIG] = -(vM * G * eta.dd + vG * eta.d);
      e[TB_DGDDIG] = -vM * eta.d;
#pragma unroll
      for (int j = 0; j < ITS; ++j) f[j] = md.fidx[k][j];
    } else {
      // inert padding slot: c = v = 0 so it adds nothing; D = -1 - s != 0
      // (its planes are the first resonance's, which exist)
      e[TB_M2] = -1.0;
      e[TB_UADD] = 1.0;
#pragma unroll
      for (int j = 0; j < ITS; ++j) f[j] = md.fidx[0][j];
      f[IT_J] = 0;
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
// Ranges start at multiples of 64 events from a set base that is itself a
// multiple of 64, so every 64-event batch is one aligned 64-event chunk of
// each plane (inside the plane: the stride is a multiple of 64).
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
  rg.base = rg.is_data ? 0 : a.mc_base;
  const int64_t chunk = ((n_set + nb_set - 1) / nb_set + 63) / 64 * 64;
  rg.begin = min(n_set, (int64_t)bi * chunk);
  rg.end = min(n_set, rg.begin + chunk);
  return rg;
}

// ------------------------------------------------------------------------
// Gradient / HVP pass.
//
// Per event and resonance, with w = 1/D and the per-event weights
//   data: gamma = conj(z)/|z|^2, alpha = (conj(zdot) - (2 Re(conj(z) zdot)/|z|^2) conj(z))/|z|^2
//   MC:   gamma = conj(z),       alpha = conj(zdot)
// (zdot = dz along v), every gradient and HVP component is 2 Re of a linear
// combination of the event moments
//   C1..C6 = gamma u {w, w^2, g w^2, w^3, g w^3, g^2 w^3},
//   B1..B3 = alpha u {w, w^2, g w^2},
// with coefficients that depend on the resonance parameters only (the
// derivatives of w = 1/D in M and Gamma are polynomials in w and g).  The
// pass therefore accumulates these 9 complex moments per resonance in FP64
// registers and the finaliser contracts them with the table.  The gradient
// pass needs C1..C3 only.  z and zdot themselves are
//   z = sum c beta u w,  zdot = sum K1 u w + K2 u w^2 + K3 u g w^2.
// ------------------------------------------------------------------------
template <typename Real, int MODE, int T, int R>
__global__ __launch_bounds__(BLOCK) void eval_kernel(EvalArgs a) {
  static_assert(64 % T == 0, "team size must divide the wavefront");
  typedef typename CPtr<Real>::type CReal;
  constexpr bool HVP = (MODE == MODE_HVP);
  constexpr bool BON = (MODE == MODE_HVPB);   // direction moments B1..B3 only
  constexpr bool ZD = HVP || BON;             // zdot needed
  constexpr bool DER = (MODE != MODE_NLL);
  constexpr int TEAMS = BLOCK / T;
  constexpr int NM = HVP ? NMOM_HVP : (DER ? NMOM_GRAD : 0);
  constexpr int NA = NM * R;
  constexpr int NV = 1 + NA;
  constexpr int NSLOT = T * R;
  constexpr int NWAVE = BLOCK / 64;
  // The next event's stream values are prefetched unless that would hold
  // too many registers (one lane per event with many resonances).
  constexpr bool PREFETCH = (T > 1) || (R <= 4);

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int team = tid / T;
  const int pos = tid % T;
  const Range rg = block_range(a);
  const Real* __restrict__ planes = (const Real*)a.planes;
  const int64_t stride = a.stride;
  const Real* tsrc = (sizeof(Real) == 8) ? (const Real*)a.tbl64 : (const Real*)a.tbl32;

  __shared__ Real s_tb[(T > 1) ? NSLOT * TB_HOT : 1];
  __shared__ int s_it[(T > 1) ? NSLOT * ITS : 1];
  if constexpr (T > 1) {
    for (int i = tid; i < NSLOT * TB_HOT; i += BLOCK) s_tb[i] = tsrc[(i / TB_HOT) * TS + i % TB_HOT];
    for (int i = tid; i < NSLOT * ITS; i += BLOCK) s_it[i] = a.itbl[i];
    __syncthreads();
  }

  // Stream values of resonance slot r at event ev.  T > 1: plane pointers
  // of this lane's rows, computed once; T == 1: plane indices read as
  // wave-uniform scalars in the loop (scalar-unit address arithmetic).
  const Real* ps[(T > 1) ? R : 1];
  const Real* pu[(T > 1) ? R : 1];
  const Real* pg[(T > 1) ? R : 1];
  if constexpr (T > 1) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      ps[r] = planes + (int64_t)s_it[(pos * R + r) * ITS + 0] * stride;
      pu[r] = planes + (int64_t)s_it[(pos * R + r) * ITS + 1] * stride;
      pg[r] = planes + (int64_t)s_it[(pos * R + r) * ITS + 2] * stride;
    }
  }
  auto load3 = [&](int64_t ev, Real* s_, Real* u_, Real* g_) {
    if constexpr (T > 1) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        s_[r] = ps[r][ev];
        u_[r] = pu[r][ev];
        g_[r] = pg[r][ev];
      }
    } else {
      // wave-uniform plane bases + one 32-bit byte offset (the stride is
      // limited to 2^32 bytes per plane at bind time)
      c_int* it = opaque_s((c_int*)a.itbl);
      const uint32_t off = (uint32_t)ev * (uint32_t)sizeof(Real);
      auto ld = [&](int field) -> Real {
        // the plane base is formed in scalar registers and kept there
        const char* base = opaque_s((const char*)(planes + (int64_t)field * stride));
        return *(const Real*)(base + off);
      };
#pragma unroll
      for (int r = 0; r < R; ++r) {
        s_[r] = ld(it[r * ITS + 0]);
        u_[r] = ld(it[r * ITS + 1]);
        g_[r] = ld(it[r * ITS + 2]);
      }
    }
  };

  double accS = 0.0;
  double acc[NA > 0 ? NA : 1];
#pragma unroll
  for (int j = 0; j < NA; ++j) acc[j] = 0.0;

  if (rg.begin < rg.end) {
    // Software pipeline: the stream values of the next event are loaded
    // while the current one is computed.
    Real sc[R], uc[R], gc[R];
    if constexpr (PREFETCH) {
      const int64_t e = rg.begin + team;
      load3(rg.base + (e < rg.end ? e : rg.begin), sc, uc, gc);
    }
    for (int64_t e0 = rg.begin; e0 < rg.end; e0 += TEAMS) {
      const bool valid = e0 + team < rg.end;
      Real sn[PREFETCH ? R : 1], un[PREFETCH ? R : 1], gn[PREFETCH ? R : 1];
      if constexpr (PREFETCH) {
        const int64_t en = e0 + TEAMS + team;
        load3(rg.base + (en < rg.end ? en : rg.begin), sn, un, gn);
      } else {
        load3(rg.base + (valid ? e0 + team : rg.begin), sc, uc, gc);
      }

      // Table access: scalar loads for T == 1, this lane's LDS rows otherwise.
      CReal* tb = opaque_s((CReal*)tsrc);
      const int row0 = (T > 1) ? opaque_v(pos * R) : 0;
      auto TB = [&](int r, int slot) -> Real {
        if constexpr (T == 1) return tb[r * TS + slot];
        else return s_tb[(row0 + r) * TB_HOT + slot];
      };

      // ---- pass 1: z (and zdot); keep w and u w of each resonance
      Real cwr[R], cwi[R], cuwr[R], cuwi[R];
      Real zr = 0, zi = 0, zdr = 0, zdi = 0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const Real s = sc[r];
        // scalar table operands (T == 1): multiply and add, one scalar each
        const Real u = (T == 1) ? mad_nc(uc[r], TB(r, TB_UMUL), TB(r, TB_UADD))
                                : uc[r] * TB(r, TB_UMUL) + TB(r, TB_UADD);
        const Real g = gc[r];
        const Real Dr = TB(r, TB_M2) - s;
        const Real Di = TB(r, TB_NGE) * g;
        const Real inv = rcp_r(Dr * Dr + Di * Di);
        const Real wr = Dr * inv, wi = -Di * inv;
        const Real uwr = u * wr, uwi = u * wi;
        const Real cbr = TB(r, TB_CBR), cbi = TB(r, TB_CBI);
        zr = fma_r(cbr, uwr, fma_r(-cbi, uwi, zr));
        zi = fma_r(cbr, uwi, fma_r(cbi, uwr, zi));
        if constexpr (ZD) {
          // zdot += K1 u w + (K2 + K3 g) u w^2
          const Real uw2r = uwr * wr - uwi * wi, uw2i = uwr * wi + uwi * wr;
          const Real kr = (T == 1) ? mad_nc(TB(r, TB_K3R), g, TB(r, TB_K2R))
                                   : fma_r(TB(r, TB_K3R), g, TB(r, TB_K2R));
          const Real ki = (T == 1) ? mad_nc(TB(r, TB_K3I), g, TB(r, TB_K2I))
                                   : fma_r(TB(r, TB_K3I), g, TB(r, TB_K2I));
          const Real k1r = TB(r, TB_K1R), k1i = TB(r, TB_K1I);
          zdr = fma_r(k1r, uwr, fma_r(-k1i, uwi, fma_r(kr, uw2r, fma_r(-ki, uw2i, zdr))));
          zdi = fma_r(k1r, uwi, fma_r(k1i, uwr, fma_r(kr, uw2i, fma_r(ki, uw2r, zdi))));
        }
        cwr[r] = wr;
        cwi[r] = wi;
        cuwr[r] = uwr;
        cuwi[r] = uwi;
      }
      if constexpr (T > 1) {
#pragma unroll
        for (int off = 1; off < T; off <<= 1) {
          zr += __shfl_xor(zr, off);
          zi += __shfl_xor(zi, off);
          if constexpr (ZD) {
            zdr += __shfl_xor(zdr, off);
            zdi += __shfl_xor(zdi, off);
          }
        }
      }

      // ---- per-event weights
      const Real om = zr * zr + zi * zi;
      Real gr = 0, gi = 0, alr = 0, ali = 0;
      double sterm = 0.0;
      if (rg.is_data) {
        if constexpr (!BON) sterm = (double)log_r(om);
        if constexpr (DER) {
          const Real io = rcp_r(om);
          gr = zr * io;
          gi = -zi * io;
          if constexpr (ZD) {
            const Real t = 2 * (zr * zdr + zi * zdi) * io;
            alr = (zdr - t * zr) * io;
            ali = (t * zi - zdi) * io;
          }
        }
      } else {
        if constexpr (!BON) sterm = (double)om;
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

      // ---- pass 2: moments, as the chain p = x u w, q = p w, r = q w
      // (x = gamma or alpha) so that C2 = sum q, C3 = sum g q, C4 = sum r, ...
      if constexpr (BON) {
        // B1..B3 = alpha u {w, w^2, g w^2} only (C1..C6 depend on theta alone)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const Real wr = cwr[r], wi = cwi[r], uwr = cuwr[r], uwi = cuwi[r], g = gc[r];
          double* m = acc + NM * r;
          const Real ar_ = alr * uwr - ali * uwi, ai_ = alr * uwi + ali * uwr;
          const Real br_ = ar_ * wr - ai_ * wi, bi_ = ar_ * wi + ai_ * wr;
          acc_add(m[0], ar_);
          acc_add(m[1], ai_);
          acc_add(m[2], br_);
          acc_add(m[3], bi_);
          acc_fma(m[4], g, br_);
          acc_fma(m[5], g, bi_);
        }
      } else if constexpr (DER) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const Real wr = cwr[r], wi = cwi[r], uwr = cuwr[r], uwi = cuwi[r], g = gc[r];
          double* m = acc + NM * r;
          const Real pr = gr * uwr - gi * uwi, pi = gr * uwi + gi * uwr;
          const Real qr = pr * wr - pi * wi, qi = pr * wi + pi * wr;
          acc_add(m[0], pr);
          acc_add(m[1], pi);
          acc_add(m[2], qr);
          acc_add(m[3], qi);
          acc_fma(m[4], g, qr);
          acc_fma(m[5], g, qi);
          if constexpr (HVP) {
            const Real ar_ = alr * uwr - ali * uwi, ai_ = alr * uwi + ali * uwr;
            const Real br_ = ar_ * wr - ai_ * wi, bi_ = ar_ * wi + ai_ * wr;
            acc_add(m[6], ar_);
            acc_add(m[7], ai_);
            acc_add(m[8], br_);
            acc_add(m[9], bi_);
            acc_fma(m[10], g, br_);
            acc_fma(m[11], g, bi_);
            const Real rr = qr * wr - qi * wi, ri = qr * wi + qi * wr;
            const Real g2 = g * g;
            acc_add(m[12], rr);
            acc_add(m[13], ri);
            acc_fma(m[14], g, rr);
            acc_fma(m[15], g, ri);
            acc_fma(m[16], g2, rr);
            acc_fma(m[17], g2, ri);
          }
        }
      }
      if constexpr (PREFETCH) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          sc[r] = sn[r];
          uc[r] = un[r];
          gc[r] = gn[r];
        }
      }
    }
  }

  // ---- reduction: wave butterfly over teams, then waves in fixed order,
  // CH values per round to bound the LDS footprint.
  // Block partial layout: [S, moments of resonance 0 (NM), resonance 1, ...].
  constexpr int CH = 8;
  __shared__ double red[NWAVE][T][CH][2];
  const int K = a.K;
  const int V = 1 + NM * K;
  double* out = a.part + (int64_t)blockIdx.x * V * 2;
#pragma unroll
  for (int j0 = 0; j0 < NV; j0 += CH) {
#pragma unroll
    for (int jj = 0; jj < CH; ++jj) {
      const int j = j0 + jj;
      if (j < NV) {
        double hi = (j == 0) ? accS : acc[j > 0 ? j - 1 : 0], lo = 0.0;
        dd_wave_reduce(hi, lo, T);
        if (lane < T) {
          red[wave][lane][jj][0] = hi;
          red[wave][lane][jj][1] = lo;
        }
      }
    }
    __syncthreads();
    for (int idx = tid; idx < T * CH; idx += BLOCK) {
      const int p = idx / CH, jj = idx % CH, j = j0 + jj;
      if (j >= NV) continue;
      int vi = -1;
      if (j == 0) {
        if (p == 0) vi = 0;
      } else {
        const int k = p * R + (j - 1) / NM;
        if (k < K) vi = 1 + NM * k + (j - 1) % NM;
      }
      if (vi < 0) continue;
      double h = red[0][p][jj][0], l = red[0][p][jj][1];
      for (int w = 1; w < NWAVE; ++w) dd_add(h, l, red[w][p][jj][0], red[w][p][jj][1]);
      out[vi * 2 + 0] = h;
      out[vi * 2 + 1] = l;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------------
// Wave-group layout of the same pass: the G waves of a block share each batch
// of 64 events (one event per lane) and wave g owns resonances
// [g R, g R + R).  The block stages the stream of each batch in LDS with
// direct global-to-LDS loads: one 16-byte load per lane brings 64 events of
// PPI planes (2 FP64 or 4 FP32 planes), the load instructions of a batch
// are spread over the block's waves, and so each plane chunk is read from
// memory once per block however many of its resonances use it.  Three stage
// buffers keep the loads of the next two batches in flight while a batch is
// computed.  Table rows are wave-uniform (scalar registers); the partial z,
// zdot of the G waves are exchanged through LDS (double-buffered, one
// barrier per batch).  Per lane the moment accumulators are those of R
// resonances, as in the team layout.
// ------------------------------------------------------------------------
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glob_void_t;
constexpr int NSTAGE = 3;

size_t stage_lds_bytes(int n_fields, int bytes) {
  return (size_t)NSTAGE * stage_planes(n_fields, bytes) * 64 * bytes;
}

// Dynamic LDS of a pass kernel: NSTAGE stage buffers (layout 2), one
// (layout 3, the general path), none (layout 1).
size_t pass_lds_bytes(int layout, int n_fields, int bytes) {
  if (layout == 2) return stage_lds_bytes(n_fields, bytes);
  if (layout == 3) return (size_t)stage_planes(n_fields, bytes) * 64 * bytes;
  return 0;
}

// s_waitcnt immediate (gfx9 field layout) that waits until at most n vector
// memory operations of this wave are in flight and leaves the other counters
// alone; and the wave-uniform dispatch of it (immediates only).
__host__ __device__ constexpr int vm_wait_imm(int n) {
  return (n & 0xF) | (0x7 << 4) | (0xF << 8) | (((n >> 4) & 3) << 14);
}
__device__ __forceinline__ void wait_vm_at_most(int n) {
  switch (n) {
    case 1: __builtin_amdgcn_s_waitcnt(vm_wait_imm(1)); break;
    case 2: __builtin_amdgcn_s_waitcnt(vm_wait_imm(2)); break;
    case 3: __builtin_amdgcn_s_waitcnt(vm_wait_imm(3)); break;
    case 4: __builtin_amdgcn_s_waitcnt(vm_wait_imm(4)); break;
    case 5: __builtin_amdgcn_s_waitcnt(vm_wait_imm(5)); break;
    case 6: __builtin_amdgcn_s_waitcnt(vm_wait_imm(6)); break;
    case 7: __builtin_amdgcn_s_waitcnt(vm_wait_imm(7)); break;
    case 8: __builtin_amdgcn_s_waitcnt(vm_wait_imm(8)); break;
    case 9: __builtin_amdgcn_s_waitcnt(vm_wait_imm(9)); break;
    default: __builtin_amdgcn_s_waitcnt(vm_wait_imm(0)); break;
  }
}

// Block barrier over LDS written by the block's waves: this wave's LDS
// operations are drained (lgkmcnt(0)), then s_barrier.  Unlike
// __syncthreads it carries no memory-model fence, which would also wait for
// the global-to-LDS loads of later batches still in flight; those are waited
// for explicitly, one batch ahead (wait_vm_at_most).
__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

template <typename Real, int MODE, int G, int R>
__global__ __launch_bounds__(64 * G) void wg_kernel(EvalArgs a) {
  typedef typename CPtr<Real>::type CReal;
  constexpr bool HVP = (MODE == MODE_HVP);
  constexpr bool BON = (MODE == MODE_HVPB);   // direction moments B1..B3 only
  constexpr bool ZD = HVP || BON;             // zdot needed
  constexpr bool DER = (MODE != MODE_NLL);
  constexpr int NM = HVP ? NMOM_HVP : (DER ? NMOM_GRAD : 0);   // B-only: 6, as GRAD
  constexpr int NA = NM * R;
  constexpr int NX = ZD ? 4 : 2;      // exchanged reals per lane: z (, zdot)
  constexpr int PPI = stage_ppi((int)sizeof(Real));   // planes per load instruction
  constexpr int LPP = 64 / PPI;                       // lanes per plane
  constexpr int JMAX = (stage_planes(MAX_FIELDS, (int)sizeof(Real)) / PPI + G - 1) / G;

  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const Range rg = block_range(a);
  const Real* __restrict__ planes = (const Real*)a.planes;
  const int64_t stride = a.stride;
  const Real* tsrc = ((sizeof(Real) == 8) ? (const Real*)a.tbl64 : (const Real*)a.tbl32) + wv * R * TS;

  // stage buffers: NSTAGE x nfp planes x 64 events (dynamic LDS)
  extern __shared__ __attribute__((aligned(16))) char stage_lds[];
  Real* stg = (Real*)stage_lds;
  // z and zdot exchange, double buffered: one array of (re, im) pairs per
  // quantity, so each lane's access is one contiguous pair (a 32-byte
  // per-lane stride for FP64 would conflict in the LDS banks)
  __shared__ Real xch[2][G][NX / 2][64][2];

  double accS = 0.0;
  double acc[NA > 0 ? NA : 1];
#pragma unroll
  for (int j = 0; j < NA; ++j) acc[j] = 0.0;
  // With the FP32 stream the moments of kRun batches are summed in FP32 run
  // accumulators and then added to the FP64 ones: one FP32 add per term
  // instead of a conversion and an FP64 add (a run of 8 per-lane terms costs
  // at most a few FP32 roundings, far inside the stream's own 2^-24).  Only
  // up to 3 resonances per wave and 8 waves per block: beyond that the extra
  // registers would spill.
  constexpr bool RUN = sizeof(Real) == 4 && NA <= 3 * NMOM_HVP && G <= 8;
  constexpr int kRun = 8;
  typedef typename std::conditional<RUN, float, double>::type AccR;
  AccR racc[RUN && NA > 0 ? NA : 1];
#pragma unroll
  for (int j = 0; j < (RUN ? NA : 0); ++j) racc[j] = 0.f;
  AccR* const macc = [&]() -> AccR* {
    if constexpr (RUN) return racc;
    else return acc;
  }();
  auto flush = [&]() {
    if constexpr (RUN) {
#pragma unroll
      for (int j = 0; j < NA; ++j) {
        acc[j] += (double)racc[j];
        racc[j] = 0.f;
      }
    }
  };

  const int nbat = (int)((rg.end - rg.begin + 63) / 64);
  if (nbat > 0) {
    const int nf = a.n_fields;
    const int ni = (nf + PPI - 1) / PPI;        // load instructions per batch
    const int nfp = ni * PPI;                   // staged planes (padded)
    // this wave's load instructions j = wv + G jj: lane l brings 16 bytes of
    // plane j PPI + l / LPP at event (l % LPP) PPI of the batch; in the last
    // group, lanes past the last plane load that plane again (same
    // addresses as its own lanes: no extra memory traffic) into padding LDS
    // slots that are never read.  The lane's byte offset from the
    // wave-uniform address of the group's first plane fits 32 bits (the
    // bound on the stride is checked at bind).
    const uint32_t pbytes = (uint32_t)(stride * (int64_t)sizeof(Real));
    const uint32_t voff = (uint32_t)(lane / LPP) * pbytes + (uint32_t)(lane % LPP) * 16u;
    const uint32_t voff_last = (uint32_t)min(lane / LPP, nf - 1 - (ni - 1) * PPI) * pbytes +
                               (uint32_t)(lane % LPP) * 16u;
    const Real* bsrc = planes + rg.base + rg.begin;
    int nmine = 0;
#pragma unroll
    for (int jj = 0; jj < JMAX; ++jj) nmine += (wv + G * jj < ni) ? 1 : 0;
    // batch b (clamped to the last one: loads past the range refetch it)
    // into stage buffer `stage`
    auto issue = [&](int b, int stage) {
      const int64_t off = (int64_t)min(b, nbat - 1) * 64;
#pragma unroll
      for (int jj = 0; jj < JMAX; ++jj) {
        const int j = wv + G * jj;
        if (j < ni) {
          const char* base = (const char*)(bsrc + (int64_t)j * PPI * stride + off);
          __builtin_amdgcn_global_load_lds((glob_void_t*)(base + (j == ni - 1 ? voff_last : voff)),
                                           (lds_void_t*)(stg + (stage * nfp + j * PPI) * 64), 16, 0, 0);
        }
      }
    };
    // LDS offsets (reals) of this wave's (s, u, g) planes
    int fo[R][3];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int k = 0; k < 3; ++k) fo[r][k] = a.itbl[(wv * R + r) * ITS + k] * 64;

    issue(0, 0);
    issue(1, 1);
    wait_vm_at_most(nmine);   // this wave's loads of batch 0 are in LDS
    lds_barrier();            // and so are every wave's
    int stage = 0, buf = 0;
    // One batch.  LAST: the block's last batch, the only one whose lanes can
    // lie past the range (a separate instance, so the others carry no
    // per-lane masking).
    auto step = [&](const int b, auto last_tag) {
      constexpr bool LAST = decltype(last_tag)::value;
      // ---- this batch's stream values, then the refill two batches ahead
      // (the buffer read one batch ago, which every wave has finished with:
      // all passed the last barrier after reading it)
      Real sc[R], uc[R], gc[R];
      {
        const Real* sb = stg + stage * nfp * 64 + lane;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          sc[r] = sb[fo[r][0]];
          uc[r] = sb[fo[r][1]];
          gc[r] = sb[fo[r][2]];
        }
      }
      asm volatile("" ::: "memory");
      issue(b + 2, stage == 0 ? 2 : stage - 1);
      const int64_t e0 = rg.begin + (int64_t)b * 64;
      if (LAST && !(e0 + lane < rg.end)) {
        // lanes past the range (last batch only) may hold the unwritten
        // padding between the data and MC sets: give them finite values
        // (D = M^2 - 0 is nonzero), their contributions are zeroed below
#pragma unroll
        for (int r = 0; r < R; ++r) sc[r] = uc[r] = gc[r] = 0;
      }
      CReal* tb = opaque_s((CReal*)tsrc);

      // ---- pass 1: this wave's share of z (and zdot)
      Real cwr[R], cwi[R], cu[R];
      Real zr = 0, zi = 0, zdr = 0, zdi = 0;
      // D = (M^2 - s) - i Gamma eta g and |D|^2 for the wave's resonances;
      // in FP64 one reciprocal serves all R (prefix products, then each
      // 1/|D_r|^2 recovered by multiplications).
      Real Dr_[R], Di_[R], inv_[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        CReal* t = tb + r * TS;
        Dr_[r] = t[TB_M2] - sc[r];
        Di_[r] = t[TB_NGE] * gc[r];
        inv_[r] = Dr_[r] * Dr_[r] + Di_[r] * Di_[r];
      }
      if constexpr (sizeof(Real) == 8 && R > 1) {
        Real pre[R];
        pre[0] = inv_[0];
#pragma unroll
        for (int r = 1; r < R; ++r) pre[r] = pre[r - 1] * inv_[r];
        Real q = rcp_r(pre[R - 1]);
#pragma unroll
        for (int r = R - 1; r > 0; --r) {
          const Real d2 = inv_[r];
          inv_[r] = q * pre[r - 1];
          q = q * d2;
        }
        inv_[0] = q;
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) inv_[r] = rcp_r(inv_[r]);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        CReal* t = tb + r * TS;
        const Real u = mad_nc(uc[r], t[TB_UMUL], t[TB_UADD]);
        const Real g = gc[r];
        const Real wr = Dr_[r] * inv_[r], wi = -Di_[r] * inv_[r];
        const Real uwr = u * wr, uwi = u * wi;
        if (r == 0) {
          zr = fma_r(t[TB_CBR], uwr, -t[TB_CBI] * uwi);
          zi = fma_r(t[TB_CBR], uwi, t[TB_CBI] * uwr);
        } else {
          zr = fma_r(t[TB_CBR], uwr, fma_r(-t[TB_CBI], uwi, zr));
          zi = fma_r(t[TB_CBR], uwi, fma_r(t[TB_CBI], uwr, zi));
        }
        if constexpr (ZD) {
          const Real uw2r = uwr * wr - uwi * wi, uw2i = uwr * wi + uwi * wr;
          const Real kr = mad_nc(t[TB_K3R], g, t[TB_K2R]);
          const Real ki = mad_nc(t[TB_K3I], g, t[TB_K2I]);
          if (r == 0) {
            zdr = fma_r(t[TB_K1R], uwr, fma_r(-t[TB_K1I], uwi, fma_r(kr, uw2r, -ki * uw2i)));
            zdi = fma_r(t[TB_K1R], uwi, fma_r(t[TB_K1I], uwr, fma_r(kr, uw2i, ki * uw2r)));
          } else {
            zdr = fma_r(t[TB_K1R], uwr, fma_r(-t[TB_K1I], uwi, fma_r(kr, uw2r, fma_r(-ki, uw2i, zdr))));
            zdi = fma_r(t[TB_K1R], uwi, fma_r(t[TB_K1I], uwr, fma_r(kr, uw2i, fma_r(ki, uw2r, zdi))));
          }
        }
        cwr[r] = wr;
        cwi[r] = wi;
        cu[r] = u;
      }
      // ---- exchange: every wave sums the G shares in group order.  Before
      // the barrier each wave also waits for its own loads of the next
      // batch, so that after it the whole next batch is in LDS.
      if constexpr (G > 1) {
        xch[buf][wv][0][lane][0] = zr;
        xch[buf][wv][0][lane][1] = zi;
        if constexpr (ZD) {
          xch[buf][wv][1][lane][0] = zdr;
          xch[buf][wv][1][lane][1] = zdi;
        }
      }
      wait_vm_at_most(nmine);
      lds_barrier();
      if constexpr (G > 1) {
        zr = xch[buf][0][0][lane][0];
        zi = xch[buf][0][0][lane][1];
        if constexpr (ZD) {
          zdr = xch[buf][0][1][lane][0];
          zdi = xch[buf][0][1][lane][1];
        }
#pragma unroll
        for (int g = 1; g < G; ++g) {
          // one share at a time (keeps the exchange's registers few)
          asm volatile("" ::: "memory");
          zr += xch[buf][g][0][lane][0];
          zi += xch[buf][g][0][lane][1];
          if constexpr (ZD) {
            zdr += xch[buf][g][1][lane][0];
            zdi += xch[buf][g][1][lane][1];
          }
        }
      }

      // ---- per-event weights (the data log is taken after pass 2, where
      // fewer registers are live)
      const Real om = zr * zr + zi * zi;
      Real gr = 0, gi = 0, alr = 0, ali = 0;
      double sterm = 0.0;
      if (rg.is_data) {
        if constexpr (DER) {
          const Real io = rcp_r(om);
          gr = zr * io;
          gi = -zi * io;
          if constexpr (ZD) {
            const Real t = 2 * (zr * zdr + zi * zdi) * io;
            alr = (zdr - t * zr) * io;
            ali = (t * zi - zdi) * io;
          }
        }
      } else {
        if (!BON) sterm = (double)om;
        gr = zr;
        gi = -zi;
        alr = zdr;
        ali = -zdi;
      }
      // only the last batch of a block can hold events past its range
      const bool dead = LAST && !(e0 + lane < rg.end);
      if (dead) gr = gi = alr = ali = 0;

      // ---- pass 2: moments (chain p = x u w, q = p w, r = q w)
      if constexpr (BON) {
        // B1..B3 = alpha u {w, w^2, g w^2}: the only moments that depend on
        // the direction v (C1..C6 depend on theta alone)
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const Real wr = cwr[r], wi = cwi[r], g = gc[r];
          const Real uwr = cu[r] * wr, uwi = cu[r] * wi;
          AccR* m = macc + NM * r;
          const Real ar_ = alr * uwr - ali * uwi, ai_ = alr * uwi + ali * uwr;
          const Real br_ = ar_ * wr - ai_ * wi, bi_ = ar_ * wi + ai_ * wr;
          acc_add(m[0], ar_);
          acc_add(m[1], ai_);
          acc_add(m[2], br_);
          acc_add(m[3], bi_);
          acc_fma(m[4], g, br_);
          acc_fma(m[5], g, bi_);
        }
      } else if constexpr (DER) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          // one resonance at a time: the scheduler may not interleave the
          // resonances' products (their temporaries would cost occupancy)
          __builtin_amdgcn_sched_barrier(0);
          const Real wr = cwr[r], wi = cwi[r], g = gc[r];
          const Real uwr = cu[r] * wr, uwi = cu[r] * wi;
          AccR* m = macc + NM * r;
          const Real pr = gr * uwr - gi * uwi, pi = gr * uwi + gi * uwr;
          const Real qr = pr * wr - pi * wi, qi = pr * wi + pi * wr;
          acc_add(m[0], pr);
          acc_add(m[1], pi);
          acc_add(m[2], qr);
          acc_add(m[3], qi);
          acc_fma(m[4], g, qr);
          acc_fma(m[5], g, qi);
          if constexpr (HVP) {
            const Real ar_ = alr * uwr - ali * uwi, ai_ = alr * uwi + ali * uwr;
            const Real br_ = ar_ * wr - ai_ * wi, bi_ = ar_ * wi + ai_ * wr;
            acc_add(m[6], ar_);
            acc_add(m[7], ai_);
            acc_add(m[8], br_);
            acc_add(m[9], bi_);
            acc_fma(m[10], g, br_);
            acc_fma(m[11], g, bi_);
            const Real rr = qr * wr - qi * wi, ri = qr * wi + qi * wr;
            const Real g2 = g * g;
            acc_add(m[12], rr);
            acc_add(m[13], ri);
            acc_fma(m[14], g, rr);
            acc_fma(m[15], g, ri);
            acc_fma(m[16], g2, rr);
            acc_fma(m[17], g2, ri);
          }
        }
      }
      if (!BON && wv == 0) {
        if (rg.is_data) sterm = (double)log_r(om);
        accS += dead ? 0.0 : sterm;
      }
      stage = (stage == NSTAGE - 1) ? 0 : stage + 1;
      buf ^= 1;
    };
    for (int b = 0; b < nbat - 1; ++b) {
      step(b, std::false_type{});
      if (RUN && (b % kRun) == kRun - 1) flush();
    }
    step(nbat - 1, std::true_type{});
    flush();
  }

  // ---- reduction: each wave owns its resonances, so a wave-level
  // butterfly (fixed order, symmetric) gives the block partial directly.
  const int K = a.K;
  const int V = 1 + NM * K;
  double* out = a.part + (int64_t)blockIdx.x * V * 2;
  if (wv == 0) {
    double hi = accS, lo = 0.0;
    dd_wave_reduce(hi, lo, 1);
    if (lane == 0) {
      out[0] = hi;
      out[1] = lo;
    }
  }
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    double x = acc[j];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) x += __shfl_xor(x, off);
    const int k = wv * R + j / NM;
    if (lane == 0 && k < K) {
      out[(1 + NM * k + j % NM) * 2] = x;
      out[(1 + NM * k + j % NM) * 2 + 1] = 0.0;
    }
  }
}

// ------------------------------------------------------------------------
// General physics path of the same pass (any Flatte resonance, or a spin-1
// parent).  Per resonance the width factor is complex, g + i h (h = 0 for a
// Breit-Wigner), so D = (M^2 - s - NGE h) + i NGE g, and each event carries
// nmu = 1 or 2 helicity amplitudes z^mu = sum_k c_k beta_k u_k^mu w_k with
// complex u^mu (eq. (1): w = sum_mu |z^mu|^2).  The moments keep their form
// with gamma u and alpha u replaced by P = sum_mu gamma^mu u^mu and
// Q = sum_mu alpha^mu u^mu, and g by the complex g + i h, so the finaliser
// is shared.  Wave-group layout as wg_kernel (G waves x R resonances, z^mu
// and zdot^mu exchanged through LDS, double buffered).  The stream of each
// batch is staged in LDS with the same 16-byte global-to-LDS loads as
// wg_kernel, in a single stage buffer (the stream has up to 55 planes here):
// the loads of batch b + 1 are issued once every wave has read batch b
// (after the exchange barrier) and are waited for before the barrier that
// opens batch b + 1, so they fly during the exchange and pass 2.
// ------------------------------------------------------------------------
template <typename Real, int MODE, int G, int R>
__global__ __launch_bounds__(64 * G) void wgx_kernel(EvalArgs a) {
  typedef typename CPtr<Real>::type CReal;
  constexpr bool HVP = (MODE == MODE_HVP);
  constexpr bool BON = (MODE == MODE_HVPB);
  constexpr bool ZD = HVP || BON;
  constexpr bool DER = (MODE != MODE_NLL);
  constexpr int NM = HVP ? NMOM_HVP : (DER ? NMOM_GRAD : 0);
  constexpr int NA = NM * R;
  constexpr int NQ = ZD ? 2 : 1;      // exchanged complex values per mu: z (, zdot)

  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const Range rg = block_range(a);
  const Real* __restrict__ planes = (const Real*)a.planes;
  const int64_t stride = a.stride;
  const int nmu = a.nmu;
  const Real* tsrc = ((sizeof(Real) == 8) ? (const Real*)a.tbl64 : (const Real*)a.tbl32) + wv * R * TS;
  constexpr int PPI = stage_ppi((int)sizeof(Real));   // planes per load instruction
  constexpr int LPP = 64 / PPI;                       // lanes per plane
  constexpr int JMAX = (stage_planes(MAX_GEN_FIELDS, (int)sizeof(Real)) / PPI + G - 1) / G;
  extern __shared__ __attribute__((aligned(16))) char stage_lds[];
  Real* stg = (Real*)stage_lds;   // nfp planes x 64 events (dynamic LDS)
  // z^mu (, zdot^mu) shares of the G waves; single buffered: the barrier
  // that opens the next batch follows every wave's reads of this one
  __shared__ Real xch[G][2][NQ][64][2];

  // LDS offsets (reals) of this wave's planes: s, g, h, u^0 (re, im), u^1 (re, im)
  int fo[R][7];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int* it = a.itbl + (wv * R + r) * ITS;
    const int sl[7] = {IT_S, IT_G, IT_H, IT_U, IT_UI, IT_U1R, IT_U1I};
#pragma unroll
    for (int f = 0; f < 7; ++f) fo[r][f] = it[sl[f]] * 64;
  }

  double accS = 0.0;
  double acc[NA > 0 ? NA : 1];
#pragma unroll
  for (int j = 0; j < NA; ++j) acc[j] = 0.0;

  const int nbat = (int)((rg.end - rg.begin + 63) / 64);
  const int nf = a.n_fields;
  const int ni = (nf + PPI - 1) / PPI;        // load instructions per batch
  // this wave's load instructions j = wv + G jj (the layout of wg_kernel:
  // lane l brings 16 bytes of plane j PPI + l / LPP at event (l % LPP) PPI;
  // in the last group, lanes past the last plane reload that plane into
  // padding slots that are never read)
  const uint32_t pbytes = (uint32_t)(stride * (int64_t)sizeof(Real));
  const uint32_t voff = (uint32_t)(lane / LPP) * pbytes + (uint32_t)(lane % LPP) * 16u;
  const uint32_t voff_last = (uint32_t)min(lane / LPP, nf - 1 - (ni - 1) * PPI) * pbytes +
                             (uint32_t)(lane % LPP) * 16u;
  const Real* bsrc = planes + rg.base + rg.begin;
  auto issue = [&](int b) {
    const int64_t off = (int64_t)b * 64;
#pragma unroll
    for (int jj = 0; jj < JMAX; ++jj) {
      const int j = wv + G * jj;
      if (j < ni) {
        const char* base = (const char*)(bsrc + (int64_t)j * PPI * stride + off);
        __builtin_amdgcn_global_load_lds((glob_void_t*)(base + (j == ni - 1 ? voff_last : voff)),
                                         (lds_void_t*)(stg + j * PPI * 64), 16, 0, 0);
      }
    }
  };
  if (nbat > 0) issue(0);

  for (int b = 0; b < nbat; ++b) {
    // batch b is in LDS: this wave's loads (vmcnt), then every wave's
    wait_vm_at_most(0);
    lds_barrier();
    const int64_t e0 = rg.begin + (int64_t)b * 64;
    const bool valid = e0 + lane < rg.end;
    CReal* tb = opaque_s((CReal*)tsrc);
    // ---- stream values of this wave's resonances; lanes past the range
    // (last batch only) hold the padding between the data and MC sets: give
    // them finite values, their contributions are zeroed below
    Real sv_[R], g_[R], h_[R], ur_[R][2], ui_[R][2];
    {
      const Real* sb = stg + lane;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        sv_[r] = valid ? sb[fo[r][0]] : Real(0);
        g_[r] = valid ? sb[fo[r][1]] : Real(0);
        h_[r] = valid ? sb[fo[r][2]] : Real(0);
        ur_[r][0] = valid ? sb[fo[r][3]] : Real(0);
        ui_[r][0] = valid ? sb[fo[r][4]] : Real(0);
        ur_[r][1] = (valid && nmu > 1) ? sb[fo[r][5]] : Real(0);
        ui_[r][1] = (valid && nmu > 1) ? sb[fo[r][6]] : Real(0);
      }
    }
    // ---- pass 1: w, u^mu of each resonance; this wave's share of z^mu, zdot^mu
    Real wr_[R], wi_[R];
    Real zr[2] = {0, 0}, zi[2] = {0, 0}, zdr[2] = {0, 0}, zdi[2] = {0, 0};
#pragma unroll
    for (int r = 0; r < R; ++r) {
      CReal* t = tb + r * TS;
      const Real sv = sv_[r];
      const Real Dr = t[TB_M2] - sv - t[TB_NGE] * h_[r];
      const Real Di = t[TB_NGE] * g_[r];
      const Real inv = rcp_r(Dr * Dr + Di * Di);
      wr_[r] = Dr * inv;
      wi_[r] = -Di * inv;
      // zdot coefficient K2 + K3 (g + i h)
      const Real kr = t[TB_K2R] + t[TB_K3R] * g_[r] - t[TB_K3I] * h_[r];
      const Real ki = t[TB_K2I] + t[TB_K3R] * h_[r] + t[TB_K3I] * g_[r];
#pragma unroll
      for (int mu = 0; mu < 2; ++mu) {
        if (mu >= nmu) break;
        const Real urr = mu == 0 ? mad_nc(ur_[r][0], t[TB_UMUL], t[TB_UADD]) : ur_[r][1];
        const Real uii = ui_[r][mu];
        ur_[r][mu] = urr;
        const Real Ur = urr * wr_[r] - uii * wi_[r], Ui = urr * wi_[r] + uii * wr_[r];
        zr[mu] += t[TB_CBR] * Ur - t[TB_CBI] * Ui;
        zi[mu] += t[TB_CBR] * Ui + t[TB_CBI] * Ur;
        if constexpr (ZD) {
          const Real Uwr = Ur * wr_[r] - Ui * wi_[r], Uwi = Ur * wi_[r] + Ui * wr_[r];
          zdr[mu] += t[TB_K1R] * Ur - t[TB_K1I] * Ui + kr * Uwr - ki * Uwi;
          zdi[mu] += t[TB_K1R] * Ui + t[TB_K1I] * Ur + kr * Uwi + ki * Uwr;
        }
      }
    }
    // ---- exchange
    if constexpr (G > 1) {
#pragma unroll
      for (int mu = 0; mu < 2; ++mu) {
        if (mu >= nmu) break;
        xch[wv][mu][0][lane][0] = zr[mu];
        xch[wv][mu][0][lane][1] = zi[mu];
        if constexpr (ZD) {
          xch[wv][mu][NQ - 1][lane][0] = zdr[mu];
          xch[wv][mu][NQ - 1][lane][1] = zdi[mu];
        }
      }
    }
    // every wave has read batch b's stream values (its LDS reads drained at
    // the barrier): refill the stage buffer with batch b + 1
    lds_barrier();
    if (b + 1 < nbat) issue(b + 1);
    if constexpr (G > 1) {
#pragma unroll
      for (int mu = 0; mu < 2; ++mu) {
        if (mu >= nmu) break;
        zr[mu] = zi[mu] = zdr[mu] = zdi[mu] = 0;
#pragma unroll
        for (int g = 0; g < G; ++g) {
          zr[mu] += xch[g][mu][0][lane][0];
          zi[mu] += xch[g][mu][0][lane][1];
          if constexpr (ZD) {
            zdr[mu] += xch[g][mu][NQ - 1][lane][0];
            zdi[mu] += xch[g][mu][NQ - 1][lane][1];
          }
        }
      }
    }
    // ---- per-event weights gamma^mu, alpha^mu
    Real om = 0, od = 0;
#pragma unroll
    for (int mu = 0; mu < 2; ++mu) {
      if (mu >= nmu) break;
      om += zr[mu] * zr[mu] + zi[mu] * zi[mu];
      od += zr[mu] * zdr[mu] + zi[mu] * zdi[mu];
    }
    Real gr[2] = {0, 0}, gi[2] = {0, 0}, alr[2] = {0, 0}, ali[2] = {0, 0};
    double sterm = 0.0;
    if (rg.is_data) {
      if (!BON && wv == 0) sterm = (double)log_r(om);
      if constexpr (DER) {
        const Real io = rcp_r(om);
        const Real tt = 2 * od * io;
#pragma unroll
        for (int mu = 0; mu < 2; ++mu) {
          gr[mu] = zr[mu] * io;
          gi[mu] = -zi[mu] * io;
          if constexpr (ZD) {
            alr[mu] = (zdr[mu] - tt * zr[mu]) * io;
            ali[mu] = (tt * zi[mu] - zdi[mu]) * io;
          }
        }
      }
    } else {
      if (!BON) sterm = (double)om;
#pragma unroll
      for (int mu = 0; mu < 2; ++mu) {
        gr[mu] = zr[mu];
        gi[mu] = -zi[mu];
        alr[mu] = zdr[mu];
        ali[mu] = -zdi[mu];
      }
    }
    if (!valid) {
      sterm = 0.0;
#pragma unroll
      for (int mu = 0; mu < 2; ++mu) gr[mu] = gi[mu] = alr[mu] = ali[mu] = 0;
    }
    if (wv == 0) accS += sterm;
    // ---- pass 2: P = sum gamma^mu u^mu, Q = sum alpha^mu u^mu, chain
    // p = P w, q = p w, r = q w (a = Q w, b = a w); complex g + i h
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const Real wr = wr_[r], wi = wi_[r], g = g_[r], hh = h_[r];
      Real Pr = 0, Pi = 0, Qr = 0, Qi = 0;
#pragma unroll
      for (int mu = 0; mu < 2; ++mu) {
        if (mu >= nmu) break;
        const Real ur = ur_[r][mu], ui = ui_[r][mu];
        Pr += gr[mu] * ur - gi[mu] * ui;
        Pi += gr[mu] * ui + gi[mu] * ur;
        Qr += alr[mu] * ur - ali[mu] * ui;
        Qi += alr[mu] * ui + ali[mu] * ur;
      }
      double* m = acc + NM * r;
      if constexpr (BON) {
        const Real ar_ = Qr * wr - Qi * wi, ai_ = Qr * wi + Qi * wr;
        const Real br_ = ar_ * wr - ai_ * wi, bi_ = ar_ * wi + ai_ * wr;
        acc_add(m[0], ar_);
        acc_add(m[1], ai_);
        acc_add(m[2], br_);
        acc_add(m[3], bi_);
        acc_add(m[4], g * br_ - hh * bi_);
        acc_add(m[5], g * bi_ + hh * br_);
      } else if constexpr (DER) {
        const Real pr = Pr * wr - Pi * wi, pi = Pr * wi + Pi * wr;
        const Real qr = pr * wr - pi * wi, qi = pr * wi + pi * wr;
        acc_add(m[0], pr);
        acc_add(m[1], pi);
        acc_add(m[2], qr);
        acc_add(m[3], qi);
        acc_add(m[4], g * qr - hh * qi);
        acc_add(m[5], g * qi + hh * qr);
        if constexpr (HVP) {
          const Real ar_ = Qr * wr - Qi * wi, ai_ = Qr * wi + Qi * wr;
          const Real br_ = ar_ * wr - ai_ * wi, bi_ = ar_ * wi + ai_ * wr;
          acc_add(m[6], ar_);
          acc_add(m[7], ai_);
          acc_add(m[8], br_);
          acc_add(m[9], bi_);
          acc_add(m[10], g * br_ - hh * bi_);
          acc_add(m[11], g * bi_ + hh * br_);
          const Real rr = qr * wr - qi * wi, ri = qr * wi + qi * wr;
          const Real g2r = g * g - hh * hh, g2i = 2 * g * hh;
          acc_add(m[12], rr);
          acc_add(m[13], ri);
          acc_add(m[14], g * rr - hh * ri);
          acc_add(m[15], g * ri + hh * rr);
          acc_add(m[16], g2r * rr - g2i * ri);
          acc_add(m[17], g2r * ri + g2i * rr);
        }
      }
    }
  }

  // ---- reduction (as wg_kernel)
  const int K = a.K;
  const int V = 1 + NM * K;
  double* out = a.part + (int64_t)blockIdx.x * V * 2;
  if (wv == 0) {
    double hi = accS, lo = 0.0;
    dd_wave_reduce(hi, lo, 1);
    if (lane == 0) {
      out[0] = hi;
      out[1] = lo;
    }
  }
#pragma unroll
  for (int j = 0; j < NA; ++j) {
    double x = acc[j];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) x += __shfl_xor(x, off);
    const int k = wv * R + j / NM;
    if (lane == 0 && k < K) {
      out[(1 + NM * k + j % NM) * 2] = x;
      out[(1 + NM * k + j % NM) * 2 + 1] = 0.0;
    }
  }
}

// ------------------------------------------------------------------------
// 3. Finaliser and combine (eq. (4), (6), (7) for NLL = -ln L).
// ------------------------------------------------------------------------
struct Cx {
  double r, i;
};
__device__ __forceinline__ Cx cx(double r, double i) { return {r, i}; }
__device__ __forceinline__ Cx operator+(Cx a, Cx b) { return {a.r + b.r, a.i + b.i}; }
__device__ __forceinline__ Cx operator*(Cx a, Cx b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ Cx operator*(double s, Cx a) { return {s * a.r, s * a.i}; }
__device__ __forceinline__ Cx mul_i(Cx a) { return {-a.i, a.r}; }

// Contract the moments of one resonance (mom: C1,C2,C3[,B1,B2,B3,C4,C5,C6]
// as doubles) with its table row: d/d(Re c, Im c, M, Gamma) of the event sum
// and (HVP) its Hessian times v, both including the factor 2 of
// d|z|^2 = 2 Re(conj(z) dz).
__device__ void contract(const double* mom, const double* t, bool hvp, double* dg, double* dh) {
  const Cx C1 = cx(mom[0], mom[1]), C2 = cx(mom[2], mom[3]), C3 = cx(mom[4], mom[5]);
  const double be = t[TB_BETA], be1 = t[TB_BETA1], bd = t[TB_BDOT], bd1 = t[TB_BDOT1];
  const Cx c = cx(t[TB_CR], t[TB_CI]), cd = cx(t[TB_VR], t[TB_VI]);
  const double twoM = t[TB_2M], nge1 = t[TB_NGE1], neta = t[TB_NETA];
  // dz/dM = c u (beta' w - beta (2M + i NGE1 g) w^2);  dz/dGamma = -i c beta NETA u g w^2
  const Cx XM = be1 * C1 + (-twoM * be) * C2 + mul_i((-be * nge1) * C3);
  const Cx XG = mul_i((-be * neta) * C3);
  dg[0] = 2.0 * be * C1.r;
  dg[1] = -2.0 * be * C1.i;
  dg[2] = 2.0 * (c * XM).r;
  dg[3] = 2.0 * (c * XG).r;
  if (!hvp) return;
  const Cx B1 = cx(mom[6], mom[7]), B2 = cx(mom[8], mom[9]), B3 = cx(mom[10], mom[11]);
  const Cx C4 = cx(mom[12], mom[13]), C5 = cx(mom[14], mom[15]), C6 = cx(mom[16], mom[17]);
  const double Ddr = t[TB_DDR], Ddig = t[TB_DDIG], dmd = t[TB_DMDDIG], dgd = t[TB_DGDDIG];
  const double vM = t[TB_VM];
  // Re c, Im c: alpha a + gamma adot
  const Cx Y = be * B1 + bd * C1 + (-be * Ddr) * C2 + mul_i((-be * Ddig) * C3);
  dh[0] = 2.0 * Y.r;
  dh[1] = -2.0 * Y.i;
  // M: alpha c aM + gamma (cdot aM + c adotM)
  const Cx BM = be1 * B1 + (-twoM * be) * B2 + mul_i((-be * nge1) * B3);
  const Cx ZM = bd1 * C1 + (-twoM * bd - be1 * Ddr - 2.0 * vM * be) * C2 +
                mul_i((-(bd * nge1 + be1 * Ddig + be * dmd)) * C3) + (2.0 * twoM * be * Ddr) * C4 +
                mul_i((2.0 * be * (Ddr * nge1 + twoM * Ddig)) * C5) + (-2.0 * be * Ddig * nge1) * C6;
  dh[2] = 2.0 * (c * BM + cd * XM + c * ZM).r;
  // Gamma: alpha c aG + gamma (cdot aG + c adotG)
  const Cx BG = mul_i((-be * neta) * B3);
  const Cx ZG = mul_i((-(bd * neta + be * dgd)) * C3) + mul_i((2.0 * be * neta * Ddr) * C5) +
                (-2.0 * be * neta * Ddig) * C6;
  dh[3] = 2.0 * (c * BG + cd * XG + c * ZG).r;
}

// Combine for one block: F, G (dd pairs), per-parameter derivative sums of
// both sets (plain doubles), direction v.
__device__ void combine_block(double F, double G, const double* dF, const double* dG,
                              const double* HF, const double* HG, int P, int mode, double nd,
                              double nm, const double* v, double* nll, double* grad, double* hv,
                              int* status) {
  __shared__ double sc[2];
  __shared__ double sv[4 * PWA_MAX_RES];
  const int tid = threadIdx.x;
  // the direction, staged in LDS by all threads (the sum below is serial)
  if (mode == MODE_HVP && v)
    for (int p = tid; p < P; p += blockDim.x) sv[p] = v[p];
  __syncthreads();
  if (tid == 0) {
    double val = -F + nd * log(G / nm);
    int flags = status ? status[0] : 0;
    if (!(G > 0.0) || !isfinite(val)) flags |= 2;
    if (flags) val = INFINITY;
    double dh = 0.0, dl = 0.0;
    if (mode == MODE_HVP && v) {
      for (int p = 0; p < P; ++p) {
        const double prod = dG[p] * sv[p];
        dd_add(dh, dl, prod, fma(dG[p], sv[p], -prod));
      }
    }
    sc[0] = dh + dl;
    if (nll) *nll = val;
    if (status) {
      status[0] = flags;
      if (flags) atomicOr(&status[1], flags);
    }
  }
  __syncthreads();
  if (mode == MODE_NLL) return;
  const double dGv = sc[0];
  const double wG = nd / G;
  for (int p = tid; p < P; p += blockDim.x) {
    if (grad) grad[p] = -dF[p] + wG * dG[p];
    if (mode == MODE_HVP && hv) hv[p] = -HF[p] + wG * HG[p] - (wG / G) * dG[p] * dGv;
  }
}

// Stage 1: fixed-order double-double sum of the block partials.  A block
// owns 16 value indices (blockIdx.x * 16 + (tid & 15); data values first,
// then MC values) and its 64 thread groups stride over the partial blocks,
// each with U independent accumulators; the groups are then combined by a
// fixed binary tree in LDS.  The order depends only on the grid, so the
// result is bitwise reproducible.
constexpr int RED_VALS = 16, RED_GROUPS = 64;
__global__ __launch_bounds__(1024) void reduce_kernel(FinalArgs f) {
  __shared__ double red[RED_GROUPS][RED_VALS][2];
  const int col = threadIdx.x % RED_VALS, grp = threadIdx.x / RED_VALS;
  const int vv = blockIdx.x * RED_VALS + col;
  double hi = 0.0, lo = 0.0;
  if (vv < 2 * f.V) {
    const int set = vv >= f.V;
    const int vi = vv - set * f.V;
    const int b0 = set ? f.nb_data : 0;
    const int nb = set ? f.nb_mc : f.nb_data;
    constexpr int U = 4;
    double h[U], l[U];
#pragma unroll
    for (int u = 0; u < U; ++u) h[u] = l[u] = 0.0;
    int b = grp;
    for (; b + RED_GROUPS * (U - 1) < nb; b += RED_GROUPS * U) {
      double qh[U], ql[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double* q = f.part + ((int64_t)(b0 + b + RED_GROUPS * u) * f.V + vi) * 2;
        qh[u] = q[0];
        ql[u] = q[1];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) dd_add(h[u], l[u], qh[u], ql[u]);
    }
    for (; b < nb; b += RED_GROUPS) {
      const double* q = f.part + ((int64_t)(b0 + b) * f.V + vi) * 2;
      dd_add(h[0], l[0], q[0], q[1]);
    }
    hi = h[0];
    lo = l[0];
#pragma unroll
    for (int u = 1; u < U; ++u) dd_add(hi, lo, h[u], l[u]);
  }
  red[grp][col][0] = hi;
  red[grp][col][1] = lo;
  __syncthreads();
#pragma unroll
  for (int half = RED_GROUPS / 2; half > 0; half >>= 1) {
    if (grp < half) {
      double a = red[grp][col][0], c = red[grp][col][1];
      dd_add(a, c, red[grp + half][col][0], red[grp + half][col][1]);
      red[grp][col][0] = a;
      red[grp][col][1] = c;
    }
    __syncthreads();
  }
  if (grp == 0 && vv < 2 * f.V) {
    hi = red[0][col][0];
    lo = red[0][col][1];
    int dst = vv;
    if (f.mode == MODE_HVPB) {
      // direction moments into their slots of the full HVP totals; the
      // theta-only values (S, C1..C6) there stay those of the last full pass
      const int set = vv >= f.V, vi = vv - set * f.V;
      if (vi == 0) return;
      const int k = (vi - 1) / NMOM_GRAD, i = (vi - 1) % NMOM_GRAD;
      dst = set * (1 + NMOM_HVP * f.K) + 1 + NMOM_HVP * k + NMOM_GRAD + i;
    }
    f.tot[2 * dst] = hi;
    f.tot[2 * dst + 1] = lo;
  }
}

// Stage 2 (one block): contraction of the moment totals with the resonance
// table, then the eq. (4)/(6)/(7) combine or the raw eq. (5) partials.
__global__ __launch_bounds__(1024) void final_kernel(FinalArgs f) {
  __shared__ double der[4][4 * PWA_MAX_RES];   // dF, dG, HF, HG
  const int tid = threadIdx.x;
  const double* tot = f.tot;
  const int K = f.K, P = 4 * K;
  const bool hvp = f.mode == MODE_HVP;
  const int NM = hvp ? NMOM_HVP : NMOM_GRAD;
  if (f.mode != MODE_NLL) {
    for (int q = tid; q < 2 * K; q += blockDim.x) {
      const int set = q / K, k = q % K;
      const double* src = tot + 2 * (set * f.V + 1 + NM * k);
      double mom[NMOM_HVP];
#pragma unroll
      for (int j = 0; j < NMOM_HVP; ++j) mom[j] = (j < NM) ? src[2 * j] + src[2 * j + 1] : 0.0;
      double dg[4], dh[4] = {0.0, 0.0, 0.0, 0.0};
      contract(mom, f.tbl + k * TS, hvp, dg, dh);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        der[set][4 * k + j] = dg[j];
        der[2 + set][4 * k + j] = dh[j];
      }
    }
  }
  __syncthreads();
  const double F = tot[0] + tot[1];
  const double G = tot[2 * f.V] + tot[2 * f.V + 1];
  if (f.out_kind == OUT_PARTIALS) {
    // [F, G, dF(P), dG(P), HFv(P), HGv(P)] as (hi, lo) pairs
    const int NOUT = 2 + 4 * P;
    for (int i = tid; i < NOUT; i += blockDim.x) {
      double h = 0.0, l = 0.0;
      if (i == 0) {
        h = tot[0];
        l = tot[1];
      } else if (i == 1) {
        h = tot[2 * f.V];
        l = tot[2 * f.V + 1];
      } else {
        const int q = i - 2, grp = q / P, p = q % P;
        const bool have = (grp < 2) ? (f.mode >= MODE_GRAD) : hvp;
        if (have) h = der[grp][p];
      }
      f.dd_out[2 * i] = h;
      f.dd_out[2 * i + 1] = l;
    }
    if (tid == 0 && f.status && f.status[0]) atomicOr(&f.status[1], f.status[0]);
    return;
  }
  combine_block(F, G, der[0], der[1], der[2], der[3], P, f.mode, f.n_data, f.n_mc, f.v, f.nll,
                f.grad, f.hv, f.status);
}

// pwa_combine: shard partials [F, G, dF, dG, HF, HG] (dd pairs), summed over
// shards in index order.
__global__ __launch_bounds__(1024) void combine_kernel(int P, int n_shards,
                                                       const double* __restrict__ parts,
                                                       double nd, double nm,
                                                       const double* __restrict__ v,
                                                       double* nll, double* grad, double* hv,
                                                       int* status) {
  __shared__ double tot[(2 + 4 * 4 * PWA_MAX_RES) * 2];
  __shared__ double flat[2 + 4 * 4 * PWA_MAX_RES];
  const int NOUT = 2 + 4 * P;
  for (int i = threadIdx.x; i < NOUT; i += blockDim.x) {
    double h = 0.0, l = 0.0;
    for (int s = 0; s < n_shards; ++s)
      dd_add(h, l, parts[((int64_t)s * NOUT + i) * 2], parts[((int64_t)s * NOUT + i) * 2 + 1]);
    tot[2 * i] = h;
    tot[2 * i + 1] = l;
    flat[i] = h + l;
  }
  if (threadIdx.x == 0 && status) status[0] = 0;
  __syncthreads();
  combine_block(tot[0] + tot[1], tot[2] + tot[3], flat + 2, flat + 2 + P, flat + 2 + 2 * P,
                flat + 2 + 3 * P, P, hv ? MODE_HVP : (grad ? MODE_GRAD : MODE_NLL), nd, nm, v,
                nll, grad, hv, status);
}

// ------------------------------------------------------------------------
// Per-event intensity omega(x) = |sum_k c_k beta_k u w_k|^2 (eq. (1)) of n
// bound events starting at `base`, one event per lane, table rows in
// resonance order.  Used to draw events from the model (accept-reject).
// ------------------------------------------------------------------------
template <typename Real>
__global__ __launch_bounds__(256) void intensity_kernel(const Real* __restrict__ planes,
                                                        int64_t stride, int64_t base, int64_t n,
                                                        const double* __restrict__ tbl,
                                                        const int* __restrict__ itbl, int K,
                                                        int gen, int nmu,
                                                        double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t e = base + i;
  auto at = [&](int k, int slot) -> double {
    return (double)planes[(int64_t)itbl[k * ITS + slot] * stride + e];
  };
  double zr[2] = {0.0, 0.0}, zi[2] = {0.0, 0.0};
  for (int k = 0; k < K; ++k) {
    const double* t = tbl + k * TS;
    const double s = at(k, IT_S), g = at(k, IT_G);
    const double h = gen ? at(k, IT_H) : 0.0;
    // D = (M^2 - s) - i Gamma eta (g + i h)
    const double Dr = t[TB_M2] - s - t[TB_NGE] * h, Di = t[TB_NGE] * g;
    const double inv = 1.0 / (Dr * Dr + Di * Di);
    const double wr = Dr * inv, wi = -Di * inv;
    for (int mu = 0; mu < nmu; ++mu) {
      const double ur = mu == 0 ? at(k, IT_U) * t[TB_UMUL] + t[TB_UADD] : at(k, IT_U1R);
      const double ui = gen ? (mu == 0 ? at(k, IT_UI) : at(k, IT_U1I)) : 0.0;
      const double uwr = ur * wr - ui * wi, uwi = ur * wi + ui * wr;
      zr[mu] += t[TB_CBR] * uwr - t[TB_CBI] * uwi;
      zi[mu] += t[TB_CBR] * uwi + t[TB_CBI] * uwr;
    }
  }
  double w = 0.0;
  for (int mu = 0; mu < nmu; ++mu) w += zr[mu] * zr[mu] + zi[mu] * zi[mu];
  out[i] = w;
}

// ------------------------------------------------------------------------
// Launchers and the table of built launch shapes.
// ------------------------------------------------------------------------
hipError_t launch_precompute(const double* s12, const double* s13, const double* cosb,
                             const double* gam, int64_t n, int64_t offset, void* planes,
                             int64_t stride, int is_f32, const ModelDev& md, const FieldSpec& fs,
                             hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((n + 255) / 256);
  if (is_f32)
    hipLaunchKernelGGL(precompute_kernel<float>, dim3(grid), dim3(256), 0, st, s12, s13, cosb, gam,
                       n, offset, (float*)planes, stride, md, fs);
  else
    hipLaunchKernelGGL(precompute_kernel<double>, dim3(grid), dim3(256), 0, st, s12, s13, cosb, gam,
                       n, offset, (double*)planes, stride, md, fs);
  return hipGetLastError();
}

hipError_t launch_intensity(bool f32, const void* planes, int64_t stride, int64_t base, int64_t n,
                            const double* tbl, const int* itbl, int K, int gen, int nmu,
                            double* out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((n + 255) / 256);
  if (f32)
    hipLaunchKernelGGL(intensity_kernel<float>, dim3(grid), dim3(256), 0, st, (const float*)planes,
                       stride, base, n, tbl, itbl, K, gen, nmu, out);
  else
    hipLaunchKernelGGL(intensity_kernel<double>, dim3(grid), dim3(256), 0, st,
                       (const double*)planes, stride, base, n, tbl, itbl, K, gen, nmu, out);
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
  X(1, 2) X(1, 4) X(2, 4) X(4, 2) X(4, 3) X(4, 4) X(8, 2) X(8, 4) X(16, 2) X(16, 4) X(32, 2)

// Wave-group shapes (waves per block G, resonances per wave R).
#define PWA_WG_SHAPES(X) X(1, 2) X(1, 4) X(2, 3) X(2, 4) X(3, 4) X(4, 2) X(4, 3) X(5, 3) X(6, 2) X(8, 2) X(8, 3) X(8, 4) X(12, 2) X(8, 8)

bool wg_shape_built(int G, int R) {
#define PWA_IS(GG, RR) if (G == GG && R == RR) return true;
  PWA_WG_SHAPES(PWA_IS)
#undef PWA_IS
  return false;
}

bool shape_built(int T, int R) {
#define PWA_IS(TT, RR) if (T == TT && R == RR) return true;
  PWA_SHAPES(PWA_IS)
#undef PWA_IS
  return false;
}

typedef void (*EvalFn)(EvalArgs);

static EvalFn eval_fn(int is_f32, int mode, int T, int R) {
#define PWA_PICK(TT, RR)                                                              \
  if (T == TT && R == RR) {                                                           \
    if (mode == MODE_NLL)                                                             \
      return is_f32 ? eval_kernel<float, MODE_NLL, TT, RR> : eval_kernel<double, MODE_NLL, TT, RR>;   \
    if (mode == MODE_GRAD)                                                            \
      return is_f32 ? eval_kernel<float, MODE_GRAD, TT, RR> : eval_kernel<double, MODE_GRAD, TT, RR>; \
    if (mode == MODE_HVPB)                                                            \
      return is_f32 ? eval_kernel<float, MODE_HVPB, TT, RR> : eval_kernel<double, MODE_HVPB, TT, RR>; \
    return is_f32 ? eval_kernel<float, MODE_HVP, TT, RR> : eval_kernel<double, MODE_HVP, TT, RR>;     \
  }
  PWA_SHAPES(PWA_PICK)
#undef PWA_PICK
  return nullptr;
}

// NLL-only shapes of layout 1 with one lane per event (no moment
// accumulators, so all K resonances fit in one lane).
#define PWA_NLL_SHAPES(X) X(8) X(12) X(16) X(24) X(32)

bool nll_shape_built(int R) {
#define PWA_IS(RR) if (R == RR) return true;
  PWA_NLL_SHAPES(PWA_IS)
#undef PWA_IS
  return false;
}

static EvalFn nll_fn(int is_f32, int R) {
#define PWA_PICK(RR) \
  if (R == RR) return is_f32 ? eval_kernel<float, MODE_NLL, 1, RR> : eval_kernel<double, MODE_NLL, 1, RR>;
  PWA_NLL_SHAPES(PWA_PICK)
#undef PWA_PICK
  return nullptr;
}

static EvalFn wg_fn(int is_f32, int mode, int G, int R) {
#define PWA_PICK(GG, RR)                                                              \
  if (G == GG && R == RR) {                                                           \
    if (mode == MODE_NLL)                                                             \
      return is_f32 ? wg_kernel<float, MODE_NLL, GG, RR> : wg_kernel<double, MODE_NLL, GG, RR>;   \
    if (mode == MODE_GRAD)                                                            \
      return is_f32 ? wg_kernel<float, MODE_GRAD, GG, RR> : wg_kernel<double, MODE_GRAD, GG, RR>; \
    if (mode == MODE_HVPB)                                                            \
      return is_f32 ? wg_kernel<float, MODE_HVPB, GG, RR> : wg_kernel<double, MODE_HVPB, GG, RR>; \
    return is_f32 ? wg_kernel<float, MODE_HVP, GG, RR> : wg_kernel<double, MODE_HVP, GG, RR>;     \
  }
  PWA_WG_SHAPES(PWA_PICK)
#undef PWA_PICK
  return nullptr;
}

// General physics path shapes (waves per block G, resonances per wave R).
#define PWA_GEN_SHAPES(X) X(1, 2) X(2, 2) X(4, 2) X(8, 2) X(4, 3)

bool gen_shape_built(int G, int R) {
#define PWA_IS(GG, RR) if (G == GG && R == RR) return true;
  PWA_GEN_SHAPES(PWA_IS)
#undef PWA_IS
  return false;
}

static EvalFn gen_fn(int is_f32, int mode, int G, int R) {
#define PWA_PICK(GG, RR)                                                              \
  if (G == GG && R == RR) {                                                           \
    if (mode == MODE_NLL)                                                             \
      return is_f32 ? wgx_kernel<float, MODE_NLL, GG, RR> : wgx_kernel<double, MODE_NLL, GG, RR>;   \
    if (mode == MODE_GRAD)                                                            \
      return is_f32 ? wgx_kernel<float, MODE_GRAD, GG, RR> : wgx_kernel<double, MODE_GRAD, GG, RR>; \
    if (mode == MODE_HVPB)                                                            \
      return is_f32 ? wgx_kernel<float, MODE_HVPB, GG, RR> : wgx_kernel<double, MODE_HVPB, GG, RR>; \
    return is_f32 ? wgx_kernel<float, MODE_HVP, GG, RR> : wgx_kernel<double, MODE_HVP, GG, RR>;     \
  }
  PWA_GEN_SHAPES(PWA_PICK)
#undef PWA_PICK
  return nullptr;
}

// layout 1: team (T lanes of a wave per event, 256-thread blocks);
// layout 2: wave group (G waves per 64 events, 64 G-thread blocks);
// layout 3: wave group of the general physics path.
static EvalFn pick_fn(int is_f32, int mode, int layout, int T, int R) {
  if (layout == 3) return gen_fn(is_f32, mode, T, R);
  if (layout == 2) return wg_fn(is_f32, mode, T, R);
  if (mode == MODE_NLL && T == 1 && nll_shape_built(R)) return nll_fn(is_f32, R);
  return eval_fn(is_f32, mode, T, R);
}

hipError_t launch_eval(int is_f32, int mode, int layout, int T, int R, const EvalArgs& a,
                       int nblocks, hipStream_t st) {
  EvalFn fn = pick_fn(is_f32, mode, layout, T, R);
  if (!fn) return hipErrorInvalidValue;
  if (layout == 3 && a.n_fields > MAX_GEN_FIELDS) return hipErrorInvalidValue;
  const size_t lds = pass_lds_bytes(layout, a.n_fields, is_f32 ? 4 : 8);
  hipLaunchKernelGGL(fn, dim3(nblocks), dim3(layout >= 2 ? 64 * T : BLOCK), lds, st, a);
  return hipGetLastError();
}

int eval_occupancy(int is_f32, int mode, int layout, int T, int R, int n_fields) {
  EvalFn fn = pick_fn(is_f32, mode, layout, T, R);
  if (!fn) return 0;
  int nb = 0;
  const size_t lds = pass_lds_bytes(layout, n_fields, is_f32 ? 4 : 8);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void*)fn, layout >= 2 ? 64 * T : BLOCK,
                                                   lds) != hipSuccess)
    return 0;
  return nb;
}

hipError_t launch_final(const FinalArgs& f, hipStream_t st) {
  const unsigned nb = (unsigned)((2 * f.V + RED_VALS - 1) / RED_VALS);
  hipLaunchKernelGGL(reduce_kernel, dim3(nb), dim3(1024), 0, st, f);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // a direction-only pass completes the full HVP totals: contract those
  FinalArgs g = f;
  if (f.mode == MODE_HVPB) {
    g.mode = MODE_HVP;
    g.V = 1 + NMOM_HVP * f.K;
  }
  hipLaunchKernelGGL(final_kernel, dim3(1), dim3(1024), 0, st, g);
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
