// Fixed-lineshape batched path (masses and widths frozen): many coupling
// vectors evaluated against one amplitude matrix, on the matrix cores.
//
// With M and Gamma fixed, the amplitude of every event is a fixed complex
// row a(x) = (a_1 .. a_K) (Sec. 2.2: "U" carries no free parameter and the
// couplings enter eq. (1) linearly), so for couplings c_b:
//   F_b = sum_data ln |A_D c_b|^2                       (a complex GEMM + log)
//   G_b = sum_MC |A_MC c_b|^2 = c_b^H Gm c_b,  Gm = A_MC^H A_MC   (eq. (1))
//   NLL_b = -F_b + N_D ln(G_b / N_MC)                   (eq. (3))
// The complex product is the real GEMM
//   [Zr | Zi] = [Ar | Ai] . [[Cr, Ci], [-Ci, Cr]]
// run on MFMA in the chosen operand format with FP32 accumulation (FP64 for
// the FP64 format).  The log epilogue is fused: Z never reaches memory.
// Per lane, the 4 rows of an MFMA result tile are combined as the product of
// their mantissas (one logarithm per 4 events) with the exponents summed as
// integers; per-start sums are FP64, reduced across blocks in double-double.
// The Gram matrix comes from FP64 MFMA over the event stream.

#include <math.h>

#include "pwa_batched.h"

namespace pwa {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef short s4_t __attribute__((ext_vector_type(4)));
typedef _Float16 h4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void dd_add_b(double& hi, double& lo, double bhi, double blo) {
  const double s = hi + bhi;
  const double bb = s - hi;
  double e = (hi - (s - bb)) + (bhi - bb);
  e += lo + blo;
  hi = s + e;
  lo = e - (hi - s);
}

__device__ __forceinline__ double rcp64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// ln of m in [1/16, 1) in single precision: m = f 2^e with f in
// [sqrt(1/2), sqrt(2)); ln f = 2 atanh(y) by its series through y^9
// (|y| <= 0.1716, truncation < 3e-9 relative); e ln 2 added in FP64.
__device__ __forceinline__ double ln_small(float m) {
  int e;
  float f = frexpf(m, &e);
  const bool lo = f < 0.70710678f;
  f = lo ? 2.0f * f : f;
  e = lo ? e - 1 : e;
  // y = (f - 1)/(f + 1): hardware reciprocal, then one correction of the
  // quotient from its exact residual (a Newton step on the reciprocal alone
  // leaves a one-signed error that would bias the log sum).
  const float fp1 = f + 1.0f, fm1 = f - 1.0f;
  const float r = __builtin_amdgcn_rcpf(fp1);
  const float y0 = fm1 * r;
  const float y = fmaf(fmaf(-y0, fp1, fm1), r, y0);
  const float y2 = y * y;
  float p = fmaf(y2, 1.0f / 9.0f, 1.0f / 7.0f);
  p = fmaf(p, y2, 1.0f / 5.0f);
  p = fmaf(p, y2, 1.0f / 3.0f);
  const float s = fmaf(2.0f * y * y2, p, 2.0f * y);
  return fma((double)e, 0.69314718055994530942, (double)s);
}

// ln of m in [1/16, 1) in double precision (FP64 format): same series
// through y^21.
__device__ __forceinline__ double ln_small64(double m) {
  int e;
  double f = frexp(m, &e);
  const bool lo = f < 0.70710678118654752440;
  f = lo ? 2.0 * f : f;
  e = lo ? e - 1 : e;
  const double y = (f - 1.0) * rcp64(f + 1.0);
  const double y2 = y * y;
  double p = 1.0 / 21.0;
  p = fma(p, y2, 1.0 / 19.0);
  p = fma(p, y2, 1.0 / 17.0);
  p = fma(p, y2, 1.0 / 15.0);
  p = fma(p, y2, 1.0 / 13.0);
  p = fma(p, y2, 1.0 / 11.0);
  p = fma(p, y2, 1.0 / 9.0);
  p = fma(p, y2, 1.0 / 7.0);
  p = fma(p, y2, 1.0 / 5.0);
  p = fma(p, y2, 1.0 / 3.0);
  const double t = 2.0 * y;
  const double de = (double)e;
  return fma(de, 6.93147180369123816490e-01, fma(de, 1.90821492927058770002e-10, fma(t * y2, p, t)));
}

// ------------------------------------------------------------------------
// Amplitude rows a_k(x) = beta_k u w for frozen (M, Gamma) from the FP64 event
// stream, written as [Re a_0..Re a_{K-1}, Im a_0..Im a_{K-1}, 0 pad] rows of
// KP operands.  For the split format, lo = fp16(a - hi) goes to a second plane.
// ------------------------------------------------------------------------
template <int FMT>
__global__ __launch_bounds__(256) void freeze_kernel(const double* __restrict__ planes, int64_t stride,
                                                     int64_t n, const double* __restrict__ tbl,
                                                     const int* __restrict__ itbl, int K, int KP,
                                                     int gen, void* out_hi, void* out_lo) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int c = 0; c < KP; ++c) {
    double v = 0.0;
    if (c < 2 * K) {
      const int k = c < K ? c : c - K;
      const double* t = tbl + k * TS;
      const double s = planes[(int64_t)itbl[k * ITS + 0] * stride + i];
      const double u = planes[(int64_t)itbl[k * ITS + 1] * stride + i] * t[TB_UMUL] + t[TB_UADD];
      const double g = planes[(int64_t)itbl[k * ITS + 2] * stride + i];
      // Flatte resonances (general path): complex width factor g + i h
      const double h = gen ? planes[(int64_t)itbl[k * ITS + IT_H] * stride + i] : 0.0;
      const double Dr = t[TB_M2] - s - t[TB_NGE] * h, Di = t[TB_NGE] * g;
      const double bu = t[TB_BETA] * u * rcp64(Dr * Dr + Di * Di);
      v = (c < K) ? bu * Dr : -bu * Di;
    }
    const int64_t o = i * KP + c;
    if constexpr (FMT == PWA_OP_F64) {
      ((double*)out_hi)[o] = v;
    } else if constexpr (FMT == PWA_OP_F32) {
      ((float*)out_hi)[o] = (float)v;
    } else if constexpr (FMT == PWA_OP_BF16) {
      ((__bf16*)out_hi)[o] = (__bf16)(float)v;
    } else {
      const _Float16 h = (_Float16)v;
      ((_Float16*)out_hi)[o] = h;
      if constexpr (FMT == PWA_OP_F16X3) ((_Float16*)out_lo)[o] = (_Float16)(v - (double)h);
    }
  }
}

// Power-of-two column scale of the split FP16 format: start b's couplings are
// multiplied by 2^shift so that their largest real component lies in
// [2^10, 2^11); the three FP16 parts of every component then stay in the
// normal FP16 range.  Z scales by 2^shift and ln |Z|^2 by 2 shift ln 2, which
// the final kernel removes exactly.
__device__ __forceinline__ int col_shift(const double* __restrict__ C, int K, int b) {
  double m = 0.0;
  for (int k = 0; k < K; ++k) m = fmax(m, fmax(fabs(C[2 * (b * K + k)]), fabs(C[2 * (b * K + k) + 1])));
  if (!(m > 0.0) || !isfinite(m)) return 0;
  int e;
  frexp(m, &e);   // m < 2^e
  return 11 - e;
}

// Expanded coupling block [[Cr, Ci], [-Ci, Cr]] as KP x 2B operands, column
// b (< B) = real part of start b, column B + b = imaginary part.  The
// couplings enter every event's sum coherently, so a rounding of C biases
// all N_D logarithms alike (the error grows like N_D times the gradient);
// the accurate formats therefore carry C as a sum of parts: FP32 hi + lo,
// or three FP16 parts (with the column scale above) for the split format.
template <int FMT>
__global__ void coupling_kernel(const double* __restrict__ C, int K, int KP, int B, void* out_hi,
                                void* out_lo, void* out_lo2) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= KP * 2 * B) return;
  const int row = idx / (2 * B), col = idx % (2 * B);
  const int b = col < B ? col : col - B;
  const bool imag_col = col >= B;
  double v = 0.0;
  if (row < 2 * K) {
    const int k = row < K ? row : row - K;
    const double cr = C[2 * (b * K + k)], ci = C[2 * (b * K + k) + 1];
    if (row < K) v = imag_col ? ci : cr;
    else v = imag_col ? cr : -ci;
  }
  if constexpr (FMT == PWA_OP_F64) {
    ((double*)out_hi)[idx] = v;
  } else if constexpr (FMT == PWA_OP_F32) {
    const float h = (float)v;
    ((float*)out_hi)[idx] = h;
    ((float*)out_lo)[idx] = (float)(v - (double)h);
  } else if constexpr (FMT == PWA_OP_BF16) {
    ((__bf16*)out_hi)[idx] = (__bf16)(float)v;
  } else if constexpr (FMT == PWA_OP_F16) {
    ((_Float16*)out_hi)[idx] = (_Float16)v;
  } else {
    v = ldexp(v, col_shift(C, K, b));
    const _Float16 h = (_Float16)v;
    const double r = v - (double)h;
    const _Float16 l = (_Float16)r;
    ((_Float16*)out_hi)[idx] = h;
    ((_Float16*)out_lo)[idx] = l;
    ((_Float16*)out_lo2)[idx] = (_Float16)(r - (double)l);
  }
}

// ------------------------------------------------------------------------
// Batched data term.  Grid: (row blocks, column chunks of CHB starts).
// Wave w of a block takes 16 rows at a time; for each of the chunk's CHB/16
// start tiles it forms the real and the imaginary 16 x 16 tile of Z with
// MFMA over the KP operands, then folds |Z|^2 of its 4 rows into the
// per-start log sums.
// MFMA operand layouts (checked on gfx950): A lane l = row l%16, k-group
// l/16; B lane l = k-group l/16, column l%16.  Result: lane l holds column
// l%16, rows 4 (l/16) + r (FP32 results) or 4 r + l/16 (FP64 results),
// r = 0..3.
// ------------------------------------------------------------------------
// Number of coupling parts per format (see coupling_kernel).
__host__ __device__ constexpr int c_parts(int fmt) {
  return fmt == PWA_OP_F32 ? 2 : (fmt == PWA_OP_F16X3 ? 3 : 1);
}

template <int FMT> struct Mma;
template <> struct Mma<PWA_OP_F64> {
  static constexpr int KSTEP = 4, E = 1;
  typedef double T;
  typedef double op_t;
  typedef d4_t acc_t;
  __device__ static acc_t mma(op_t a, op_t b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
};
template <> struct Mma<PWA_OP_F32> {
  static constexpr int KSTEP = 4, E = 1;
  typedef float T;
  typedef float op_t;
  typedef f4_t acc_t;
  __device__ static acc_t mma(op_t a, op_t b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};
template <> struct Mma<PWA_OP_BF16> {
  static constexpr int KSTEP = 16, E = 4;
  typedef __bf16 T;
  typedef s4_t op_t;
  typedef f4_t acc_t;
  __device__ static acc_t mma(op_t a, op_t b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }
};
template <> struct Mma<PWA_OP_F16> {
  static constexpr int KSTEP = 16, E = 4;
  typedef _Float16 T;
  typedef h4_t op_t;
  typedef f4_t acc_t;
  __device__ static acc_t mma(op_t a, op_t b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0); }
};
template <> struct Mma<PWA_OP_F16X3> : Mma<PWA_OP_F16> {};

template <int FMT>
__device__ __forceinline__ typename Mma<FMT>::op_t load_op(const void* base, int64_t off) {
  typedef typename Mma<FMT>::op_t op_t;
  if constexpr (Mma<FMT>::E == 1) {
    return ((const op_t*)base)[off];
  } else {
    op_t v;   // 4 contiguous 16-bit values (8-byte aligned: off is a multiple of 4)
    __builtin_memcpy(&v, (const typename Mma<FMT>::T*)base + off, sizeof(op_t));
    return v;
  }
}

template <int FMT, int CHB, int NKS>
__global__ __launch_bounds__(256) void batched_kernel(BatchArgs a) {
  typedef Mma<FMT> M;
  typedef typename M::op_t op_t;
  typedef typename M::acc_t acc_t;
  typedef typename M::T T;
  constexpr int NT = CHB / 16;             // start tiles per chunk
  constexpr int KP = NKS * M::KSTEP;       // padded real inner dimension
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int B = a.B;
  const int b0 = blockIdx.y * CHB;
  // stage this chunk's coupling columns (real: b0.., imag: B + b0..) in LDS
  extern __shared__ char smem_raw[];
  T* sC = (T*)smem_raw;                        // c_parts(FMT) planes of [2][KP][CHB]
  constexpr int NCP = c_parts(FMT);
  const int plane = 2 * KP * CHB;
  for (int i = threadIdx.x; i < plane; i += blockDim.x) {
    const int part = i / (KP * CHB), rem = i % (KP * CHB), row = rem / CHB, col = rem % CHB;
    const int64_t g = (int64_t)row * 2 * B + (part ? B : 0) + b0 + col;
    sC[i] = ((const T*)a.C_hi)[g];
    if constexpr (NCP > 1) sC[plane + i] = ((const T*)a.C_lo)[g];
    if constexpr (NCP > 2) sC[2 * plane + i] = ((const T*)a.C_lo2)[g];
  }
  __syncthreads();
  // B operands (real and imaginary column) of one coupling part from LDS
  auto load_b = [&](const T* src, int ro, op_t& br, op_t& bi) {
    if constexpr (M::E == 1) {
      br = src[ro];
      bi = src[KP * CHB + ro];
    } else {
      T tr[4], ti[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        tr[e] = src[ro + e * CHB];
        ti[e] = src[KP * CHB + ro + e * CHB];
      }
      __builtin_memcpy(&br, tr, sizeof(op_t));
      __builtin_memcpy(&bi, ti, sizeof(op_t));
    }
  };

  const int64_t rows_per_block = (a.n + gridDim.x - 1) / gridDim.x;
  const int64_t r_begin = min(a.n, (int64_t)blockIdx.x * rows_per_block);
  const int64_t r_end = min(a.n, r_begin + rows_per_block);
  double accL[NT];
  int accE[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    accL[t] = 0.0;
    accE[t] = 0;
  }
  const int col = lane & 15, kg = lane >> 4;
  for (int64_t r0 = r_begin + 16 * wave; r0 < r_end; r0 += 64) {
    // A operands of rows r0 .. r0 + 15 (row l % 16, k-group l / 16)
    const int64_t row = min(r0 + col, a.n - 1);
    op_t ah[NKS], al[FMT == PWA_OP_F16X3 ? NKS : 1];
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      ah[ks] = load_op<FMT>(a.A_hi, row * KP + ks * M::KSTEP + kg * M::E);
      if constexpr (FMT == PWA_OP_F16X3) al[ks] = load_op<FMT>(a.A_lo, row * KP + ks * M::KSTEP + kg * M::E);
    }
    // rows held by this lane in the result tile
    bool valid[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      valid[q] = (r0 + (FMT == PWA_OP_F64 ? 4 * q + kg : 4 * kg + q)) < r_end;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      acc_t zr = {0, 0, 0, 0}, zi = {0, 0, 0, 0};
      // Accumulate the products smallest-first over the whole inner
      // dimension: the low parts of C (and A) carry a systematic correction
      // of relative size 2^-22 .. 2^-24; added step by step to an accumulator
      // that already holds the large partial sums they would fall below half
      // an ulp and be dropped every time.
      if constexpr (NCP > 2) {
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
          const int ro = (ks * M::KSTEP + kg * M::E) * CHB + t * 16 + col;
          op_t br, bi;
          load_b(sC + 2 * plane, ro, br, bi);
          zr = M::mma(ah[ks], br, zr);
          zi = M::mma(ah[ks], bi, zi);
        }
      }
      if constexpr (FMT == PWA_OP_F16X3) {
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
          const int ro = (ks * M::KSTEP + kg * M::E) * CHB + t * 16 + col;
          op_t br, bi;
          load_b(sC, ro, br, bi);
          zr = M::mma(al[ks], br, zr);
          zi = M::mma(al[ks], bi, zi);
        }
      }
      if constexpr (NCP > 1) {
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
          const int ro = (ks * M::KSTEP + kg * M::E) * CHB + t * 16 + col;
          op_t br, bi;
          load_b(sC + plane, ro, br, bi);
          zr = M::mma(ah[ks], br, zr);
          zi = M::mma(ah[ks], bi, zi);
        }
      }
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
        const int ro = (ks * M::KSTEP + kg * M::E) * CHB + t * 16 + col;
        op_t br, bi;
        load_b(sC, ro, br, bi);
        zr = M::mma(ah[ks], br, zr);
        zi = M::mma(ah[ks], bi, zi);
      }
      // epilogue: product of the 4 mantissas, exponents summed
      if constexpr (FMT == PWA_OP_F64) {
        double prod = 1.0;
        int es = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double om = valid[q] ? zr[q] * zr[q] + zi[q] * zi[q] : 1.0;
          int e;
          prod *= frexp(om, &e);
          es += e;
        }
        accL[t] += ln_small64(prod);
        accE[t] += es;
      } else {
        float prod = 1.0f;
        int es = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float om = valid[q] ? zr[q] * zr[q] + zi[q] * zi[q] : 1.0f;
          int e;
          prod *= frexpf(om, &e);
          es += e;
        }
        accL[t] += ln_small(prod);
        accE[t] += es;
      }
    }
  }
  // reduce the 4 k-groups (lanes col, col+16, col+32, col+48) and the 4 waves
  __shared__ double red[4][CHB][2];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    double hi = accL[t] + (double)accE[t] * 6.93147180369123816490e-01;
    double lo = (double)accE[t] * 1.90821492927058770002e-10;
    for (int off = 16; off < 64; off <<= 1) {
      const double oh = __shfl_xor(hi, off), ol = __shfl_xor(lo, off);
      dd_add_b(hi, lo, oh, ol);
    }
    if (kg == 0) {
      red[wave][t * 16 + col][0] = hi;
      red[wave][t * 16 + col][1] = lo;
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < CHB; b += blockDim.x) {
    double h = red[0][b][0], l = red[0][b][1];
    for (int w = 1; w < 4; ++w) dd_add_b(h, l, red[w][b][0], red[w][b][1]);
    if (b0 + b < B) {
      a.part[((int64_t)blockIdx.x * B + b0 + b) * 2] = h;
      a.part[((int64_t)blockIdx.x * B + b0 + b) * 2 + 1] = l;
    }
  }
}

// ------------------------------------------------------------------------
// Gram matrix of the MC amplitudes with FP64 MFMA: X = [Ar | Ai] (events x
// 2K, padded to 48), XtX += X^T X per block, then Gm from XtX.  Each wave
// stages 16 event rows of X in LDS, computed in FP64 from the stream.
// ------------------------------------------------------------------------
constexpr int GP = 48;   // padded 2K (K <= 24 on this path)

__global__ __launch_bounds__(256) void gram_kernel(const double* __restrict__ planes, int64_t stride,
                                                   int64_t base, int64_t n,
                                                   const double* __restrict__ tbl,
                                                   const int* __restrict__ itbl, int K, int gen,
                                                   double* __restrict__ part) {
  __shared__ double X[4][16][GP];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t per_block = (n + gridDim.x - 1) / gridDim.x;
  const int64_t e_begin = min(n, (int64_t)blockIdx.x * per_block);
  const int64_t e_end = min(n, e_begin + per_block);
  d4_t acc[3][3];
#pragma unroll
  for (int I = 0; I < 3; ++I)
#pragma unroll
    for (int J = 0; J < 3; ++J) acc[I][J] = (d4_t){0, 0, 0, 0};
  const int col = lane & 15, kg = lane >> 4;
  for (int64_t e0 = e_begin; e0 < e_end; e0 += 64) {   // same trip count in every wave
    // lane l computes features of event e0 + 16 wave + l % 16, resonances kg, kg + 4, ...
    const int64_t ev = e0 + 16 * wave + col;
    const bool valid = ev < e_end;
    for (int k = kg; k < GP / 2; k += 4) {
      double re = 0.0, im = 0.0;
      if (valid && k < K) {
        const double* t = tbl + k * TS;
        const int64_t x = base + ev;
        const double s = planes[(int64_t)itbl[k * ITS + 0] * stride + x];
        const double u = planes[(int64_t)itbl[k * ITS + 1] * stride + x] * t[TB_UMUL] + t[TB_UADD];
        const double g = planes[(int64_t)itbl[k * ITS + 2] * stride + x];
        const double h = gen ? planes[(int64_t)itbl[k * ITS + IT_H] * stride + x] : 0.0;
        const double Dr = t[TB_M2] - s - t[TB_NGE] * h, Di = t[TB_NGE] * g;
        const double bu = t[TB_BETA] * u * rcp64(Dr * Dr + Di * Di);
        re = bu * Dr;
        im = -bu * Di;
      }
      if (k < K) {
        X[wave][col][k] = re;
        X[wave][col][K + k] = im;
      }
    }
    for (int c = 2 * K + kg; c < GP; c += 4) X[wave][col][c] = 0.0;
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {   // 4 events per MFMA step
#pragma unroll
      for (int I = 0; I < 3; ++I) {
        const double av = X[wave][4 * ks + kg][16 * I + col];   // (X^T)[16 I + col][event]
#pragma unroll
        for (int J = 0; J < 3; ++J) {
          const double bv = X[wave][4 * ks + kg][16 * J + col];
          acc[I][J] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[I][J], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // block partial of X^T X: combine the 4 waves in order through LDS
  __shared__ double red[4][GP][GP];
#pragma unroll
  for (int I = 0; I < 3; ++I)
#pragma unroll
    for (int J = 0; J < 3; ++J)
#pragma unroll
      for (int q = 0; q < 4; ++q) red[wave][16 * I + 4 * q + kg][16 * J + col] = acc[I][J][q];
  __syncthreads();
  for (int i = threadIdx.x; i < GP * GP; i += blockDim.x) {
    const int r = i / GP, c = i % GP;
    double h = red[0][r][c], l = 0.0;
    for (int w = 1; w < 4; ++w) dd_add_b(h, l, red[w][r][c], 0.0);
    part[((int64_t)blockIdx.x * GP * GP + i) * 2] = h;
    part[((int64_t)blockIdx.x * GP * GP + i) * 2 + 1] = l;
  }
}

// Sum the per-block X^T X in block order and form Gm[k][l] (complex):
//   Re = XtX[k][l] + XtX[K+k][K+l],  Im = XtX[k][K+l] - XtX[K+k][l].
__global__ void gram_final_kernel(const double* __restrict__ part, int nblocks, int K,
                                  double* __restrict__ gram) {
  __shared__ double xtx[GP * GP];
  for (int i = threadIdx.x; i < GP * GP; i += blockDim.x) {
    double h = 0.0, l = 0.0;
    for (int b = 0; b < nblocks; ++b)
      dd_add_b(h, l, part[((int64_t)b * GP * GP + i) * 2], part[((int64_t)b * GP * GP + i) * 2 + 1]);
    xtx[i] = h + l;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < K * K; i += blockDim.x) {
    const int k = i / K, l = i % K;
    gram[2 * i] = xtx[k * GP + l] + xtx[(K + k) * GP + K + l];
    gram[2 * i + 1] = xtx[k * GP + K + l] - xtx[(K + k) * GP + l];
  }
}

// Per-start sum of the row-block partials in two fixed-order stages.  Stage
// 1: block (x, c) adds rows c*rpc .. of starts 64x .. 64x+63 (one start per
// lane, coalesced over starts).
__global__ __launch_bounds__(64) void batched_rowsum_kernel(const double* __restrict__ part,
                                                           int nblocks, int B,
                                                           double* __restrict__ part2) {
  const int b = blockIdx.x * 64 + threadIdx.x;
  if (b >= B) return;
  const int rpc = (nblocks + kBatchChunks - 1) / kBatchChunks;
  const int r0 = blockIdx.y * rpc, r1 = min(nblocks, r0 + rpc);
  double h = 0.0, l = 0.0;
  for (int r = r0; r < r1; ++r)
    dd_add_b(h, l, part[((int64_t)r * B + b) * 2], part[((int64_t)r * B + b) * 2 + 1]);
  part2[((int64_t)blockIdx.y * B + b) * 2] = h;
  part2[((int64_t)blockIdx.y * B + b) * 2 + 1] = l;
}

// Stage 2 and the likelihood: F_b from the chunk partials in order
// (double-double), less the column scale of the split format, G_b by the
// quadratic form in FP64, NLL_b = -F_b + N_D ln(c_b^H Gm c_b / N_MC).
__global__ void batched_final_kernel(const double* __restrict__ part2, int B, int K,
                                     const double* __restrict__ C, const double* __restrict__ gram,
                                     double nd, double nm, int scaled, double* __restrict__ nll) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double h = 0.0, l = 0.0;
  for (int c = 0; c < kBatchChunks; ++c)
    dd_add_b(h, l, part2[((int64_t)c * B + b) * 2], part2[((int64_t)c * B + b) * 2 + 1]);
  if (scaled) {   // remove N_D * 2 shift ln 2 (an exact integer times ln 2 in two parts)
    const double m = -2.0 * nd * (double)col_shift(C, K, b);
    dd_add_b(h, l, m * 6.93147180369123816490e-01, m * 1.90821492927058770002e-10);
  }
  const double F = h + l;
  double G = 0.0;
  for (int k = 0; k < K; ++k) {
    const double ckr = C[2 * (b * K + k)], cki = C[2 * (b * K + k) + 1];
    double sr = 0.0, si = 0.0;   // (Gm c)_k
    for (int j = 0; j < K; ++j) {
      const double gr = gram[2 * (k * K + j)], gi = gram[2 * (k * K + j) + 1];
      const double cr = C[2 * (b * K + j)], ci = C[2 * (b * K + j) + 1];
      sr += gr * cr - gi * ci;
      si += gr * ci + gi * cr;
    }
    G += ckr * sr + cki * si;    // Re(conj(c_k) (Gm c)_k)
  }
  double val = -F + nd * log(G / nm);
  if (!(G > 0.0) || !isfinite(val)) val = INFINITY;
  nll[b] = val;
}

// ------------------------------------------------------------------------
// Launchers.
// ------------------------------------------------------------------------
// Padded real inner dimension: a multiple of 8 (FP64/FP32, 4-deep MFMA
// steps, built for 2 to 12 steps) or of 16 (16-bit formats, 1 to 3 steps).
int batched_kp(int fmt, int K) {
  if (fmt == PWA_OP_F64 || fmt == PWA_OP_F32) return (2 * K + 7) / 8 * 8;
  return (2 * K + 15) / 16 * 16;
}
int batched_elem_bytes(int fmt) { return fmt == PWA_OP_F64 ? 8 : (fmt == PWA_OP_F32 ? 4 : 2); }

hipError_t launch_freeze(int fmt, const double* planes, int64_t stride, int64_t n,
                         const double* tbl, const int* itbl, int K, int KP, int gen, void* out_hi,
                         void* out_lo, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((n + 255) / 256);
#define PWA_FZ(F) hipLaunchKernelGGL(freeze_kernel<F>, dim3(grid), dim3(256), 0, st, planes, stride, n, tbl, itbl, K, KP, gen, out_hi, out_lo)
  switch (fmt) {
    case PWA_OP_F64: PWA_FZ(PWA_OP_F64); break;
    case PWA_OP_F32: PWA_FZ(PWA_OP_F32); break;
    case PWA_OP_BF16: PWA_FZ(PWA_OP_BF16); break;
    case PWA_OP_F16: PWA_FZ(PWA_OP_F16); break;
    default: PWA_FZ(PWA_OP_F16X3); break;
  }
#undef PWA_FZ
  return hipGetLastError();
}

hipError_t launch_gram(const double* planes, int64_t stride, int64_t base, int64_t n,
                       const double* tbl, const int* itbl, int K, int gen, int nblocks, double* part,
                       double* gram, hipStream_t st) {
  hipLaunchKernelGGL(gram_kernel, dim3(nblocks), dim3(256), 0, st, planes, stride, base, n, tbl,
                     itbl, K, gen, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gram_final_kernel, dim3(1), dim3(1024), 0, st, part, nblocks, K, gram);
  return hipGetLastError();
}

hipError_t launch_batched(int fmt, const BatchArgs& a, int row_blocks, const double* C,
                          const double* gram, int K, double nd, double nm, double* nll,
                          hipStream_t st) {
  const unsigned cg = (unsigned)((a.KP * 2 * a.B + 255) / 256);
#define PWA_CP(F) hipLaunchKernelGGL(coupling_kernel<F>, dim3(cg), dim3(256), 0, st, C, K, a.KP, a.B, (void*)a.C_hi, (void*)a.C_lo, (void*)a.C_lo2)
  switch (fmt) {
    case PWA_OP_F64: PWA_CP(PWA_OP_F64); break;
    case PWA_OP_F32: PWA_CP(PWA_OP_F32); break;
    case PWA_OP_BF16: PWA_CP(PWA_OP_BF16); break;
    case PWA_OP_F16: PWA_CP(PWA_OP_F16); break;
    default: PWA_CP(PWA_OP_F16X3); break;
  }
#undef PWA_CP
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  constexpr int CHB = 64;
  const dim3 grid(row_blocks, (a.B + CHB - 1) / CHB);
  const size_t lds = (size_t)2 * a.KP * CHB * batched_elem_bytes(fmt) * c_parts(fmt);
  const bool wide = (fmt == PWA_OP_F64 || fmt == PWA_OP_F32);
  const int nks = a.KP / (wide ? 4 : 16);
#define PWA_BK(F, N) hipLaunchKernelGGL((batched_kernel<F, CHB, N>), grid, dim3(256), lds, st, a)
#define PWA_WIDE(F)                      \
  switch (nks) {                         \
    case 2: PWA_BK(F, 2); break;         \
    case 4: PWA_BK(F, 4); break;         \
    case 6: PWA_BK(F, 6); break;         \
    case 8: PWA_BK(F, 8); break;         \
    case 10: PWA_BK(F, 10); break;       \
    default: PWA_BK(F, 12); break;       \
  }
#define PWA_NARROW(F)                    \
  switch (nks) {                         \
    case 1: PWA_BK(F, 1); break;         \
    case 2: PWA_BK(F, 2); break;         \
    default: PWA_BK(F, 3); break;        \
  }
  switch (fmt) {
    case PWA_OP_F64: PWA_WIDE(PWA_OP_F64); break;
    case PWA_OP_F32: PWA_WIDE(PWA_OP_F32); break;
    case PWA_OP_BF16: PWA_NARROW(PWA_OP_BF16); break;
    case PWA_OP_F16: PWA_NARROW(PWA_OP_F16); break;
    default: PWA_NARROW(PWA_OP_F16X3); break;
  }
#undef PWA_NARROW
#undef PWA_WIDE
#undef PWA_BK
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(batched_rowsum_kernel, dim3((a.B + 63) / 64, kBatchChunks), dim3(64), 0, st,
                     a.part, row_blocks, a.B, a.part2);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(batched_final_kernel, dim3((a.B + 255) / 256), dim3(256), 0, st, a.part2,
                     a.B, K, C, gram, nd, nm, fmt == PWA_OP_F16X3 ? 1 : 0, nll);
  return hipGetLastError();
}

}  // namespace pwa
