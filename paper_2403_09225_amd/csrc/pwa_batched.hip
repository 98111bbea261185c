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
// the FP64 format; exact integer sums for the sliced FP16 format).  The log
// epilogue is fused: Z never reaches memory.
// Per lane, the 4 rows of an MFMA result tile are combined as the product of
// their mantissas (one logarithm per 4 events) with the exponents summed as
// integers; per-start sums are FP64, reduced across blocks in double-double.
// The Gram matrix comes from FP64 MFMA over the event stream.

#include <math.h>

#include "pwa_batched.h"
#include "pwa_batched_dev.h"

namespace pwa {

// ------------------------------------------------------------------------
// Amplitude rows a_k(x) = beta_k u w for frozen (M, Gamma) from the FP64 event
// stream, written as [Re a_0..Re a_{K-1}, Im a_0..Im a_{K-1}, 0 pad] rows of
// KP operands.
// ------------------------------------------------------------------------
template <int FMT>
__global__ __launch_bounds__(256) void freeze_kernel(const double* __restrict__ planes, int64_t stride,
                                                     int64_t n, const double* __restrict__ tbl,
                                                     const int* __restrict__ itbl, int K, int KP,
                                                     int gen, void* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  auto put = [&](int c, double v) {
    const int64_t o = i * KP + c;
    if constexpr (FMT == PWA_OP_F64) {
      ((double*)out)[o] = v;
    } else if constexpr (FMT == PWA_OP_F32) {
      ((float*)out)[o] = (float)v;
    } else if constexpr (FMT == PWA_OP_BF16) {
      ((__bf16*)out)[o] = (__bf16)(float)v;
    } else {
      ((_Float16*)out)[o] = (_Float16)v;
    }
  };
  for (int k = 0; k < K; ++k) {
    double re, im;
    frozen_amp(planes, stride, i, tbl, itbl, k, gen, re, im);
    put(k, re);
    put(K + k, im);
  }
  for (int c = 2 * K; c < KP; ++c) put(c, 0.0);
}

// Expanded coupling block [[Cr, Ci], [-Ci, Cr]] as KP x 2B operands, column
// b (< B) = real part of start b, column B + b = imaginary part.  The
// couplings enter every event's sum coherently, so a rounding of C biases
// all N_D logarithms alike (the error grows like N_D times the gradient);
// the FP32 format therefore carries C as FP32 hi + lo.
template <int FMT>
__global__ void coupling_kernel(const double* __restrict__ C, int K, int KP, int B, void* out_hi,
                                void* out_lo) {
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
  } else {
    ((_Float16*)out_hi)[idx] = (_Float16)v;
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
__host__ __device__ constexpr int c_parts(int fmt) { return fmt == PWA_OP_F32 ? 2 : 1; }

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
    sC[i] = ((const T*)a.C[0])[g];
    if constexpr (NCP > 1) sC[plane + i] = ((const T*)a.C[1])[g];
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
    op_t ah[NKS];
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) ah[ks] = load_op<FMT>(a.A[0], row * KP + ks * M::KSTEP + kg * M::E);
    // rows held by this lane in the result tile
    bool valid[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      valid[q] = (r0 + (FMT == PWA_OP_F64 ? 4 * q + kg : 4 * kg + q)) < r_end;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      acc_t zr = {0, 0, 0, 0}, zi = {0, 0, 0, 0};
      // Accumulate the low part of C first over the whole inner dimension:
      // it carries a systematic correction of relative size 2^-24; added
      // step by step to an accumulator that already holds the large partial
      // sums it would fall below half an ulp and be dropped every time.
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
  // one LDS buffer: the waves' event rows X[4][16][GP] during the pass, the
  // block's double-double sum of X^T X after it (37 KB: 4 blocks per CU)
  __shared__ double smem[2 * GP * GP];
  double(*X)[16][GP] = (double(*)[16][GP])smem;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t per_block = (n + gridDim.x - 1) / gridDim.x;
  const int64_t e_begin = min(n, (int64_t)blockIdx.x * per_block);
  const int64_t e_end = min(n, e_begin + per_block);
  // X^T X is symmetric: only the tiles (I, J), I <= J, are formed
  constexpr int TI[6] = {0, 0, 0, 1, 1, 2}, TJ[6] = {0, 1, 2, 1, 2, 2};
  d4_t acc[6];
#pragma unroll
  for (int t = 0; t < 6; ++t) acc[t] = (d4_t){0, 0, 0, 0};
  const int col = lane & 15, kg = lane >> 4;
  for (int64_t e0 = e_begin + 16 * wave; e0 < e_end; e0 += 64) {
    // lane l computes features of event e0 + l % 16, resonances kg, kg + 4, ...
    const int64_t ev = e0 + col;
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
    // X[wave] belongs to this wave alone and one wave's LDS operations are
    // carried out in order, so its reads below see its writes above; the
    // fences keep the compiler from moving LDS accesses across this point.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {   // 4 events per MFMA step
      double v[3];
#pragma unroll
      for (int I = 0; I < 3; ++I) v[I] = X[wave][4 * ks + kg][16 * I + col];   // (X^T)[16 I + col][event]
#pragma unroll
      for (int t = 0; t < 6; ++t)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(v[TI[t]], v[TJ[t]], acc[t], 0, 0, 0);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  // block partial of X^T X: the waves add their tiles in order, wave 0
  // first, into a double-double buffer (the tiles below the diagonal are the
  // transposes of those above; every lane owns distinct entries)
  __syncthreads();   // every wave is done with X
  double* rh = smem;
  double* rl = smem + GP * GP;
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int t = 0; t < 6; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = 16 * TI[t] + 4 * q + kg, c = 16 * TJ[t] + col;
#pragma unroll
          for (int m = 0; m < (TI[t] != TJ[t] ? 2 : 1); ++m) {
            const int i = m == 0 ? r * GP + c : c * GP + r;
            if (w == 0) {
              rh[i] = acc[t][q];
              rl[i] = 0.0;
            } else {
              double h = rh[i], l = rl[i];
              dd_add_b(h, l, acc[t][q], 0.0);
              rh[i] = h;
              rl[i] = l;
            }
          }
        }
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < GP * GP; i += blockDim.x) {
    part[((int64_t)blockIdx.x * GP * GP + i) * 2] = rh[i];
    part[((int64_t)blockIdx.x * GP * GP + i) * 2 + 1] = rl[i];
  }
}

// Sum the per-block X^T X, one wave per element: lane j adds blocks j,
// j + 64, ... in order (double-double), then a fixed butterfly over the
// lanes (symmetric in its operands: every lane ends with the same sum).
__global__ __launch_bounds__(64) void gram_sum_kernel(const double* __restrict__ part, int nblocks,
                                                      double* __restrict__ xtx) {
  const int i = blockIdx.x, lane = threadIdx.x;
  double h = 0.0, l = 0.0;
  for (int b = lane; b < nblocks; b += 64)
    dd_add_b(h, l, part[((int64_t)b * GP * GP + i) * 2], part[((int64_t)b * GP * GP + i) * 2 + 1]);
  for (int off = 32; off > 0; off >>= 1) {
    const double oh = __shfl_xor(h, off), ol = __shfl_xor(l, off);
    dd_add_b(h, l, oh, ol);
  }
  if (lane == 0) xtx[i] = h + l;
}

// Gm[k][l] (complex) from X^T X:
//   Re = XtX[k][l] + XtX[K+k][K+l],  Im = XtX[k][K+l] - XtX[K+k][l].
__global__ void gram_final_kernel(const double* __restrict__ xtx, int K, double* __restrict__ gram) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= K * K) return;
  const int k = i / K, l = i % K;
  gram[2 * i] = xtx[k * GP + l] + xtx[(K + k) * GP + K + l];
  gram[2 * i + 1] = xtx[k * GP + K + l] - xtx[(K + k) * GP + l];
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

// Stage 2 and the likelihood, one wave per start: F_b from the chunk
// partials (double-double, a fixed butterfly over the lanes), plus the powers
// of two of the sliced format; G_b = c_b^H Gm c_b with lane k forming
// Re(conj(c_k) (Gm c)_k); NLL_b = -F_b + N_D ln(G_b / N_MC).
__global__ __launch_bounds__(64) void batched_final_kernel(const double* __restrict__ part2, int B,
                                                          int K, const double* __restrict__ C,
                                                          const double* __restrict__ gram,
                                                          double nd, double nm,
                                                          const unsigned long long* esum,
                                                          double* __restrict__ nll) {
  const int b = blockIdx.x, lane = threadIdx.x;
  double h = 0.0, l = 0.0;
  if (lane < kBatchChunks) {
    h = part2[((int64_t)lane * B + b) * 2];
    l = part2[((int64_t)lane * B + b) * 2 + 1];
  }
  double g = 0.0;
  if (lane < K) {
    const double ckr = C[2 * (b * K + lane)], cki = C[2 * (b * K + lane) + 1];
    double sr = 0.0, si = 0.0;   // (Gm c)_k
    for (int j = 0; j < K; ++j) {
      const double gr = gram[2 * (lane * K + j)], gi = gram[2 * (lane * K + j) + 1];
      const double cr = C[2 * (b * K + j)], ci = C[2 * (b * K + j) + 1];
      sr += gr * cr - gi * ci;
      si += gr * ci + gi * cr;
    }
    g = ckr * sr + cki * si;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double oh = __shfl_xor(h, off), ol = __shfl_xor(l, off);
    dd_add_b(h, l, oh, ol);
    g += __shfl_xor(g, off);
  }
  if (lane != 0) return;
  if (esum) {
    // ln |Z|^2 = ln |Z_s|^2 + 2 (E_i + G_b - 18) ln 2 per event: an exact
    // integer m times ln 2 (two parts; m ln2_hi split exactly by an FMA)
    const long long n = (long long)nd;
    const double m = 2.0 * (double)((long long)*esum + ((long long)coupling_exponent(C, K, b) - 18) * n);
    const double p = m * 6.93147180369123816490e-01;
    const double pe = fma(m, 6.93147180369123816490e-01, -p);
    dd_add_b(h, l, p, fma(m, 1.90821492927058770002e-10, pe));
  }
  const double F = h + l;
  double val = -F + nd * log(g / nm);
  if (!(g > 0.0) || !isfinite(val)) val = INFINITY;
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
int batched_a_planes(int fmt) { return fmt == PWA_OP_F16S ? kSlices : 1; }
int batched_c_planes(int fmt) { return fmt == PWA_OP_F16S ? kSlices : c_parts(fmt); }

hipError_t launch_freeze(int fmt, const double* planes, int64_t stride, int64_t n,
                         const double* tbl, const int* itbl, int K, int KP, int gen,
                         void* const* out, unsigned long long* esum, hipStream_t st) {
  if (fmt == PWA_OP_F16S)
    return launch_freeze_slices(planes, stride, n, tbl, itbl, K, KP, gen, (_Float16*)out[0], esum, st);
  if (n <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((n + 255) / 256);
#define PWA_FZ(F) hipLaunchKernelGGL(freeze_kernel<F>, dim3(grid), dim3(256), 0, st, planes, stride, n, tbl, itbl, K, KP, gen, out[0])
  switch (fmt) {
    case PWA_OP_F64: PWA_FZ(PWA_OP_F64); break;
    case PWA_OP_F32: PWA_FZ(PWA_OP_F32); break;
    case PWA_OP_BF16: PWA_FZ(PWA_OP_BF16); break;
    default: PWA_FZ(PWA_OP_F16); break;
  }
#undef PWA_FZ
  return hipGetLastError();
}

hipError_t launch_gram(const double* planes, int64_t stride, int64_t base, int64_t n,
                       const double* tbl, const int* itbl, int K, int gen, int nblocks, double* part,
                       double* xtx, double* gram, hipStream_t st) {
  hipLaunchKernelGGL(gram_kernel, dim3(nblocks), dim3(256), 0, st, planes, stride, base, n, tbl,
                     itbl, K, gen, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gram_sum_kernel, dim3(GP * GP), dim3(64), 0, st, part, nblocks, xtx);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gram_final_kernel, dim3((K * K + 255) / 256), dim3(256), 0, st, xtx, K, gram);
  return hipGetLastError();
}

namespace {
// FP64, FP32, BF16 and FP16 formats: coupling block, then the data term.
hipError_t launch_plain(int fmt, const BatchArgs& a, int row_blocks, const double* C, int K,
                        hipStream_t st) {
  const unsigned cg = (unsigned)((a.KP * 2 * a.B + 255) / 256);
#define PWA_CP(F) hipLaunchKernelGGL(coupling_kernel<F>, dim3(cg), dim3(256), 0, st, C, K, a.KP, a.B, (void*)a.C[0], (void*)a.C[1])
  switch (fmt) {
    case PWA_OP_F64: PWA_CP(PWA_OP_F64); break;
    case PWA_OP_F32: PWA_CP(PWA_OP_F32); break;
    case PWA_OP_BF16: PWA_CP(PWA_OP_BF16); break;
    default: PWA_CP(PWA_OP_F16); break;
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
    default: PWA_NARROW(PWA_OP_F16); break;
  }
#undef PWA_NARROW
#undef PWA_WIDE
#undef PWA_BK
  return hipGetLastError();
}
}  // namespace

hipError_t launch_batched(int fmt, const BatchArgs& a, int row_blocks, const double* C,
                          const double* gram, int K, double nd, double nm, double* nll,
                          hipStream_t st) {
  hipError_t e = fmt == PWA_OP_F16S ? launch_sliced(a, row_blocks, C, K, st)
                                    : launch_plain(fmt, a, row_blocks, C, K, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(batched_rowsum_kernel, dim3((a.B + 63) / 64, kBatchChunks), dim3(64), 0, st,
                     a.part, row_blocks, a.B, a.part2);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(batched_final_kernel, dim3(a.B), dim3(64), 0, st, a.part2,
                     a.B, K, C, gram, nd, nm, fmt == PWA_OP_F16S ? a.esum : nullptr, nll);
  return hipGetLastError();
}

}  // namespace pwa
